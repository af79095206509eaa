"""Pins of the oracle's wall-shear-stress diagnostic (the paper's case study:
WSS = mu dv1/dx3, the axial velocity's derivative along the wall normal,
taken through the fluid next to the wall), on the small elastic tube's
cylinder mesh (r = 7) with manufactured velocity fields: every cell set to
the equilibrium at a prescribed velocity, nothing stepped.

* Uniform axial flow U past a wall at rest: trilinear interpolation of a
  constant is exact, so WSS = mu U / d at every point (1e-12).
* The same flow past a wall moving axially at U: WSS = 0 (the wall's own
  velocity is subtracted).
* Poiseuille profile U (1 - r^2/R^2): the fluid at distance d inside the
  wall moves at U (2 R d - d^2)/R^2, so WSS = mu U (2R - d)/R^2 up to the
  trilinear interpolation of r^2, whose error is at most 1/2 (in cell units
  squared) -- a bar of mu U / (2 R^2 d) per point.  An outward normal, a
  wrong distance, viscosity or axial projection all miss it by far.
* Reversed flow reverses the sign.
"""
import numpy as np

import lbm_inputs as L
import oracle


def _setup(vfield, wall_velocity=0.0, d=2.0):
    c = L.small_fsi()
    nz, ny, nx = c["flags"].shape
    o = oracle.from_config(c)
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    V = vfield(xx - (nx - 1) / 2.0, yy - (ny - 1) / 2.0)
    g = np.zeros((nz * ny * nx, 19))
    p0 = c["p_init"]
    fl = (c["flags"] == L.FLUID).ravel()
    for idx in np.flatnonzero(fl):
        g[idx] = oracle.feq(p0, [0.0, 0.0, V.ravel()[idx]])
    o.set_pops(g)
    if wall_velocity:
        o.set_wall_options(0, external=True)
        X = c["mesh"]["X0"].copy()
        Vw = np.zeros_like(X)
        Vw[:, 2] = wall_velocity
        o.set_wall(X, Vw)
    mu = (c["tau"] - 0.5) / 3.0
    return o.wss(d), mu, c


def test_uniform_flow_gives_mu_u_over_d():
    U = 3e-3
    w, mu, _ = _setup(lambda x, y: np.full_like(x, U, dtype=float))
    assert np.allclose(w, mu * U / 2.0, rtol=1e-12, atol=0)


def test_wall_moving_with_the_flow_feels_no_shear():
    U = 3e-3
    w, mu, _ = _setup(lambda x, y: np.full_like(x, U, dtype=float), wall_velocity=U)
    assert np.abs(w).max() <= 1e-12 * mu * U


def test_poiseuille_profile_within_interpolation_bound():
    U, R, d = 4e-3, 7.0, 2.0
    w, mu, _ = _setup(lambda x, y: U * (1.0 - (x * x + y * y) / (R * R)), d=d)
    want = mu * U * (2 * R - d) / (R * R)
    err = np.abs(w - want).max()
    print({"want": want, "max_err_rel": err / want})
    assert err <= mu * U / (2 * R * R * d) * 1.001
    wr, _, _ = _setup(lambda x, y: -U * (1.0 - (x * x + y * y) / (R * R)), d=d)
    assert np.allclose(wr, -w, rtol=1e-12, atol=0)
