"""Pins of the axisymmetric D2Q9 oracle (Eqs. Afi, AH1: the planar model with
the mass source -w_i u_r / r and the axisymmetric terms as a body force).

* Hagen-Poiseuille: a periodic pipe driven by a uniform axial force G tends
  to u_x = G (R^2 - r^2) / (4 nu) at second order in 1/R (the bounce-back
  wall's slip), with u_r = 0 and a uniform pressure to rounding.  The planar
  model without the axisymmetric terms would give G (R^2 - r^2) / (2 nu),
  twice as fast.
* Womersley: a periodic pipe under G cos(omega t) against the Bessel-function
  solution at Wo = 4; second-order convergence under diffusive scaling.
* Mass conservation in the axisymmetric sense: steady flow through a pipe
  with a stenosis between constant pressures carries the same ring-weighted
  flux sum 2 pi r u_x through every cross-section, while the planar flux sum
  u_x changes by tens of percent where the lumen narrows (the mass source
  is what makes the difference).
* Steady Windkessel at the outlet: Pw = Rd Q and P* = Q (Rp + Rd).
* Axisymmetric Stokes mode with u_r != 0: exact decay rate and pressure.
"""
import math

import numpy as np
import pytest
from scipy import special

import lbm_inputs as L
import oracle


def _poiseuille(R, tau, G=1e-6, steps=None):
    nu = (tau - 0.5) / 3.0
    o = oracle.Axi(L.axi_pipe(R, 3, periodic=True), tau, periodic_x=True)
    o.set_body_force(G)
    o.step(steps or int(40 * R * R / (nu * 5.78)) + 200)
    p, ux, ur = o.fields()
    r = np.arange(R) + 0.5
    exact = G * (R * R - r * r) / (4 * nu)
    return ux[:, 1], ur, p, exact


def test_hagen_poiseuille_second_order():
    errs = []
    for R in (4, 8, 16):
        ux, ur, p, exact = _poiseuille(R, 0.8, steps=int(12 * R * R / 0.1) + 200)
        errs.append(np.abs(ux - exact).max() / exact.max())
        assert np.abs(ur).max() < 1e-12 * exact.max()
        assert np.ptp(p) < 1e-12
    print(errs)
    assert errs[-1] < 5e-3
    assert 3.3 < errs[0] / errs[1] < 4.7 and 3.3 < errs[1] / errs[2] < 4.7


def _womersley(R, Wo=4.0, tau=0.8, periods=6, G0=1e-6):
    nu = (tau - 0.5) / 3.0
    omega = Wo * Wo * nu / (R * R)
    o = oracle.Axi(L.axi_pipe(R, 3, periodic=True), tau, periodic_x=True)
    o.set_body_force(G0, omega)
    T = 2 * math.pi / omega
    o.step(int(round(periods * T)) - 8)
    r = np.arange(R) + 0.5
    alpha = (1j ** 1.5) * Wo
    err, scale = 0.0, 0.0
    for k in range(8):
        o.step(int(round(T / 8)) if k else 8)
        n = o.L.axo_get_waveforms(o.h, None, 0)
        _, ux, _ = o.fields()
        exact = np.real(G0 / (1j * omega) * (1 - special.jv(0, alpha * r / R) / special.jv(0, alpha))
                        * np.exp(1j * omega * n))
        err = max(err, np.abs(ux[:, 1] - exact).max())
        scale = max(scale, np.abs(exact).max())
    return err / scale


def test_womersley_second_order():
    errs = [_womersley(R) for R in (6, 12, 24)]
    print(errs)
    assert errs[-1] < 5e-3
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0


def _stenosis_fluxes(R):
    nx = 8 * R
    f = L.axi_pipe(R, nx, stenosis=(int(3.25 * R), int(4.75 * R), (5 * R) // 8))
    o = oracle.Axi(f, 0.8)
    o.set_bc(0, L.BC_PRESSURE_CONST, [2e-5 * 8 / R])
    o.set_bc(1, L.BC_PRESSURE_CONST, [0.0])
    o.step(int(60 * R * R / 0.1 / 5.78 * 8 / 8) + 2000)
    _, ux, _ = o.fields()
    fluid = f == L.FLUID
    r = (np.arange(R) + 0.5)[:, None]
    ring = (2 * np.pi * r * ux * fluid).sum(axis=0)[1:-1]
    planar = (ux * fluid).sum(axis=0)[1:-1]
    return np.ptp(ring) / ring.mean(), np.ptp(planar) / planar.mean()


def test_ring_weighted_flux_is_conserved_through_a_stenosis():
    (r8, p8), (r16, p16) = _stenosis_fluxes(8), _stenosis_fluxes(16)
    print({"ring": (r8, r16), "planar": (p8, p16)})
    assert r16 < 3e-3 and 3.0 < r8 / r16 < 5.0      # the ring flux's variation is discretisation error
    assert p8 > 0.2 and p16 > 0.2                    # the planar flux changes where the lumen narrows


def test_steady_windkessel_outlet():
    R, nx = 6, 40
    o = oracle.Axi(L.axi_pipe(R, nx), 0.8)
    Rp, C, Rd = 0.002, 2000.0, 0.5      # Rp < c_s / A, C > A / c_s: the flux-driven coupling is stable
    o.set_bc(0, L.BC_PRESSURE_CONST, [1e-4])
    o.set_bc(1, L.BC_WINDKESSEL3, [Rp, C, Rd, 0.0], [0.0])
    o.step(30000)
    w = o.waveforms()
    Q, Pw, Pst = w[-1, 3], w[-1, 10], w[-1, 8]
    print({"Q": Q, "Pw": Pw, "P*": Pst})
    assert Q > 0
    assert abs(Pw - Rd * Q) <= 1e-6 * abs(Pw)
    assert abs(Pst - Q * (Rp + Rd)) <= 1e-6 * abs(Pst)
    assert abs(w[-1, 1] - Q) <= 1e-3 * Q            # inflow = outflow at steady state


# D2Q9 in the oracle's order, for building initial states
_E = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]], float)
_W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def _stokes_mode(R, kR=4.0, tau=0.8, nsamp=120):
    """Axisymmetric Stokes mode of a pipe periodic along x with wavenumber k:
    stream function f(r) sin(kx), f = A r I1(kr) + B r J1(beta r), no slip at
    r = R (f(R) = f'(R) = 0 gives I1(kR) beta J0(beta R) = k I0(kR) J1(beta R)),
    decaying at s = -nu (beta^2 + k^2); its potential part carries the
    pressure s A I0(kr) cos(kx).  The lattice run starts from the mode's
    velocity and pressure at equilibrium; the amplitude of u_r (projection on
    the mode's shape) is sampled over 0.2-1.5 decay times.  Returns the
    decay-rate error and the spread of amplitude / exp(s t), which measures
    the sound the start leaves behind: it is small only if the lattice's
    pressure of the mode is the exact one."""
    from scipy import optimize
    nu = (tau - 0.5) / 3.0
    nx = int(round(2 * math.pi * R / kR))
    k = 2 * math.pi / nx
    g = lambda b: special.iv(1, k * R) * b * special.jv(0, b * R) - k * special.iv(0, k * R) * special.jv(1, b * R)
    bs = np.linspace(0.5 / R, 8.0 / R, 4000)
    v = g(bs)
    i = np.flatnonzero(np.sign(v[:-1]) != np.sign(v[1:]))[0]
    beta = optimize.brentq(g, bs[i], bs[i + 1])
    s = -nu * (beta ** 2 + k ** 2)
    A = 1e-4
    B = -A * special.iv(1, k * R) / special.jv(1, beta * R)
    r = (np.arange(R) + 0.5)[:, None]
    x = np.arange(nx)[None, :]
    ux = (A * k * special.iv(0, k * r) + B * beta * special.jv(0, beta * r)) * np.sin(k * x)
    ur = -k * (A * special.iv(1, k * r) + B * special.jv(1, beta * r)) * np.cos(k * x)
    p = s * A * special.iv(0, k * r) * np.cos(k * x)
    eu = ux.reshape(-1, 1) * _E[:, 0] + ur.reshape(-1, 1) * _E[:, 1]
    # the lattice holds D = 3 p + u_r / (2 r): its pressure reading subtracts u_r / (6 r)
    D0 = 3 * p + ur / (2 * r)
    geq = _W * (D0.reshape(-1, 1) + 3 * eu + 4.5 * eu ** 2 - 1.5 * (ux ** 2 + ur ** 2).reshape(-1, 1))
    o = oracle.Axi(L.axi_pipe(R, nx, periodic=True), tau, periodic_x=True)
    o.set_pops(geq)
    ts = np.linspace(0.2 / -s, 1.5 / -s, nsamp).astype(int)
    t, amps = 0, []
    for tt in ts:
        o.step(tt - t)
        t = tt
        amps.append(float((o.fields()[2] * ur * r).sum() / (ur * ur * r).sum()))
    amps = np.array(amps)
    s_lb = np.polyfit(ts, np.log(amps), 1)[0]
    ratio = amps / np.exp(s * ts)
    return abs(s_lb - s) / abs(s), np.ptp(ratio) / ratio.mean()


def test_radial_stokes_mode():
    """The pin with u_r != 0 in the momentum equation: an axisymmetric Stokes
    mode decays at the exact rate (the radial terms -u_r^2 / r,
    (2 nu / r) d_r u_r - 2 nu u_r / r^2 and the mass source), and it carries
    its exact pressure (the start from the exact pressure, held as
    D = 3 p + u_r / (2 r), leaves sound that falls at second order; read
    without the u_r / (6 r) term it falls at first order only)."""
    res = [_stokes_mode(R) for R in (8, 16, 32)]
    rate, spread = [a for a, _ in res], [b for _, b in res]
    print({"rate": rate, "spread": spread})
    assert rate[1] < 5e-3 and rate[2] < 1e-3
    assert spread[0] / spread[1] > 3.0 and spread[1] / spread[2] > 3.0
