"""Pins of the oracle's shell model: the full Eq. structure with its
off-diagonal (i != j) terms, in-plane shear with phi_12 = 1 / (2 (1 + nu))
and mixed bending with gamma_12 = 1, on the cylinder mesh (theta periodic,
simply supported end rings).

* Rest shape: no force (the rest cylinder has X_theta . X_z = 0).
* Bending: for a displacement e_a sin(2 pi m j / n_theta) sin(pi q k / (n_z - 1))
  every second difference is an eigen-operator (eigenvalues -l_theta, -l_z,
  l = 4 sin^2(half the mode's phase step) / ds^2; the sine vanishes on the end
  rings with its curvature, the simply supported condition), so the bending
  force is -EI (l_theta^2 + l_z^2) f with the two coordinate directions only
  and -EI (l_theta + l_z)^2 f, the discrete biharmonic, with the mixed terms.
  Exact up to the rounding of D = X - X0 through the stencil.
* Twisted cylinder X = (R cos(theta + kappa z), R sin(...), z): the continuum
  force of Eq. structure (stretching only) is radial, inward, of size
  R kappa^2 Eh (sqrt(1 + R^2 kappa^2) - 1 + 2 phi_12) -- the z-stretching part
  and the shear part S = R kappa acting on d X_z / d s_theta + d X_theta / dz =
  -2 kappa e_r.  The discrete force converges to it at second order, and the
  shear part alone (shell minus no shell) too.
* The shear part is linear in phi_12: two Poisson ratios give parts in the
  ratio of their phi_12 = 1 / (2 (1 + nu)) exactly.
* Rigid rotation of the shape and the rest shape together rotates the force.
"""
import math

import numpy as np

import lbm_inputs as L


def _oracle(oracle_mod, mesh, k, ei, shell, nu=0.5):
    fl = np.zeros((8, 8, 8), np.uint8)
    o = oracle_mod.Oracle(fl, 0.8)
    o.set_membrane(mesh, k, ei, 1.0, -0.1, -0.5)
    o.set_shell(shell, nu)
    return o


def test_rest_shape_is_force_free_with_the_shell_terms(oracle_mod):
    mesh = L.cylinder_mesh(10.0, 10.0, 6.0, 3.0, 13.0, 0.8)
    o = _oracle(oracle_mod, mesh, 0.05, 1e-3, True, 0.3)
    assert np.abs(o.membrane_force(mesh["X0"])).max() < 1e-15


def test_bending_fourier_mode_is_the_discrete_biharmonic(oracle_mod):
    mesh = L.cylinder_mesh(0.0, 0.0, 7.0, 0.0, 12.0, 0.6)
    nth, nzl = mesh["n_theta"], mesh["n_z"]
    dth, dz = mesh["ds_theta"], mesh["ds_z"]
    ei = 2e-3
    j = np.arange(nth)[None, :]
    k = np.arange(nzl)[:, None]
    interior = np.zeros((nzl, nth), bool)
    interior[1:-1] = True
    for m, q, a in ((3, 2, 0), (5, 1, 1), (1, 3, 2)):
        f = np.sin(2 * math.pi * m * j / nth) * np.sin(math.pi * q * k / (nzl - 1))
        D = np.zeros((nzl, nth, 3))
        D[..., a] = f
        X = mesh["X0"] + D.reshape(-1, 3)
        lt = 4.0 * math.sin(math.pi * m / nth) ** 2 / dth ** 2
        lz = 4.0 * math.sin(math.pi * q / (2 * (nzl - 1))) ** 2 / dz ** 2
        for shell, want in ((False, -ei * (lt * lt + lz * lz)), (True, -ei * (lt + lz) ** 2)):
            F = _oracle(oracle_mod, mesh, 0.0, ei, shell).membrane_force(X).reshape(nzl, nth, 3)
            exp = want * f
            # rounding: D = X - X0 carries eps |X| and the stencil's absolute
            # weights sum to at most (4 / dth^2 + 4 / dz^2)^2
            tol = 4 * np.finfo(float).eps * np.abs(X).max() * ei * (4 / dth ** 2 + 4 / dz ** 2) ** 2
            assert tol < 1e-9 * abs(want)
            assert np.abs(F[interior][:, a] - exp[interior]).max() <= tol, (m, q, shell)
            others = [b for b in range(3) if b != a]
            assert np.abs(F[interior][:, others]).max() <= tol


def _twist_force(oracle_mod, h, R, kappa, Eh, shell, nu):
    mesh = L.cylinder_mesh(0.0, 0.0, R, 0.0, 10.0, h)
    nth, nzl = mesh["n_theta"], mesh["n_z"]
    X0 = mesh["X0"].reshape(nzl, nth, 3)
    th = np.arctan2(X0[..., 1], X0[..., 0])
    z = X0[..., 2]
    phi = th + kappa * z
    X = np.stack([R * np.cos(phi), R * np.sin(phi), z], axis=-1)
    F = _oracle(oracle_mod, mesh, Eh, 0.0, shell, nu).membrane_force(X.reshape(-1, 3)).reshape(nzl, nth, 3)
    er = np.stack([np.cos(phi), np.sin(phi), np.zeros_like(phi)], axis=-1)
    fr = (F * er).sum(-1)[1:-1]          # radial component, interior rings
    return fr, F[1:-1], er[1:-1]


def test_twisted_cylinder_converges_to_the_continuum_force(oracle_mod):
    R, kappa, Eh, nu = 6.0, 0.03, 0.05, 0.3
    phi12 = 1.0 / (2.0 * (1.0 + nu))
    full = -R * kappa ** 2 * Eh * (math.sqrt(1 + (R * kappa) ** 2) - 1 + 2 * phi12)
    shear = -2.0 * Eh * phi12 * R * kappa ** 2
    e_full, e_shear = [], []
    for h in (0.5, 0.25, 0.125):
        f1, F1, er = _twist_force(oracle_mod, h, R, kappa, Eh, True, nu)
        f0, _, _ = _twist_force(oracle_mod, h, R, kappa, Eh, False, nu)
        # helical symmetry: every interior point feels the same radial force
        # (up to the rounding of edge vectors of length ~h between points at
        # radius R, divided twice by h)
        assert np.ptp(f1) <= 16 * np.finfo(float).eps * R * Eh / h ** 2
        e_full.append(abs(f1.mean() - full) / abs(full))
        e_shear.append(abs((f1 - f0).mean() - shear) / abs(shear))
    print({"full": e_full, "shear": e_shear})
    assert e_full[-1] < 2e-3 and e_shear[-1] < 2e-3
    for e in (e_full, e_shear):
        assert 3.5 < e[0] / e[1] < 4.5 and 3.5 < e[1] / e[2] < 4.5, e


def test_shear_part_is_linear_in_phi12(oracle_mod):
    mesh = L.cylinder_mesh(0.0, 0.0, 5.0, 0.0, 8.0, 0.7)
    rng = np.random.default_rng(21)
    X = mesh["X0"] + 0.05 * rng.standard_normal(mesh["X0"].shape)
    F0 = _oracle(oracle_mod, mesh, 0.04, 0.0, False).membrane_force(X)
    parts = {}
    for nu in (0.0, 0.45):          # no bending: the mixed term does not depend on nu
        parts[nu] = _oracle(oracle_mod, mesh, 0.04, 0.0, True, nu).membrane_force(X) - F0
    ratio = (1.0 / (2 * 1.0)) / (1.0 / (2 * 1.45))
    assert np.abs(parts[0.0]).max() > 1e-6
    assert np.abs(parts[0.0] - ratio * parts[0.45]).max() <= 1e-12 * np.abs(parts[0.0]).max()


def test_rigid_rotation_rotates_the_force(oracle_mod):
    mesh = L.cylinder_mesh(0.0, 0.0, 5.0, 0.0, 8.0, 0.7)
    rng = np.random.default_rng(22)
    X = mesh["X0"] + 0.05 * rng.standard_normal(mesh["X0"].shape)
    A = rng.standard_normal((3, 3))
    Q, _ = np.linalg.qr(A)
    rot = dict(mesh, X0=mesh["X0"] @ Q.T)
    F = _oracle(oracle_mod, mesh, 0.04, 1e-3, True, 0.3).membrane_force(X)
    Fr = _oracle(oracle_mod, rot, 0.04, 1e-3, True, 0.3).membrane_force(X @ Q.T)
    assert np.abs(Fr - F @ Q.T).max() <= 1e-12 * np.abs(F).max()
