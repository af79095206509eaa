"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-types the oracle's formulas: they check moments and
isotropy identities of the lattice, closed forms of the 0D recursions, special
values of the smoothing function, moment conditions of the delta kernel, the
paper's manufactured-solution filament and exact discrete force balances of
the membrane.
"""
import math
import os

import numpy as np
import pytest

import lbm_inputs as L

HERE = os.path.dirname(os.path.abspath(__file__))


# ----------------------------------------------------------------------------
# lattice, equilibrium, forcing (Eqs. feq, f, rho, v)
# ----------------------------------------------------------------------------

def test_lattice_isotropy(oracle_mod):
    e, w = oracle_mod.lattice()
    e = e.astype(float)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.abs((w[:, None] * e).sum(0)).max() < 1e-15
    M2 = np.einsum("i,ia,ib->ab", w, e, e)
    assert np.abs(M2 - np.eye(3) / 3.0).max() < 1e-15
    M3 = np.einsum("i,ia,ib,ic->abc", w, e, e, e)
    assert np.abs(M3).max() < 1e-15
    M4 = np.einsum("i,ia,ib,ic,id->abcd", w, e, e, e, e)
    d = np.eye(3)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) +
           np.einsum("ad,bc->abcd", d, d)) / 9.0
    assert np.abs(M4 - iso).max() < 1e-15
    # every velocity has its opposite
    for i in range(19):
        assert any((e[k] == -e[i]).all() for k in range(19))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_equilibrium_moments(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    p = 1e-3 * rng.standard_normal()
    v = 0.05 * rng.standard_normal(3)
    e, w = oracle_mod.lattice()
    e = e.astype(float)
    g = oracle_mod.feq(p, v)
    delta = 3.0 * p
    assert abs(g.sum() - delta) < 1e-16                      # sum f = P / c_s^2
    assert np.abs(e.T @ g - v).max() < 1e-16                 # sum e f = rho0 v
    Pi = np.einsum("i,ia,ib->ab", g, e, e)
    # incompressible model: Pi = P I + rho0 v v  (shifted: -c_s^2 I)
    assert np.abs(Pi - (p * np.eye(3) + np.outer(v, v))).max() < 1e-15


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_forcing_moments(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    tau = 0.5 + rng.random()
    v = 0.05 * rng.standard_normal(3)
    b = 1e-4 * rng.standard_normal(3)
    e, _ = oracle_mod.lattice()
    e = e.astype(float)
    F = oracle_mod.forcing(tau, v, b)
    c = 1.0 - 1.0 / (2.0 * tau)
    assert abs(F.sum()) < 1e-19
    assert np.abs(e.T @ F - c * b).max() < 1e-19
    S = np.einsum("i,ia,ib->ab", F, e, e)
    assert np.abs(S - c * (np.outer(v, b) + np.outer(b, v))).max() < 1e-19


def test_rest_state_is_a_fixed_point_bitwise(oracle_mod):
    fl = L.tube_flags(12, 12, 16, 5.5, 5.5, 4.0)
    o = oracle_mod.Oracle(fl, 0.7)
    o.step(50)
    assert np.all(o.get_pops() == 0.0)


# ----------------------------------------------------------------------------
# smoothing-to-zero (Eq. SmoothFunction) and the LV elastance curve
# ----------------------------------------------------------------------------

def test_smoothing_special_values(oracle_mod):
    rows = np.loadtxt(os.path.join(HERE, "golden", "smoothing_S.txt"))
    for u, s in rows:
        assert abs(oracle_mod.smooth_S(10.0 + 4.0 * u, 10.0, 4.0) - s) < 1e-10


def test_smoothing_properties(oracle_mod):
    S = lambda t: oracle_mod.smooth_S(t, 0.5, 0.075)
    assert S(0.4) == 1.0 and S(0.5) == 1.0 and S(0.575) == 0.0 and S(0.7) == 0.0
    ts = np.linspace(0.5, 0.575, 2001)
    vals = np.array([S(t) for t in ts])
    assert np.all(np.diff(vals) <= 0.0)
    # C-infinity at both ends: one-sided slopes vanish faster than any power
    h = 1e-3 * 0.075
    assert abs(S(0.5 + h) - 1.0) / h < 1e-6
    assert abs(S(0.575 - h)) / h < 1e-6
    # the paper's worked example: t0 = T_d = 0.5 s, dt = 0.005 s, N_S = 15
    samples = [S(0.5 + k * 0.005) for k in range(16)]
    assert samples[0] == 1.0 and samples[-1] == 0.0 and all(a >= b for a, b in zip(samples, samples[1:]))


def test_elastance_curve(oracle_mod):
    sc = L.scales()
    par = L.lv_params(2.0, 0.06, 75.0, 8.0, 0.075, sc)
    Emax, Emin, Tc, Tmax = par[0], par[1], par[2], par[3]
    E0, dE0 = oracle_mod.elastance(par, 0.0)
    assert E0 == Emin and dE0 == 0.0
    ts = np.linspace(0.0, Tc, 20001)
    Es = np.array([oracle_mod.elastance(par, t)[0] for t in ts])
    k = int(np.argmax(Es))
    # normalised double-Hill: peak at ~T_max, peak value E_max to the rounding of k
    assert abs(ts[k] / Tmax - 1.0) < 0.02
    assert abs(Es[k] / Emax - 1.0) < 0.01
    assert abs(Es[-1] - Emin) / Emin < 1e-3
    # derivative against central differences
    for t in (0.1 * Tmax, 0.5 * Tmax, 0.9 * Tmax, 1.1 * Tmax, 1.3 * Tmax):
        h = 1e-4 * Tmax
        fd = (oracle_mod.elastance(par, t + h)[0] - oracle_mod.elastance(par, t - h)[0]) / (2 * h)
        assert abs(oracle_mod.elastance(par, t)[1] - fd) <= 1e-6 * abs(fd) + 1e-12 * Emax / Tmax


# ----------------------------------------------------------------------------
# 0D models: exact discrete recursions (Eqs. rightbc, rightQ, LVE)
# ----------------------------------------------------------------------------

def test_windkessel_flux_driven_recursion(oracle_mod):
    Z, C, R, Q, P0 = 0.05, 50.0, 1.0, 3e-4, 1e-4
    m = oracle_mod.ZeroD(1, L.BC_WINDKESSEL3, [Z, C, R, 0.0], [P0])
    lam = 1.0 - 1.0 / (R * C)
    for n in range(300):
        r = m.update(n, Q, 0.0)
        Pw = Q * R + (P0 - Q * R) * lam ** (n + 1)
        assert abs(r["Pw"] - Pw) < 1e-15
        assert abs(r["pstar"] - (Pw + Z * Q)) < 1e-15 and r["vmode"] == 0
    # steady state: P = Q (Rp + Rd)
    for n in range(300, 20000):
        r = m.update(n, Q, 0.0)
    assert abs(r["pstar"] - Q * (Z + R)) < 1e-15


def test_windkessel_pressure_driven_recursion(oracle_mod):
    Z, C, R, P = 0.05, 50.0, 1.0, 3e-4
    m = oracle_mod.ZeroD(1, L.BC_WINDKESSEL3, [Z, C, R, 1.0], [0.0])
    lam = 1.0 - (R + Z) / (C * R * Z)
    Pinf = P * R / (R + Z)
    for n in range(200):
        r = m.update(n, 0.0, P)
        Pw = Pinf + (0.0 - Pinf) * lam ** (n + 1)
        assert abs(r["Pw"] - Pw) < 1e-16
        assert r["vmode"] == 1
        assert abs(r["pstar"]) == 0.0
    # steady outflow Q = P / (Rp + Rd): the correction with zero measured flux
    assert abs(r["Pw"] - Pinf) < 1e-16


def test_lv_isovolumic_first_order(oracle_mod):
    """Valve closed (Q = 0): C_v P_v is conserved, P_v(t) = P_v(0) E(t)/E(0);
    forward Euler converges to it at first order."""
    errs = []
    for m in (1, 2, 4):
        sc = L.scales(sigma_t=2000.0 * m)
        par = L.lv_params(2.0, 0.06, 75.0, 8.0, 0.075, sc)
        z = oracle_mod.ZeroD(0, L.BC_LV_ELASTANCE, par)
        P0 = par[4]
        E0 = oracle_mod.elastance(par, 0.0)[0]
        nsteps = int(0.25 * par[2])
        for n in range(nsteps):
            r = z.update(n, 0.0, 1e9)          # aortic pressure huge: stays closed
            assert r["open"] == 0 and r["vmode"] == 1 and r["S"] == 0.0
        Eend = oracle_mod.elastance(par, float(nsteps))[0]
        errs.append(abs(r["Pv"] - P0 * Eend / E0) / (P0 * Eend / E0))
    assert errs[0] > errs[1] > errs[2]
    assert 1.7 < errs[0] / errs[1] < 2.3 and 1.7 < errs[1] / errs[2] < 2.3


def test_lv_valve_switching(oracle_mod):
    sc = L.scales(sigma_t=1000.0)
    par = L.lv_params(2.0, 0.06, 75.0, 8.0, 0.075, sc)     # Tc = 800 steps, N_S = 75
    z = oracle_mod.ZeroD(0, L.BC_LV_ELASTANCE, par)
    r = z.update(0, 0.0, 1.0)                               # P_v < P_bar: stays closed
    assert r["open"] == 0 and r["vmode"] == 1
    r = z.update(1, 0.0, -1.0)                              # P_v > P_bar: opens
    assert r["open"] == 1 and r["vmode"] == 0 and r["pstar"] == r["Pv"]
    r = z.update(2, -1e-9, -1.0)        # residual backflow before any inflow: stays open
    assert r["open"] == 1 and r["snap"] == 0
    z = oracle_mod.ZeroD(0, L.BC_LV_ELASTANCE, par)
    z.update(0, 0.0, 1.0)
    r = z.update(1, 0.0, -1.0)
    Pv = r["Pv"]
    E, dE = oracle_mod.elastance(par, 2.0)
    r = z.update(2, 1e-3, -1.0)                             # ejecting: P_v follows Eq. LVE
    assert abs(r["Pv"] - (Pv + dE / E * Pv - E * 1e-3)) < 1e-18
    r = z.update(3, -1e-9, -1.0)                            # Q < 0: valve closes at T_d = 3
    assert r["open"] == 0 and r["snap"] == 1 and r["Td"] == 3 and r["vmode"] == 1
    assert abs(r["S"] - oracle_mod.smooth_S(4.0, 3.0, 75.0)) == 0.0
    for n in range(4, 100):
        r = z.update(n, 5e-3, -1.0)                         # no re-opening in this beat
        assert r["open"] == 0 and r["snap"] == 0
    assert r["S"] == 0.0
    r = z.update(800, 0.0, 1.0)                             # next beat: reset to P_ed
    assert r["Pv"] == par[4]                                # dE/dt = 0 at the beat start
    assert r["Td"] == -1 and r["open"] == 0


# ----------------------------------------------------------------------------
# delta kernel and immersed-boundary transfer (Eqs. interpolation, EulForce)
# ----------------------------------------------------------------------------

def test_peskin_kernel_moments(oracle_mod):
    rng = np.random.default_rng(5)
    for r in rng.random(50) * 4.0 - 2.0:
        js = np.arange(-4, 5)
        ph = np.array([oracle_mod.phi4(r - j) for j in js])
        assert abs(ph.sum() - 1.0) < 1e-15
        assert abs(((r - js) * ph).sum()) < 1e-15
        assert abs((ph * ph).sum() - 3.0 / 8.0) < 1e-15
    assert oracle_mod.phi4(0.0) == 0.5 and oracle_mod.phi4(2.0) == 0.0 and oracle_mod.phi4(2.5) == 0.0


def test_cosine_kernel_values_and_moments(oracle_mod):
    """The variant kernel (1 + cos(pi r / 2)) / 4: closed values, even,
    support |r| < 2, partition of unity (four cosines a quarter period
    apart sum to zero) and sum of squares 3/8 (cos^2 + sin^2 in pairs)."""
    phi = oracle_mod.phicos
    assert phi(0.0) == 0.5 and phi(2.0) == 0.0 and phi(-2.0) == 0.0 and phi(3.1) == 0.0
    assert abs(phi(1.0) - 0.25) < 1e-16 and abs(phi(0.5) - (2 + math.sqrt(2)) / 8) < 1e-16
    rng = np.random.default_rng(6)
    for r in rng.random(50) * 4.0 - 2.0:
        js = np.arange(-4, 5)
        ph = np.array([phi(r - j) for j in js])
        assert phi(r) == phi(-r)
        assert abs(ph.sum() - 1.0) < 1e-15
        assert abs((ph * ph).sum() - 3.0 / 8.0) < 1e-15
    xs = np.linspace(0, 2, 41)
    assert np.all(np.diff([phi(x) for x in xs]) < 0)


def _box_oracle(oracle_mod, n=16):
    fl = np.zeros((n, n, n), np.uint8)
    return oracle_mod.Oracle(fl, 0.8), n


def test_ib_interpolates_linear_fields_exactly(oracle_mod):
    o, n = _box_oracle(oracle_mod)
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    A = np.array([0.1, -0.2, 0.3])
    B = np.array([[0.01, 0.02, -0.03], [0.005, -0.01, 0.02], [-0.02, 0.01, 0.015]])
    pos = np.stack([x, y, z], -1).astype(float)
    u = A + pos @ B.T
    X = L.random_points(40, [3, 3, 3], [12, 12, 12], seed=3)
    V = o.ib_interp(X, u.reshape(-1, 3))
    assert np.abs(V - (A + X @ B.T)).max() < 1e-14


def test_ib_spread_adjoint_and_conservative(oracle_mod):
    o, n = _box_oracle(oracle_mod)
    rng = np.random.default_rng(4)
    X = L.random_points(60, [3, 3, 3], [12, 12, 12], seed=7)
    F = rng.standard_normal((60, 3))
    u = rng.standard_normal((n ** 3, 3))
    area = 0.3
    b = o.ib_spread(X, F, area)
    V = o.ib_interp(X, u)
    assert abs((b * u).sum() - area * (F * V).sum()) < 1e-12
    assert np.abs(b.sum(0) - area * F.sum(0)).max() < 1e-13


def test_ib_transfer_with_the_cosine_kernel(oracle_mod):
    """Kernel 1 in the wall exchange: a unit spike interpolates to the
    product of the kernel's values, constants interpolate exactly, and the
    spreading stays the adjoint of the interpolation and conserves force;
    a linear field is no longer reproduced (no first-moment condition),
    which tells the variant apart from the default kernel."""
    o, n = _box_oracle(oracle_mod)
    o.set_wall_options(kernel=1)
    X = L.random_points(30, [3, 3, 3], [12, 12, 12], seed=8)
    node = np.floor(X[0]).astype(int)
    u = np.zeros((n, n, n, 3))
    u[node[2], node[1], node[0], 0] = 1.0
    V = o.ib_interp(X[:1], u.reshape(-1, 3))
    d = node - X[0]
    assert abs(V[0, 0] - oracle_mod.phicos(d[0]) * oracle_mod.phicos(d[1]) * oracle_mod.phicos(d[2])) < 1e-15
    c = np.array([0.3, -0.1, 0.2])
    assert np.abs(o.ib_interp(X, np.tile(c, (n ** 3, 1))) - c).max() < 1e-14
    rng = np.random.default_rng(9)
    F = rng.standard_normal((30, 3))
    u = rng.standard_normal((n ** 3, 3))
    b = o.ib_spread(X, F, 0.4)
    assert abs((b * u).sum() - 0.4 * (F * o.ib_interp(X, u)).sum()) < 1e-12
    assert np.abs(b.sum(0) - 0.4 * F.sum(0)).max() < 1e-13
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    lin = np.stack([x, y, z], -1).astype(float).reshape(-1, 3) * 0.01
    assert np.abs(o.ib_interp(X, lin) - X * 0.01).max() > 1e-5


def test_external_solid_moves_ballistically_and_drags_the_fluid(oracle_mod):
    """External-solid mode: between updates the points keep their velocity
    (D after k steps = D + k V, with no membrane forces), and a wall
    translating along +z pushes the fluid along +z (force on the fluid
    parallel to the wall's velocity for alpha, beta < 0)."""
    c = L.small_fsi()
    c["wall_mode"] = 1
    o = oracle_mod.from_config(c)
    X0 = c["mesh"]["X0"]
    V = np.zeros_like(X0)
    V[:, 2] = 2e-3
    X = X0 + 0.1 * V
    o.set_wall(X, V)
    k = 25
    o.step(k)
    Dn, Dp = o.displacement()
    assert np.abs(Dn - (X - X0 + k * V)).max() < 1e-13
    assert np.abs((Dn - Dp) - V).max() < 1e-13
    p, u = o.fields()
    fl = c["flags"] == L.FLUID
    assert u[fl][:, 2].sum() > 0
    assert o.lagrangian()["F"][:, 2].mean() > 0


# ----------------------------------------------------------------------------
# wall operators (Eqs. tension, bending; manufactured solution Eq. MMSsolid)
# ----------------------------------------------------------------------------

def _mms_forcing():
    sp = pytest.importorskip("sympy")
    s, t = sp.symbols("s t", real=True)
    A, Eh, EI, rhoh = sp.symbols("A Eh EI rhoh", positive=True)
    X = sp.Matrix([s, A * sp.cos(sp.pi * s) * sp.sin(sp.pi * t)])
    Xs = X.diff(s)
    T = Eh * (sp.sqrt((Xs.T * Xs)[0]) - 1)
    rhs = (T * Xs).diff(s) - EI * X.diff(s, 4)
    f = rhoh * X.diff(t, 2) - rhs
    return sp.lambdify((s, t, A, Eh, EI, rhoh), list(f), "numpy"), \
        sp.lambdify((s, t, A), list(X), "numpy")


def test_filament_manufactured_solution_second_order(oracle_mod):
    """The paper's MMS filament (Sec. 3.1.2): X = (s, A cos(pi s) sin(pi t)),
    A = 0.01 m, E = 0.5 MPa, h = 1 mm, L = 1 m, dt = 1e-5 s; max error over
    space and time decreases at second order under refinement."""
    f, Xex = _mms_forcing()
    A, E, h = 0.01, 0.5e6, 1e-3
    Eh, EI, rhoh = E * h, E * h ** 3 / 12.0, 1000.0 * h      # rho_s: 1000 kg/m^3
    dt, nsteps = 1e-5, 20000
    errs = []
    for N in (25, 50, 100):
        ds = 1.0 / N
        s = ds * np.arange(-2, N + 3)                           # two given points per end
        inner = slice(2, N + 1)                                 # s = ds .. 1 - ds
        def exact(tt):
            X = np.zeros((s.size, 3))
            ex = Xex(s, tt, A)
            X[:, 0] = ex[0]
            X[:, 1] = ex[1]
            return X
        Xm, X = exact(-dt), exact(0.0)
        err = 0.0
        for n in range(nsteps):
            tn = n * dt
            F = oracle_mod.filament_force(X, ds, Eh, EI)
            fm = f(s, tn, A, Eh, EI, rhoh)
            acc = (F[:, :2] + np.stack([np.broadcast_to(fm[0], s.shape), fm[1]], -1)) / rhoh
            Xn = exact(tn + dt)
            Xn[inner, :2] = 2 * X[inner, :2] - Xm[inner, :2] + dt * dt * acc[inner]
            Xm, X = X, Xn
            if n % 50 == 0 or n == nsteps - 1:
                err = max(err, np.abs(X[inner] - exact(tn + dt)[inner]).max())
        errs.append(err)
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.3 < r1 < 4.8 and 3.3 < r2 < 4.8, errs


def _ring_oracle(oracle_mod, r=6.0, h=0.8, k=0.05, ei=1e-3):
    mesh = L.cylinder_mesh(10.0, 10.0, r, 3.0, 13.0, h)
    fl = np.zeros((18, 21, 21), np.uint8)
    o = oracle_mod.Oracle(fl, 0.8)
    o.set_membrane(mesh, k, ei, 1.0, -0.1, -0.5)
    return o, mesh


def test_membrane_rest_shape_is_force_free(oracle_mod):
    o, mesh = _ring_oracle(oracle_mod)
    assert np.abs(o.membrane_force(mesh["X0"])).max() < 1e-15


def test_membrane_uniform_inflation_closed_form(oracle_mod):
    """X = X0 + eps (X0 - axis): every chord grows by (1+eps), so the hoop
    tension is k eps and the net tension force is k eps (1+eps) / R inward;
    bending acts on eps (X0 - axis), an eigenvector of the discrete
    second difference around the ring (eigenvalue lam)."""
    r, k, ei = 6.0, 0.05, 1e-3
    o, mesh = _ring_oracle(oracle_mod, r=r, k=k, ei=ei)
    eps = 0.02
    X0 = mesh["X0"]
    rad = X0.copy(); rad[:, 2] = 0.0; rad[:, :2] -= 10.0
    X = X0 + eps * rad
    F = o.membrane_force(X)
    nth, ds = mesh["n_theta"], mesh["ds_theta"]
    lam = -2.0 * (1.0 - math.cos(2.0 * math.pi / nth)) / ds ** 2
    expect = (-k * eps * (1 + eps) / r - ei * eps * lam * lam * r) * rad / r
    assert np.abs(F - expect).max() < 1e-14


def test_membrane_matches_brute(oracle_mod):
    from oracle import brute
    o, mesh = _ring_oracle(oracle_mod)
    rng = np.random.default_rng(9)
    X = mesh["X0"] + 0.05 * rng.standard_normal(mesh["X0"].shape)
    b = brute.Brute(np.zeros((18, 21, 21), np.uint8), 0.8)
    b.set_membrane(mesh, 0.05, 1e-3, 1.0, -0.1, -0.5)
    assert np.abs(o.membrane_force(X) - b.wall_force(X)).max() < 1e-13
