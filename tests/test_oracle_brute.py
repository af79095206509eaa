"""The C oracle against the independent numpy brute force on tiny lattices.

Random geometry (solid cells, inlet / outlet / exterior ghost planes), random
populations, every 0D model kind and the immersed membrane; agreement to FP64
rounding.  A wrong weight, sign, index or dropped term in either
implementation fails here.
"""
import numpy as np
import pytest

import lbm_inputs as L
from oracle import brute


def _pair(oracle_mod, flags, tau, seed, bcs, membrane=None, amp=1e-3):
    g = L.random_populations(flags.size, seed, amp=amp)
    o = oracle_mod.Oracle(flags, tau)
    b = brute.Brute(flags, tau)
    o.set_pops(g)
    b.set_pops(g)
    for k, (kind, par, st) in enumerate(bcs):
        o.set_bc(k, kind, par, st)
        b.bc[k] = brute.Boundary(k, kind, par, st)
    if membrane is not None:
        o.set_membrane(*membrane)
        b.set_membrane(*membrane)
    return o, b


# The brute force works on unshifted f ~ w_i ~ 1/3, so its rounding floor is
# ~1e-16 absolute per step; with populations of amplitude 1e-3 any real
# discrepancy (a term, a sign, an index) is >= 1e-8.
ATOL = 1e-14


def _compare(o, b, steps, atol=ATOL):
    for _ in range(steps):
        o.step(1)
        b.step()
        go, gb = o.get_pops(), b.pops()
        assert np.abs(go - gb).max() <= atol
    wo = o.waveforms()[:, :5]
    wb = np.array(b.records)
    assert np.abs(wo - wb).max() <= atol * 100


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_pressure_and_windkessel(oracle_mod, seed):
    fl = L.random_flags(7, 6, 9, seed=seed)
    bcs = [(L.BC_PRESSURE_CONST, [2e-4], ()),
           (L.BC_WINDKESSEL3, [0.01, 30.0, 0.5, 0.0], [1e-4]),
           (L.BC_PRESSURE_CONST, [-1e-4], ())]
    o, b = _pair(oracle_mod, fl, 0.55 + 0.1 * seed, seed + 10, bcs)
    _compare(o, b, 6)


@pytest.mark.parametrize("seed", [4, 5])
def test_velocity_type_couplings(oracle_mod, seed):
    fl = L.random_flags(8, 7, 8, seed=seed)
    bcs = [(L.BC_VELOCITY_CONST, [3e-3], ()),
           (L.BC_WINDKESSEL3, [0.05, 50.0, 1.0, 1.0], [2e-4]),
           (L.BC_VELOCITY_CONST, [-1e-3], ())]
    o, b = _pair(oracle_mod, fl, 0.9, seed + 20, bcs)
    _compare(o, b, 6)


def test_lv_valve_cycle(oracle_mod):
    """LV inlet through opening, ejection, closure (snapshot + smoothing)."""
    fl = L.tube_flags(9, 9, 10, 4.0, 4.0, 3.2)
    sc = L.scales(sigma_t=400.0, sigma_V=40.0, sigma_P=2.5e-5)
    par = L.lv_params(2.0, 0.06, 75.0, 8.0, 0.01, sc)            # Tc 320 steps, N_S 4
    bcs = [(L.BC_LV_ELASTANCE, par, ()),
           (L.BC_WINDKESSEL3, L.wk_params(0.05, 1.5, 1.0, sc), [80 * 2.5e-5]),
           (L.BC_PRESSURE_CONST, [0.0], ())]
    o, b = _pair(oracle_mod, fl, 0.8, 31, bcs, amp=0.0)
    for _ in range(150):
        o.step(1)
        b.step()
    w = o.waveforms()
    assert w[:, 11].max() == 1.0 and w[-1, 11] == 0.0     # valve opened, then closed
    go, gb = o.get_pops(), b.pops()
    assert np.abs(go - gb).max() <= ATOL
    assert np.abs(w[:, :5] - np.array(b.records)).max() <= ATOL * 100


def test_immersed_membrane(oracle_mod):
    fl = L.tube_flags(14, 14, 12, 6.5, 6.5, 4.0, elastic=True)
    mesh = L.cylinder_mesh(6.5, 6.5, 4.0, 2.0, 9.0, 1.1)
    bcs = [(L.BC_PRESSURE_CONST, [3e-4], ()),
           (L.BC_PRESSURE_CONST, [0.0], ()),
           (L.BC_PRESSURE_CONST, [1e-4], ())]
    o, b = _pair(oracle_mod, fl, 0.7, 41, bcs, membrane=(mesh, 0.05, 1e-3, 2.0, -0.05, -0.5))
    _compare(o, b, 4)
    lo, lb = o.lagrangian(), b.mesh
    assert np.abs(lo["X"] - lb["X"]).max() < 1e-14
    assert np.abs(lo["slip"] - lb["slip"]).max() < 1e-14     # V_s = X - Xprev at |X| ~ 10


def _normal(o, b):
    o.set_nee_variant(1)
    b.nee_normal = True


@pytest.mark.parametrize("seed", [1, 2])
def test_normal_neighbour_extrapolation(oracle_mod, seed):
    """The normal-neighbour variant of Eq. Non-equilibrium3 (x_f one cell in
    from the ghost along its plane's normal) with pressure- and
    velocity-type boundaries on random geometry, where some ghosts have a
    solid normal neighbour (the receiving cell stands in for it)."""
    fl = L.random_flags(7, 6, 9, seed=seed)
    bcs = [(L.BC_PRESSURE_CONST, [2e-4], ()),
           (L.BC_WINDKESSEL3, [0.05, 50.0, 1.0, 1.0], [2e-4]),
           (L.BC_VELOCITY_CONST, [-1e-3], ())]
    o, b = _pair(oracle_mod, fl, 0.7 + 0.1 * seed, seed + 50, bcs)
    _normal(o, b)
    _compare(o, b, 6)


def test_normal_neighbour_lv_valve_cycle(oracle_mod):
    """LV inlet with the normal-neighbour variant: the snapshot and the
    smoothed closure read the normal neighbour's record."""
    fl = L.tube_flags(9, 9, 10, 4.0, 4.0, 3.2)
    sc = L.scales(sigma_t=400.0, sigma_V=40.0, sigma_P=2.5e-5)
    par = L.lv_params(2.0, 0.06, 75.0, 8.0, 0.01, sc)
    bcs = [(L.BC_LV_ELASTANCE, par, ()),
           (L.BC_WINDKESSEL3, L.wk_params(0.05, 1.5, 1.0, sc), [80 * 2.5e-5]),
           (L.BC_PRESSURE_CONST, [0.0], ())]
    o, b = _pair(oracle_mod, fl, 0.8, 31, bcs, amp=0.0)
    _normal(o, b)
    for _ in range(150):
        o.step(1)
        b.step()
    w = o.waveforms()
    assert w[:, 11].max() == 1.0 and w[-1, 11] == 0.0
    assert np.abs(o.get_pops() - b.pops()).max() <= ATOL
    assert np.abs(w[:, :5] - np.array(b.records)).max() <= ATOL * 100
