"""Parity of the normal-neighbour variant of the non-equilibrium
extrapolation (Eq. Non-equilibrium3 with x_f the ghost's neighbour along the
inward normal of its face) between the HIP path and the oracle.

Same bars as the literal reading: FP64 storage <= 1e-12 relative L2 against
the extended-precision oracle, FP32 <= 1e-5.  Every case also checks that
the variant moves the oracle's result well past the bar, so that the cases
do exercise the cells where the two readings differ (edge directions out of
a ghost whose normal neighbour is fluid).
"""
import numpy as np
import pytest

import lbm_inputs as L
from test_gpu_parity import _compare, _run_pair, rel_l2, wall_bar

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def amd():
    import paper_2112_05258_amd as amd
    amd.lib()
    return amd


def _literal_differs(oracle_mod, cfg, steps, pops=None, floor=1e-6):
    """The literal reading's oracle ends measurably away from the variant's."""
    a = oracle_mod.from_config(dict(cfg, nee_variant=0), pops=pops)
    b = oracle_mod.from_config(dict(cfg, nee_variant=1), pops=pops)
    a.step(steps)
    b.step(steps)
    d = rel_l2(a.get_pops(), b.get_pops())
    assert d > floor, d


@pytest.mark.parametrize("seed,dims", [(1, (29, 23, 37)), (2, (17, 40, 21)), (3, (64, 9, 13))])
def test_random_geometry_fp64(oracle_mod, amd, seed, dims):
    """Random solid cells and ghost planes (ghost edges and corners, ghosts
    whose normal neighbour is solid), random populations, an odd number of
    steps (both AA parities)."""
    nx, ny, nz = dims
    fl = L.random_flags(nx, ny, nz, seed=seed)
    c = dict(nx=nx, ny=ny, nz=nz, tau=0.6 + 0.1 * seed, flags=fl, nee_variant=1,
             inlet=(L.BC_PRESSURE_CONST, [2e-4]),
             outlet=(L.BC_WINDKESSEL3, [1e-4, 1e5, 0.5, 0.0]), outlet_state=[1e-4],
             exterior=(L.BC_PRESSURE_CONST, [-1e-4]))
    g = L.random_populations(fl.size, seed=100 + seed)
    o, s = _run_pair(oracle_mod, amd, c, 57, amd.FP64, pops=g)
    _compare(o, s, fl, 1e-12)
    _literal_differs(oracle_mod, c, 57, pops=g)


@pytest.mark.parametrize("precision,tol", [("FP64", 1e-12), ("FP32", 1e-5)])
def test_velocity_couplings(oracle_mod, amd, precision, tol):
    """Velocity-type boundaries: constant v*, and the flux-corrected v(x_f)
    of the Windkessel in mode 1 (read at the normal neighbour)."""
    fl = L.random_flags(20, 18, 24, seed=7)
    c = dict(nx=20, ny=18, nz=24, tau=0.9, flags=fl, nee_variant=1,
             inlet=(L.BC_VELOCITY_CONST, [3e-3]),
             outlet=(L.BC_WINDKESSEL3, [0.05, 50.0, 1.0, 1.0]), outlet_state=[2e-4],
             exterior=(L.BC_VELOCITY_CONST, [-1e-3]))
    g = L.random_populations(fl.size, seed=8)
    o, s = _run_pair(oracle_mod, amd, c, 40, getattr(amd, precision), pops=g)
    _compare(o, s, fl, tol)
    if precision == "FP64":
        _literal_differs(oracle_mod, c, 40, pops=g)


@pytest.mark.parametrize("precision,tol", [("FP64", 1e-12), ("FP32", 1e-5)])
def test_lv_inlet_valve_cycle(oracle_mod, amd, precision, tol):
    """LV inlet over a beat and a half: the closure's snapshot and smoothed
    velocity are read at the normal neighbour's column."""
    fl = L.tube_flags(16, 16, 24, 7.5, 7.5, 6.0)
    sc = L.scales(sigma_t=400.0, sigma_V=2.0, sigma_P=2.5e-5)
    par = L.lv_params(2.0, 0.06, 75.0, 8.0, 0.03, sc)
    c = dict(nx=16, ny=16, nz=24, tau=0.8, flags=fl, nee_variant=1,
             inlet=(L.BC_LV_ELASTANCE, par),
             outlet=(L.BC_WINDKESSEL3, L.wk_params(0.05, 1.5, 1.0, sc)), outlet_state=[80 * 2.5e-5],
             p_init=80 * 2.5e-5, p_ref=80 * 2.5e-5)
    o, s = _run_pair(oracle_mod, amd, c, 400, getattr(amd, precision))
    v = o.waveforms()[:, 11]
    assert (np.diff(v) == -1).sum() == 1 and (np.diff(v) == 1).sum() == 2
    _compare(o, s, fl, tol)
    if precision == "FP64":
        _literal_differs(oracle_mod, c, 400)


@pytest.mark.parametrize("precision,tol", [("FP64", 1e-12), ("FP32", 1e-5)])
def test_elastic_tube(oracle_mod, amd, precision, tol):
    """Elastic wall (IB forcing on band cells) with the variant at the inlet
    and outlet planes.  Wall bar as for the elastic tube without the variant
    (wall_bar: sqrt(n) tol in FP64 for the atomic-order rounding the slip
    integral and the displacement recursion sum over n steps, tol in FP32);
    the wall is compared through X - X0 with X read back in absolute
    coordinates, so the bar on the displacement adds the rounding of that
    read-back, eps |X| / |D| (~1e-11 here: |X| ~ 10, |D| ~ 3e-4 after 120
    steps)."""
    c = dict(L.small_fsi(), nee_variant=1)
    o, s = _run_pair(oracle_mod, amd, c, 120, getattr(amd, precision))
    _compare(o, s, c["flags"], tol)
    Do, _ = o.displacement()
    X = s.read_wall()["X"]
    e_x = rel_l2(X - c["mesh"]["X0"], Do)
    e_f = rel_l2(s.read_wall()["F"], o.lagrangian()["F"])
    floor = np.finfo(float).eps * np.linalg.norm(X) / np.linalg.norm(Do)
    print({"wall_X": f"{e_x:.2e}", "wall_F": f"{e_f:.2e}", "readback": f"{floor:.2e}"}, flush=True)
    bar = wall_bar(precision, tol, 120)
    assert e_x <= bar + floor and e_f <= bar
    if precision == "FP64":
        _literal_differs(oracle_mod, c, 120)


def test_mixed_ensemble_fp64(oracle_mod, amd):
    """One context holding instances with and without the variant: each
    instance follows its own reading."""
    cfgs = []
    for k, (seed, dims) in enumerate([(11, (13, 12, 17)), (12, (21, 9, 14)), (13, (10, 15, 11))]):
        nx, ny, nz = dims
        fl = L.random_flags(nx, ny, nz, seed=seed)
        cfgs.append(dict(nx=nx, ny=ny, nz=nz, tau=0.7 + 0.05 * k, flags=fl, nee_variant=k % 2,
                         inlet=(L.BC_PRESSURE_CONST, [1e-4 * (k + 1)]),
                         outlet=(L.BC_PRESSURE_CONST, [-1e-4]),
                         exterior=(L.BC_VELOCITY_CONST, [5e-4])))
    pops = [L.random_populations(c["flags"].size, seed=200 + k) for k, c in enumerate(cfgs)]
    s = amd.solver_from_configs(cfgs, precision=amd.FP64)
    for k, g in enumerate(pops):
        s.write_populations(g, inst=k)
    s.step(33)
    s.sync()
    for k, c in enumerate(cfgs):
        o = oracle_mod.from_config(c, pops=pops[k], extended=True)
        o.step(33)
        e = rel_l2(s.read_populations(k), o.get_pops())
        print(k, c["nee_variant"], f"{e:.2e}", flush=True)
        assert e <= 1e-12, (k, e)
