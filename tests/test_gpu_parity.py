"""Parity of the HIP path (through the C interface) with the CPU oracle.

Bars: FP64 storage <= 1e-12 relative L2, FP32 storage <= 1e-5 relative L2 on
the velocity (first moment) and the gauge pressure over the fluid cells, and
on the boundary waveforms.  FP64 runs are compared with the extended-precision
(long double) build of the oracle: the FP64 build's own rounding is ~1e-12
relative on slow flows (see test_oracle_noise_floor), as large as the bar.
Inputs are seeded (lbm_inputs); no expected value comes from the GPU.
"""
import numpy as np
import pytest

import lbm_inputs as L

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    a = np.asarray(a, float).ravel()
    b = np.asarray(b, float).ravel()
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


@pytest.fixture(scope="module")
def amd():
    import paper_2112_05258_amd as amd
    amd.lib()
    return amd


def wall_bar(precision, tol, n):
    """Bar of the wall's displacement and penalty force after n steps: FP64
    sums the spread force's atomic-order rounding through the slip integral
    and the displacement recursion, sqrt(n) * tol; FP32 meets tol itself."""
    return tol * np.sqrt(n) if precision == "FP64" else tol


def _run_pair(oracle_mod, amd, cfg, steps, precision, pops=None, **kw):
    o = oracle_mod.from_config(cfg, pops=pops, extended=(precision == amd.FP64))
    s = amd.solver_from_config(cfg, precision=precision, pops=pops, **kw)
    o.step(steps)
    s.step(steps)
    s.sync()
    return o, s


def _compare(o, s, fl, tol, wave_cols=(1, 2, 3, 4, 9, 10, 12, 13), check_pops=True):
    po, uo = o.fields()
    ps, us = s.fields()
    fluid = fl == L.FLUID
    e_u = rel_l2(us[fluid], uo[fluid])
    e_p = rel_l2(ps[fluid], po[fluid])
    wo = o.waveforms()
    ws = s.waveforms()
    assert ws.shape == wo.shape, (ws.shape, wo.shape)
    errs = {"u": e_u, "p": e_p}
    # waveforms: error over the norm of their family (fluxes Q_in, Q_out,
    # Q_mid; pressures p_in, p_out, Pv, Pw, p_mid), so that a boundary whose flux is ~0
    # (closed valve) is not judged by its rounding noise alone
    fam = {c: (1, 3, 12) for c in (1, 3, 12)}
    fam.update({c: (2, 4, 9, 10, 13) for c in (2, 4, 9, 10, 13)})
    for c in wave_cols:
        den = max(np.linalg.norm(wo[:, k]) for k in fam[c])
        if den > 0:
            errs[f"wave{c}"] = np.linalg.norm(ws[:, c] - wo[:, c]) / den
    assert np.array_equal(ws[:, 0], wo[:, 0])
    assert np.array_equal(ws[:, 5], wo[:, 5]) and np.array_equal(ws[:, 11], wo[:, 11])
    if check_pops:
        gs, go = s.read_populations(), o.get_pops()
        errs["g"] = rel_l2(gs, go)
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v <= tol, (k, v, tol)
    return errs


def test_rigid_tube_fp64_1000_steps(oracle_mod, amd):
    """Rigid tube r = 8 in 24x24x64, constant inlet, Windkessel outlet."""
    c = L.cfg0()
    o, s = _run_pair(oracle_mod, amd, c, 1000, amd.FP64)
    _compare(o, s, c["flags"], 1e-12)


def test_rigid_tube_fp32_1000_steps(oracle_mod, amd):
    c = L.cfg0()
    o, s = _run_pair(oracle_mod, amd, c, 1000, amd.FP32)
    _compare(o, s, c["flags"], 1e-5)


@pytest.mark.parametrize("seed,dims", [(1, (29, 23, 37)), (2, (17, 40, 21)), (3, (64, 9, 13))])
def test_random_geometry_fp64(oracle_mod, amd, seed, dims):
    """Random solid cells, random ghost planes, random populations; an odd
    number of steps so both AA parities and the ragged last block are hit."""
    nx, ny, nz = dims
    fl = L.random_flags(nx, ny, nz, seed=seed)
    c = dict(nx=nx, ny=ny, nz=nz, tau=0.6 + 0.1 * seed, flags=fl,
             inlet=(L.BC_PRESSURE_CONST, [2e-4]),
             # flux-driven coupling is stable for Rp << c_s / A and C >> A / c_s
             outlet=(L.BC_WINDKESSEL3, [1e-4, 1e5, 0.5, 0.0]), outlet_state=[1e-4],
             exterior=(L.BC_PRESSURE_CONST, [-1e-4]))
    g = L.random_populations(fl.size, seed=100 + seed)
    o, s = _run_pair(oracle_mod, amd, c, 57, amd.FP64, pops=g)
    _compare(o, s, fl, 1e-12)


@pytest.mark.parametrize("precision,tol", [("FP64", 1e-12), ("FP32", 1e-5)])
def test_velocity_couplings(oracle_mod, amd, precision, tol):
    fl = L.random_flags(20, 18, 24, seed=7)
    c = dict(nx=20, ny=18, nz=24, tau=0.9, flags=fl,
             inlet=(L.BC_VELOCITY_CONST, [3e-3]),
             outlet=(L.BC_WINDKESSEL3, [0.05, 50.0, 1.0, 1.0]), outlet_state=[2e-4],
             exterior=(L.BC_VELOCITY_CONST, [-1e-3]))
    g = L.random_populations(fl.size, seed=8)
    o, s = _run_pair(oracle_mod, amd, c, 40, getattr(amd, precision), pops=g)
    _compare(o, s, fl, tol)


@pytest.mark.parametrize("precision,tol", [("FP64", 1e-12), ("FP32", 1e-5)])
def test_lv_inlet_valve_cycle(oracle_mod, amd, precision, tol):
    """LV elastance inlet over a beat and a half (320 steps a beat): opening,
    ejection, closure with the per-node snapshot and the smoothing to zero,
    the reset at the next beat and the second opening."""
    fl = L.tube_flags(16, 16, 24, 7.5, 7.5, 6.0)
    sc = L.scales(sigma_t=400.0, sigma_V=2.0, sigma_P=2.5e-5)
    par = L.lv_params(2.0, 0.06, 75.0, 8.0, 0.03, sc)
    c = dict(nx=16, ny=16, nz=24, tau=0.8, flags=fl,
             inlet=(L.BC_LV_ELASTANCE, par),
             outlet=(L.BC_WINDKESSEL3, L.wk_params(0.05, 1.5, 1.0, sc)), outlet_state=[80 * 2.5e-5],
             p_init=80 * 2.5e-5, p_ref=80 * 2.5e-5)
    o, s = _run_pair(oracle_mod, amd, c, 400, getattr(amd, precision))
    v = o.waveforms()[:, 11]
    assert (np.diff(v) == -1).sum() == 1 and (np.diff(v) == 1).sum() == 2   # open, close, reopen
    _compare(o, s, fl, tol)


@pytest.mark.parametrize("precision,tol", [("FP64", 1e-12), ("FP32", 1e-5)])
def test_small_elastic_tube(oracle_mod, amd, precision, tol):
    """Elastic tube (immersed membrane, LV inlet, Windkessel outlet, exterior
    at P0): lattice fields, waveforms and wall positions.  Wall bar in FP64
    (wall_bar): the order of the spread force's atomic additions varies, and
    both the slip integral behind the penalty force F (a small difference
    Vf - Vs) and the displacement recursion D^{n+1} = 2 D^n - D^{n-1} +
    (f - F)/m sum that rounding over the n steps like a random walk, so the
    bar is sqrt(n) times the fields' 1e-12; FP32 meets the plain bar."""
    c = L.small_fsi()
    o, s = _run_pair(oracle_mod, amd, c, 120, getattr(amd, precision))
    _compare(o, s, c["flags"], tol)
    lo, ls = o.lagrangian(), s.read_wall()
    Do, _ = o.displacement()
    X0 = c["mesh"]["X0"]
    e_x = rel_l2(ls["X"] - X0, Do)
    e_f = rel_l2(ls["F"], lo["F"])
    print({"wall_X": f"{e_x:.2e}", "wall_F": f"{e_f:.2e}"}, flush=True)
    assert e_x <= wall_bar(precision, tol, 120) and e_f <= wall_bar(precision, tol, 120)


@pytest.mark.parametrize("precision,tol", [("FP64", 1e-12), ("FP32", 1e-5)])
def test_cosine_kernel_small_elastic_tube(oracle_mod, amd, precision, tol):
    """The variant delta kernel (1 + cos(pi r / 2)) / 4 in interpolation and
    spreading: the small elastic tube against the oracle's kernel 1."""
    c = L.small_fsi()
    c["kernel"] = 1
    o, s = _run_pair(oracle_mod, amd, c, 120, getattr(amd, precision))
    _compare(o, s, c["flags"], tol)
    Do, _ = o.displacement()
    e_x = rel_l2(s.read_wall()["X"] - c["mesh"]["X0"], Do)
    e_f = rel_l2(s.read_wall()["F"], o.lagrangian()["F"])
    print({"wall_X": f"{e_x:.2e}", "wall_F": f"{e_f:.2e}"}, flush=True)
    assert e_x <= wall_bar(precision, tol, 120) and e_f <= wall_bar(precision, tol, 120)


@pytest.mark.parametrize("precision,tol", [("FP64", 1e-12), ("FP32", 1e-5)])
def test_external_solid_prescribed_motion(oracle_mod, amd, precision, tol):
    """External-solid mode: the caller breathes the tube radially (amplitude
    0.3 lu, period 60 steps), handing positions and velocities over every
    third step (ballistic motion in between); the library interpolates,
    forms the penalty force and spreads it.  Fields, waveforms, positions
    and the force on the fluid against the oracle's external mode."""
    c = L.small_fsi()
    c["wall_mode"] = 1
    o = oracle_mod.from_config(c, extended=(precision == "FP64"))
    s = amd.solver_from_config(c, precision=getattr(amd, precision))
    X0 = c["mesh"]["X0"]
    rad = X0 - np.array([(c["nx"] - 1) / 2, (c["ny"] - 1) / 2, 0.0])
    rad[:, 2] = 0.0
    rad /= np.linalg.norm(rad, axis=1, keepdims=True)
    w = 2 * np.pi / 60
    for n in range(0, 90, 3):
        X = X0 + 0.3 * np.sin(w * n) * rad
        V = 0.3 * w * np.cos(w * n) * rad
        o.set_wall(X, V)
        s.set_wall(X, V)
        o.step(3)
        s.step(3)
    s.sync()
    _compare(o, s, c["flags"], tol)
    lo, ls = o.lagrangian(), s.read_wall()
    e_x = rel_l2(ls["X"] - X0, lo["X"] - X0)
    e_f = rel_l2(ls["F"], lo["F"])
    print({"wall_X": f"{e_x:.2e}", "wall_F": f"{e_f:.2e}"}, flush=True)
    assert e_x <= tol and e_f <= tol   # the positions are the caller's
    with pytest.raises(amd.LbmError):   # a built-in membrane takes no positions
        t = amd.solver_from_config(L.small_fsi(), precision=amd.FP32)
        try:
            t.set_wall(X, V)
        finally:
            t.close()


@pytest.mark.parametrize("h,tj,tk", [(0.7, 16, 0), (0.7, 32, 0), (1.4, 16, 0), (0.7, 8, 8), (0.7, 16, 8),
                                     (1.4, 8, 16), (1.4, 8, 8)])
def test_wall_staging_paths(oracle_mod, amd, h, tj, tk):
    """The wall exchange's three ways of handling a tile's stencil box, each
    against the oracle (the library picks the kernel from the rest shape; the
    box sizes below follow from the mesh).  h = 0.7, 16 x 16 tiles: boxes of
    600-1694 cells, the large-box kernel stages them all; h = 0.7, 32 x 8:
    1188-1782 cells, the standard kernel stages them all; h = 1.4, 16 x 16:
    3060-4950 cells, the large-box kernel stages those up to 4096 and the
    rest take the unstaged path (stencils read and spread in global memory).
    The smaller tiles: h = 0.7, 8 x 8: 252-486 cells and 16 x 8: 600-1089,
    the standard kernel (lanes without a point idle); h = 1.4, 8 x 16:
    1700-2750 and 8 x 8: 600-1540, the large-box kernel."""
    c = L.small_fsi(h=h)
    o = oracle_mod.from_config(c, extended=True)
    s = amd.solver_from_config(c, precision=amd.FP64)
    s.set_launch(0, 256, 1, tj, tk)
    assert s.classes()[0]["wall_tile_z"] == (tk or 256 // tj)
    o.step(60)
    s.step(60)
    s.sync()
    _compare(o, s, c["flags"], 1e-12)
    Do, _ = o.displacement()
    X = s.read_wall()["X"]
    e_x = rel_l2(X - c["mesh"]["X0"], Do)
    floor = np.finfo(float).eps * np.linalg.norm(X) / np.linalg.norm(Do)
    assert e_x <= 1e-11 + floor, (e_x, floor)


def test_band_follows_a_moving_wall(oracle_mod, amd):
    """The wall moves 2.9 lu outwards: with the band fixed where it was
    built the stencils leave it (LBM_E_BAND); with the periodic motion test
    the band is rebuilt around the wall and the run matches the oracle
    (which interpolates over every fluid cell) to the FP64 bar."""
    c = L.inflating_tube()
    s = amd.solver_from_config(c, precision=amd.FP64)
    s.set_band_check(0)
    s.step(c["steps"])
    with pytest.raises(amd.LbmError) as e:
        s.sync()
    assert e.value.code == -6
    s.close()
    o, s = _run_pair(oracle_mod, amd, c, c["steps"], amd.FP64)
    _compare(o, s, c["flags"], 1e-12, wave_cols=(1, 2, 3, 4))
    Do, _ = o.displacement()
    e_x = rel_l2(s.read_wall()["X"] - c["mesh"]["X0"], Do)
    print({"wall_X": f"{e_x:.2e}", "max_D": f"{np.abs(Do).max():.2f}"}, flush=True)
    assert np.abs(Do).max() > 2.5 and e_x <= 1e-11


def test_graph_replay_matches_eager(amd):
    c = L.cfg0()
    out = []
    for graph in (True, False):
        s = amd.solver_from_config(c, precision=amd.FP64)
        s.set_graph(graph)
        s.step(101)
        s.sync()
        out.append((s.read_populations(), s.waveforms()))
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])


def test_edge_cases(oracle_mod, amd):
    # thinnest box: one fluid layer between the planes
    fl = np.full((3, 5, 5), L.SOLID, np.uint8)
    fl[1, 1:4, 1:4] = L.FLUID
    fl[0, 1:4, 1:4] = L.INLET
    fl[2, 1:4, 1:4] = L.OUTLET
    c = dict(nx=5, ny=5, nz=3, tau=0.7, flags=fl, inlet=(L.BC_PRESSURE_CONST, [1e-4]),
             outlet=(L.BC_PRESSURE_CONST, [0.0]))
    o, s = _run_pair(oracle_mod, amd, c, 9, amd.FP64)
    _compare(o, s, fl, 1e-12)
    # no fluid at all: steps and 0D models still advance
    fl = np.full((4, 4, 4), L.SOLID, np.uint8)
    c = dict(nx=4, ny=4, nz=4, tau=0.7, flags=fl, outlet=(L.BC_WINDKESSEL3, [0.1, 10.0, 1.0, 0.0]),
             outlet_state=[1e-3])
    o, s = _run_pair(oracle_mod, amd, c, 5, amd.FP32)
    assert s.t == 5
    assert np.allclose(s.waveforms()[:, 10], o.waveforms()[:, 10], rtol=1e-6)


def test_invalid_inputs_rejected(amd):
    fl = L.tube_flags(8, 8, 8, 3.5, 3.5, 3.0)
    bad = fl.copy()
    bad[0, 4, 4] = L.FLUID
    with pytest.raises(amd.LbmError):
        amd.Solver(dict(nx=8, ny=8, nz=8, tau=0.8, flags=bad))
    with pytest.raises(amd.LbmError):
        amd.Solver(dict(nx=8, ny=8, nz=8, tau=0.5, flags=fl))
    s = amd.Solver(dict(nx=8, ny=8, nz=8, tau=0.8, flags=fl))
    with pytest.raises(amd.LbmError):
        s.couple_0d(0, 1, L.BC_LV_ELASTANCE, [1.0] * 11)
    s.step(1)
    with pytest.raises(amd.LbmError):
        s.write_populations(np.zeros((fl.size, 19)))
