"""Launch shapes per size class and the autotuner.

The collide-stream result is independent of the workgroup size and cells
per lane (bitwise); the wall tile (any of the six shapes) changes only the
rounding order of the spread force's float additions.  The autotuner's trial steps are ordinary
steps of the method, and its choices round-trip through the JSON cache.
"""
import json

import numpy as np
import pytest

import lbm_inputs as L

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def amd():
    import paper_2112_05258_amd as amd
    amd.lib()
    return amd


# the wall tile shapes (theta x z mesh points)
TILES = [(8, 32), (16, 16), (32, 8), (8, 16), (16, 8), (8, 8)]


def _rigid(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        r = int(rng.integers(3, 8))
        nz = int(rng.integers(10, 30))
        nx = ny = 2 * r + 4
        out.append(dict(nx=nx, ny=ny, nz=nz, tau=0.7, flags=L.tube_flags(nx, ny, nz, (nx - 1) / 2, (ny - 1) / 2, r),
                        inlet=(L.BC_PRESSURE_CONST, [(1 + k) * 1e-4]),
                        outlet=(L.BC_WINDKESSEL3, [1e-4, 1e6, 0.5, 0.0]), outlet_state=[0.0],
                        p_init=(1 + k) * 1e-4, p_ref=(1 + k) * 1e-4))
    return out


def test_collide_shapes_do_not_change_results(amd):
    cfgs = _rigid(9, seed=4)
    ref = amd.solver_from_configs(cfgs, precision=amd.FP64)
    assert len(ref.classes()) == 4
    ref.step(23)
    ref.sync()
    shapes = [(128, 2, 8), (512, 1, 32), (128, 1, 16), (512, 2, 8)]
    s = amd.solver_from_configs(cfgs, precision=amd.FP64)
    for q, sh in enumerate(shapes):
        s.set_launch(q, *sh)
    assert [(c["block"], c["cells_per_lane"], c["wall_tile_theta"]) for c in s.classes()] == shapes
    s.step(23)
    s.sync()
    for k in range(len(cfgs)):
        assert np.array_equal(s.read_populations(k), ref.read_populations(k)), k
        assert np.array_equal(s.waveforms(k), ref.waveforms(k)), k


def test_wall_tiles_agree_to_rounding(amd):
    ps = L.ensemble(8, seed=5)
    for p in ps:
        p["L"] = min(p["L"], 40)
    cfgs = [L.ensemble_config(p) for p in ps]
    out = []
    for tj, tk in TILES:
        s = amd.solver_from_configs(cfgs, precision=amd.FP64)
        for q in range(len(s.classes())):
            s.set_launch(q, 256, 1, tj, tk)
        s.step(31)
        s.sync()
        out.append([s.read_wall(k)["X"] - c["mesh"]["X0"] for k, c in enumerate(cfgs)])
        s.close()
    for a in out[1:]:
        for k in range(len(cfgs)):
            e = np.linalg.norm(a[k] - out[0][k]) / np.linalg.norm(out[0][k])
            assert e <= 1e-12, (k, e)


def test_autotune_steps_are_ordinary_and_cache_round_trips(amd, tmp_path):
    cfgs = _rigid(9, seed=6)
    cache = str(tmp_path / "launch.json")
    s = amd.solver_from_configs(cfgs, precision=amd.FP64)
    adv = s.autotune(trial_steps=4, cache=cache)
    assert adv == 7 * (4 + 2)                  # no walls: current + 6 collide shapes
    assert s.t == adv
    ref = amd.solver_from_configs(cfgs, precision=amd.FP64)
    ref.step(adv)
    s.sync()
    ref.sync()
    for k in range(len(cfgs)):
        assert np.array_equal(s.read_populations(k), ref.read_populations(k)), k
    tab = json.load(open(cache))["classes"]
    assert len(tab) >= 1
    chosen = s.classes()
    s2 = amd.solver_from_configs(cfgs, precision=amd.FP64)
    assert s2.autotune(trial_steps=4, cache=cache) == 0      # from the cache
    assert s2.classes() == chosen


def test_autotune_with_walls_and_bad_shapes(amd):
    ps = L.ensemble(8, seed=7)
    for p in ps:
        p["L"] = min(p["L"], 40)
    s = amd.solver_from_configs([L.ensemble_config(p) for p in ps], precision=amd.FP32)
    adv = s.autotune(trial_steps=2)
    assert adv == (7 + 7) * (2 + 2)           # current + 6 shapes, current + 6 tiles
    for c in s.classes():
        assert c["block"] in (128, 256, 512) and c["cells_per_lane"] in (1, 2)
        assert (c["wall_tile_theta"], c["wall_tile_z"]) in TILES
    s.step(10)
    s.sync()
    with pytest.raises(amd.LbmError):
        s.set_launch(0, 64, 1, 16)
    with pytest.raises(amd.LbmError):
        s.set_launch(0, 256, 3, 16)
    with pytest.raises(amd.LbmError):
        s.set_launch(0, 256, 1, 12)
    with pytest.raises(amd.LbmError):
        s.set_launch(0, 256, 1, 32, 16)      # 512 points: more than a workgroup's lanes
    with pytest.raises(amd.LbmError):
        s.set_launch(0, 256, 1, 8, 4)


def test_default_wall_tile_follows_the_mesh(amd):
    """Without shapes set, attaching a wall picks the square 256-point tile
    unless its stencil boxes would fill more than 60 % of the standard
    staging; then the first of 16 x 8, 8 x 16, 8 x 8 whose boxes do not.
    Largest boxes at rest (cells; standard staging 1 792): cfg1 at 0.5 lu,
    16 x 16: 990, kept; at 0.9 lu: 16 x 16 3 276, 16 x 8 2 002, 8 x 16
    1 296, 8 x 8 792 -> 8 x 8; the small tube at 0.7 lu: 16 x 16 1 694,
    16 x 8 1 089, 8 x 16 756 -> 8 x 16.  Shapes set by the caller stay."""
    cases = [(L.cfg1(h=0.5), (16, 16)), (L.cfg1(h=0.9), (8, 8)), (L.small_fsi(h=0.7), (8, 16))]
    for c, want in cases:
        s = amd.solver_from_config(c, precision=amd.FP32)
        k = s.classes()[0]
        assert (k["wall_tile_theta"], k["wall_tile_z"]) == want, (c["name"], k)
        s.close()
    c = L.small_fsi(h=0.7)
    s = amd.solver_from_config(c, precision=amd.FP32)
    s.set_launch(0, 256, 1, 32)
    s.step(2)
    s.sync()
    k = s.classes()[0]
    assert (k["wall_tile_theta"], k["wall_tile_z"]) == (32, 8)
    s.close()
