"""Batched ensemble: many independent tubes of uneven size in one context.

Every instance of a batched run must evolve exactly as the same instance run
alone (bitwise for rigid tubes; to FP64 rounding with walls, whose spreading
sums the contributions of neighbouring tiles in a scheduling-dependent order),
and an ensemble member must match the oracle to the FP64 bar.
"""
import numpy as np
import pytest

import lbm_inputs as L

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    den = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (den if den > 0 else 1.0)


@pytest.fixture(scope="module")
def amd():
    import paper_2112_05258_amd as amd
    amd.lib()
    return amd


def _rigid_members(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        r = int(rng.integers(4, 9))
        L_ = int(rng.integers(12, 40))
        nx = 2 * r + 4 + int(rng.integers(0, 3))
        ny = 2 * r + 4
        cx, cy = (nx - 1) / 2, (ny - 1) / 2
        out.append(dict(nx=nx, ny=ny, nz=L_, tau=0.6 + 0.05 * k, flags=L.tube_flags(nx, ny, L_, cx, cy, r),
                        inlet=(L.BC_PRESSURE_CONST, [(1 + k) * 1e-4]),
                        outlet=(L.BC_WINDKESSEL3, [1e-4, 1e6, 0.5 + 0.1 * k, 0.0]), outlet_state=[0.0],
                        p_init=(1 + k) * 1e-4, p_ref=(1 + k) * 1e-4))
    return out


def test_rigid_batch_equals_single_runs_bitwise(amd):
    cfgs = _rigid_members(7, seed=21)
    b = amd.solver_from_configs(cfgs, precision=amd.FP64)
    b.step(63)
    b.sync()
    for k, c in enumerate(cfgs):
        s = amd.solver_from_config(c, precision=amd.FP64)
        s.step(63)
        s.sync()
        assert np.array_equal(b.read_populations(k), s.read_populations()), k
        assert np.array_equal(b.waveforms(k), s.waveforms()), k
        s.close()


@pytest.mark.parametrize("precision,tol", [("FP64", 1e-13), ("FP32", 1e-6)])
def test_elastic_batch_equals_single_runs(amd, precision, tol):
    ps = L.ensemble(5, seed=3)
    for p in ps:                      # keep the tubes short for the test
        p["L"] = min(p["L"], 40)
    cfgs = [L.ensemble_config(p) for p in ps]
    prec = getattr(amd, precision)
    b = amd.solver_from_configs(cfgs, precision=prec)
    b.step(41)
    b.sync()
    for k, c in enumerate(cfgs):
        s = amd.solver_from_config(c, precision=prec)
        s.step(41)
        s.sync()
        pb, ub = b.fields(k)
        ps_, us = s.fields()
        fl = c["flags"] == L.FLUID
        assert rel_l2(ub[fl], us[fl]) <= tol and rel_l2(pb[fl], ps_[fl]) <= tol, k
        # the wall: the two runs' spread forces differ by the order of their
        # atomic additions, a rounding that the slip integral and the
        # displacement recursion sum over the n steps like a random walk
        # (sqrt(n) tol), and X is read back in absolute coordinates, so the
        # displacement X - X0 carries eps |X| / |D| on top
        wb, ws = b.read_wall(k), s.read_wall()
        D = ws["X"] - c["mesh"]["X0"]
        floor = np.finfo(float).eps * np.linalg.norm(ws["X"]) / np.linalg.norm(D)
        e_x = rel_l2(wb["X"] - c["mesh"]["X0"], D)
        print({"member": k, "wall_X": f"{e_x:.2e}", "bar": f"{tol * np.sqrt(41) + floor:.2e}"}, flush=True)
        assert e_x <= tol * np.sqrt(41) + floor, k
        s.close()


def test_ensemble_member_matches_oracle(oracle_mod, amd):
    ps = L.ensemble(3, seed=3)
    for p in ps:
        p["L"] = min(p["L"], 36)
    cfgs = [L.ensemble_config(p) for p in ps]
    # members start in equilibrium with the valve shut; drive them with an
    # inlet pressure 50 mmHg above P0 so that there is flow to compare
    for c in cfgs:
        c["inlet"] = (L.BC_PRESSURE_CONST, [c["p_init"] + 50 * c["scales"]["sigma_P"]])
    b = amd.solver_from_configs(cfgs, precision=amd.FP64)
    b.step(60)
    b.sync()
    k = 1
    o = oracle_mod.from_config(cfgs[k], extended=True)
    o.step(60)
    pb, ub = b.fields(k)
    po, uo = o.fields()
    fl = cfgs[k]["flags"] == L.FLUID
    e_u, e_p = rel_l2(ub[fl], uo[fl]), rel_l2(pb[fl], po[fl])
    wb, wo = b.waveforms(k), o.waveforms()
    e_q = np.linalg.norm(wb[:, 3] - wo[:, 3]) / max(np.linalg.norm(wo[:, 1]), np.linalg.norm(wo[:, 3]))
    print({"u": f"{e_u:.2e}", "p": f"{e_p:.2e}", "Q_out": f"{e_q:.2e}"})
    assert e_u <= 1e-12 and e_p <= 1e-12 and e_q <= 1e-12
