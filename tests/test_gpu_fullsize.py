"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (HIP graph replays, default or autotuned launch shapes), on outputs the
oracle computes directly: every fluid cell, the boundary waveforms and every
wall point after a few steps of cfg1 (8.4 M cells, 612 045 wall points),
members of the 256-tube ensemble, the 16-bit storage mode, and the
surrogate's inference at batch 65 536.  The oracle runs on the host's cores
(about a second per cfg1 step on 16 threads), so the runs are short; the
initial populations are seeded random deviations so that every cell moves.
"""
import os

import numpy as np
import pytest

import lbm_inputs as L

pytestmark = pytest.mark.gpu

STEPS = 24


@pytest.fixture(scope="module")
def amd():
    import paper_2112_05258_amd as amd
    amd.lib()
    return amd


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def cfg1_runs(oracle_mod, amd):
    c = L.cfg1()
    g = L.random_populations(c["flags"].size, seed=61, amp=2e-4)
    o = oracle_mod.from_config(c, pops=g)
    o.step(STEPS)
    res = {"cfg": c, "oracle": (o.fields(), o.waveforms(), o.displacement()[0])}
    for name, prec in (("fp32", amd.FP32), ("fp16s", amd.FP16S)):
        s = amd.solver_from_config(c, precision=prec, pops=g)
        s.step(STEPS)
        s.sync()
        res[name] = (s.fields(), s.waveforms(), s.read_wall()["X"] - c["mesh"]["X0"])
        s.close()
    return res


def _fluid(c):
    return np.flatnonzero(c["flags"].ravel() == L.FLUID)


def test_cfg1_fp32_full_size_matches_oracle(cfg1_runs):
    c = cfg1_runs["cfg"]
    (po, uo), wo, Do = cfg1_runs["oracle"]
    (ps, us), ws, Ds = cfg1_runs["fp32"]
    k = _fluid(c)
    e = {"u": _rel(us.reshape(-1, 3)[k], uo.reshape(-1, 3)[k]),
         "p": _rel(ps.ravel()[k], po.ravel()[k]),
         "Q": _rel(ws[:, (1, 3, 12)], wo[:, (1, 3, 12)]),
         "P": _rel(ws[:, (2, 4, 13)], wo[:, (2, 4, 13)]),
         "wall": _rel(Ds, Do)}
    print({a: f"{b:.2e}" for a, b in e.items()}, flush=True)
    for a, b in e.items():
        assert b <= 1e-5, (a, b)
    # error-vs-step curve of the boundary records (flux, pressure per step)
    curve = [max(_rel(ws[k, (1, 3, 12)], wo[k, (1, 3, 12)]), _rel(ws[k, (2, 4, 13)], wo[k, (2, 4, 13)]))
             for k in range(len(wo))]
    print({"error_vs_step": [f"{v:.1e}" for v in curve]}, flush=True)
    assert max(curve) <= 1e-5


def test_cfg1_fp16s_full_size_within_storage_bound(cfg1_runs):
    """FP16 keeps 11 significant bits: each stored deviation is rounded
    with relative error <= 2^-11 = 4.9e-4, and the velocity sums 19 of
    them per step, so after 24 steps the field agrees to about
    2^-11 * sqrt(19 * 24) ~ 1e-2 relative at most (random rounding); the
    bar is that estimate."""
    c = cfg1_runs["cfg"]
    (po, uo), wo, Do = cfg1_runs["oracle"]
    (ps, us), ws, Ds = cfg1_runs["fp16s"]
    k = _fluid(c)
    e = {"u": _rel(us.reshape(-1, 3)[k], uo.reshape(-1, 3)[k]),
         "p": _rel(ps.ravel()[k], po.ravel()[k]),
         "wall": _rel(Ds, Do)}
    print({a: f"{b:.2e}" for a, b in e.items()}, flush=True)
    for a, b in e.items():
        assert b <= 1e-2, (a, b)


def test_ensemble_members_full_size_match_oracle(oracle_mod, amd):
    """All 256 tubes advanced together with autotuned launch shapes; the
    smallest, the median and the largest member against the oracle."""
    cfgs = [L.ensemble_config(p) for p in L.ensemble(256, 3)]
    for c in cfgs:   # drive every member with an inlet 50 mmHg above P0
        c["inlet"] = (L.BC_PRESSURE_CONST, [c["p_init"] + 50 * c["scales"]["sigma_P"]])
    s = amd.solver_from_configs(cfgs, precision=amd.FP32)
    adv = s.autotune(trial_steps=4)
    s.step(60 - adv % 2)
    s.sync()
    n = s.t
    sizes = np.array([c["flags"].size for c in cfgs])
    order = np.argsort(sizes)
    for k in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
        o = oracle_mod.from_config(cfgs[k])
        o.step(n)
        (po, uo), (ps, us) = o.fields(), s.fields(k)
        fl = cfgs[k]["flags"] == L.FLUID
        e_u, e_p = _rel(us[fl], uo[fl]), _rel(ps[fl], po[fl])
        e_w = _rel(s.read_wall(k)["X"] - cfgs[k]["mesh"]["X0"], o.displacement()[0])
        print({"member": k, "cells": int(sizes[k]), "u": f"{e_u:.2e}", "p": f"{e_p:.2e}", "wall": f"{e_w:.2e}"},
              flush=True)
        assert e_u <= 1e-5 and e_p <= 1e-5 and e_w <= 1e-5
    s.close()


WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2112_05258_amd",
                       "surrogate_weights.npz")


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained surrogate weights in the package")
def test_surrogate_inference_full_batch_matches_oracle(amd):
    """Inference of 65 536 parameter sets in one call; 512 rows spread
    over the batch against the FP64 network (BF16 operands: bar 2e-2)."""
    from oracle import mlp
    from paper_2112_05258_amd import surrogate as S
    s = S.Surrogate.load(WEIGHTS, max_batch=65536)
    X = L.surrogate_params(65536, seed=77)
    Y = s.predict(X).cpu().numpy()
    d = np.load(WEIGHTS)
    rows = np.linspace(0, 65535, 512).astype(int)
    yo, _, _ = mlp.forward(d["theta"].astype(np.float64), mlp.layer_shapes(),
                           mlp.normalise_inputs(X[rows], d["lo"], d["hi"]))
    yo = d["mu"] + d["sigma"] * yo
    e = _rel((Y[rows] - d["mu"]) / d["sigma"], (yo - d["mu"]) / d["sigma"])
    print({"rows": len(rows), "rel_l2_standardised": f"{e:.2e}"}, flush=True)
    assert e <= 2e-2
    s.close()
