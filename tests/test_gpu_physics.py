"""The small rigid tube (cfg0: r = 8 in 24 x 24 x 64, constant inlet
pressure, 3-element Windkessel outlet) on the GPU for 5 000 steps, to its
steady state: the physics the oracle is pinned by, now checked on the GPU's
own output, and the error against the oracle as a curve over the run.

* Steady Windkessel: the mean outlet pressure is Q (Rp + Rd) (the outlet's
  flux correction leaves ~0.3 %), inflow equals outflow, the recorded
  mid-length flux equals both, and the history has settled.
* Developed flow: the pressure falls linearly along the tube, the recorded
  mid-length pressure sits on that line, and the axial velocity across the
  mid section is a paraboloid of curvature slope / (4 nu) (Poiseuille).
* Error-vs-step curve: relative error of the inlet flux and pressure
  records against the oracle in windows of 500 steps; every window within
  the bar (FP64 1e-12 against the long-double oracle, FP32 1e-5), and the
  fields at the end too.
"""
import numpy as np
import pytest

import lbm_inputs as L

pytestmark = pytest.mark.gpu

STEPS = 5000


@pytest.fixture(scope="module")
def amd():
    import paper_2112_05258_amd as amd
    amd.lib()
    return amd


@pytest.fixture(scope="module")
def oracle_runs(oracle_mod):
    c = L.cfg0()
    out = {}
    for ext in (True, False):
        o = oracle_mod.from_config(c, extended=ext)
        o.step(STEPS)
        out[ext] = (o.fields(), o.waveforms())
    return c, out


def _steady_checks(c, w, p, u):
    Qin, Pin, Qout, Pout = w[-1, 1:5]
    Rp, Cw, Rd = c["outlet"][1][:3]
    assert abs(Qout - Qin) < 1e-4 * Qin
    assert abs(Pout / (Qout * (Rp + Rd)) - 1.0) < 5e-3
    assert np.abs(w[-500:, 3] - Qout).max() < 1e-4 * Qout
    Qmid, Pmid = w[-1, 12:14]
    assert abs(Qmid - Qin) < 1e-4 * Qin
    fl = c["flags"]
    lum = fl[32] == L.FLUID
    pz = np.array([p[z][lum].mean() for z in range(16, 49)])
    slope, icpt = np.polyfit(np.arange(16, 49), pz, 1)
    assert abs(Pmid - (icpt + 32 * slope)) < 0.1 * abs(slope)
    nu = (c["tau"] - 0.5) / 3.0
    y, x = np.meshgrid(np.arange(24), np.arange(24), indexing="ij")
    r2 = (x - 11.5) ** 2 + (y - 11.5) ** 2
    sel = lum & (r2 < 30.0)
    A = np.stack([np.ones(sel.sum()), r2[sel]], 1)
    (a, mb), *_ = np.linalg.lstsq(A, u[32, :, :, 2][sel], rcond=None)
    assert abs(mb / (slope / (4 * nu)) - 1.0) < 0.02


@pytest.mark.parametrize("precision,tol", [("FP64", 1e-12), ("FP32", 1e-5)])
def test_small_rigid_tube_steady_state_on_the_gpu(oracle_runs, amd, precision, tol):
    c, ref = oracle_runs
    (po, uo), wo = ref[precision == "FP64"]
    s = amd.solver_from_config(c, precision=getattr(amd, precision), wave_cap=STEPS)
    s.step(STEPS)
    s.sync()
    p, u = s.fields()
    w = s.waveforms()
    s.close()
    _steady_checks(c, w, p, u)
    assert np.array_equal(w[:, 0], wo[:, 0])
    curve = []
    for k in range(0, STEPS, 500):
        sl = slice(k, k + 500)
        eq = np.linalg.norm(w[sl, 1] - wo[sl, 1]) / np.linalg.norm(wo[sl, 1])
        ep = np.linalg.norm(w[sl, 2] - wo[sl, 2]) / np.linalg.norm(wo[sl, 2])
        curve.append((k, max(eq, ep)))
    print({"error_vs_step": [(k, f"{e:.1e}") for k, e in curve]}, flush=True)
    assert max(e for _, e in curve) <= tol
    fl = c["flags"] == L.FLUID
    eu = np.linalg.norm(u[fl] - uo[fl]) / np.linalg.norm(uo[fl])
    epf = np.linalg.norm(p[fl] - po[fl]) / np.linalg.norm(po[fl])
    print({"u": f"{eu:.1e}", "p": f"{epf:.1e}"}, flush=True)
    assert eu <= tol and epf <= tol
