"""The shell model of the wall (the full Eq. structure: in-plane shear with
phi_12 = 1 / (2 (1 + nu)) and mixed bending with gamma_12 = 1, beside the
stretching and bending along the two mesh directions) on the GPU against the
oracle's shell model.

Workload: the small elastic tube (LV inlet, Windkessel outlet, exterior at
P0) whose rest mesh is twisted, ring k turned by kappa z_k about the axis.
The twisted rest shape is not strain free under the shell model
(X_theta . X_z = R kappa != 0), so the shear term drives the wall from the
first step, and the flow and the bending do the rest.  Bars: fields and
waveforms FP64 1e-12 (against the long-double oracle), FP32 1e-5; the wall's
displacement and penalty force sqrt(n) x 1e-12 in FP64 (the order of the
spread force's atomic additions, summed by the displacement recursion) and
1e-5 in FP32."""
import numpy as np
import pytest

import lbm_inputs as L

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def amd():
    import paper_2112_05258_amd as amd
    amd.lib()
    return amd


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def twisted_tube(kappa=0.02, poisson=0.3, shell=1):
    c = L.small_fsi()
    m = dict(c["mesh"])
    X0 = m["X0"].copy()
    cx, cy = (c["nx"] - 1) / 2.0, (c["ny"] - 1) / 2.0
    a = kappa * (X0[:, 2] - X0[:, 2].min())
    x, y = X0[:, 0] - cx, X0[:, 1] - cy
    X0[:, 0] = cx + np.cos(a) * x - np.sin(a) * y
    X0[:, 1] = cy + np.sin(a) * x + np.cos(a) * y
    m["X0"] = X0
    c.update(mesh=m, shell=shell, poisson=poisson, name="small_fsi_twisted")
    return c


@pytest.mark.parametrize("precision,tol", [("FP64", 1e-12), ("FP32", 1e-5)])
def test_shell_model_small_twisted_tube(oracle_mod, amd, precision, tol):
    n = 120
    c = twisted_tube()
    o = oracle_mod.from_config(c, extended=(precision == "FP64"))
    s = amd.solver_from_config(c, precision=getattr(amd, precision))
    o.step(n)
    s.step(n)
    s.sync()
    fl = c["flags"] == L.FLUID
    po, uo = o.fields()
    ps, us = s.fields()
    wo, ws = o.waveforms(), s.waveforms()
    Do, _ = o.displacement()
    lo, ls = o.lagrangian(), s.read_wall()
    X0 = c["mesh"]["X0"]
    e = {"u": rel(us[fl], uo[fl]), "p": rel(ps[fl], po[fl]), "wave": rel(ws[:, 1:5], wo[:, 1:5])}
    w = {"wall_X": rel(ls["X"] - X0, Do), "wall_F": rel(ls["F"], lo["F"])}
    print({k: f"{v:.2e}" for k, v in {**e, **w}.items()}, flush=True)
    for k, v in e.items():
        assert v <= tol, (k, v)
    wall_bar = tol * np.sqrt(n) if precision == "FP64" else tol
    for k, v in w.items():
        assert v <= wall_bar, (k, v)
    # the shell terms matter here: without them the oracle's wall moves
    # differently by far more than the bar
    o2 = oracle_mod.from_config(twisted_tube(shell=0), extended=False)
    o2.step(n)
    D2, _ = o2.displacement()
    moved = rel(D2, Do)
    print({"shell_vs_plain": f"{moved:.2e}"}, flush=True)
    assert moved > 1e3 * wall_bar
    s.close()


def test_shell_inputs_rejected(amd):
    for bad in (dict(shell=2), dict(shell=1, poisson=-1.0), dict(shell=1, poisson=float("nan"))):
        c = dict(twisted_tube(), **bad)
        with pytest.raises(amd.LbmError):
            amd.solver_from_config(c, precision=amd.FP32)
