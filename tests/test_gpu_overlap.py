"""The wall exchange overlapped with the bulk collide (a second stream; the
band cells collide last; an option, off by default) against the same steps
run in sequence.  The
cells' slot sets are disjoint, so the two orders compute the same values;
they differ only in the order of the spread force's float additions."""
import numpy as np
import pytest

import lbm_inputs as L

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def amd():
    import paper_2112_05258_amd as amd
    amd.lib()
    return amd


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("graph", [True, False])
def test_overlap_matches_sequential_fp64(amd, graph):
    c = L.small_fsi()
    out = []
    for overlap in (False, True):
        s = amd.solver_from_config(c, precision=amd.FP64)
        s.set_graph(graph)
        s.set_overlap(overlap)
        s.step(75)
        s.sync()
        out.append((s.read_populations(), s.waveforms(), s.read_wall()["X"] - c["mesh"]["X0"]))
        s.close()
    e = [_rel(out[1][k], out[0][k]) for k in range(3)]
    print({"pops": f"{e[0]:.1e}", "waves": f"{e[1]:.1e}", "wall": f"{e[2]:.1e}"}, flush=True)
    assert max(e) <= 1e-13


def test_overlap_ensemble_fp32(amd):
    ps = L.ensemble(6, seed=9)
    for p in ps:
        p["L"] = min(p["L"], 40)
    cfgs = [L.ensemble_config(p) for p in ps]
    res = []
    for overlap in (False, True):
        s = amd.solver_from_configs(cfgs, precision=amd.FP32)
        s.set_overlap(overlap)
        s.step(40)
        s.sync()
        res.append([s.fields(k)[1] for k in range(len(cfgs))])
        s.close()
    for k in range(len(cfgs)):
        assert _rel(res[1][k], res[0][k]) <= 1e-6, k
