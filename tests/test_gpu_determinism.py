"""The deterministic spreading mode (lbm_set_deterministic): the wall tiles
are launched colour by colour, so that every cell receives the tiles' exact
fixed-point sums in one order.  Two runs from the same state must then be
bitwise equal -- fields, populations, waveforms, wall positions and forces --
in FP32 and FP64, through the HIP graph and through a band rebuild; the mode
changes only the rounding order of the spread force's float additions, so
it meets the oracle at the usual bars (Eq. EulForce sums the same terms).
Without the mode two such runs differ (measured: populations by up to 7e-12
on the small tube in FP32, 2e-7 on the inflating tube, 1e-10 on cfg2)."""
import numpy as np
import pytest

import lbm_inputs as L
from test_gpu_parity import _compare, rel_l2, wall_bar

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def amd():
    import paper_2112_05258_amd as amd
    amd.lib()
    return amd


def _run(amd, c, precision, steps, band_check=None):
    s = amd.solver_from_config(c, precision=precision)
    s.set_deterministic(True)
    if band_check is not None:
        s.set_band_check(band_check)
    s.step(steps)
    s.sync()
    w = s.read_wall()
    out = dict(pops=s.read_populations(), wave=s.waveforms(), X=w["X"], F=w["F"], slip=w["slip"])
    s.close()
    return out


@pytest.mark.parametrize("precision", ["FP32", "FP64"])
def test_two_runs_are_bitwise_equal(amd, precision):
    c = L.small_fsi()
    a = _run(amd, c, getattr(amd, precision), 120)
    b = _run(amd, c, getattr(amd, precision), 120)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_bitwise_through_a_band_rebuild(amd):
    """The inflating tube moves ~3 lu: the band is rebuilt on the device
    around the moved wall (checked every 16 steps) in both runs."""
    c = L.inflating_tube()
    a = _run(amd, c, amd.FP32, 600, band_check=16)
    b = _run(amd, c, amd.FP32, 600, band_check=16)
    assert np.abs(a["X"] - c["mesh"]["X0"]).max() > 2.0      # the wall did move past the margin
    for k in a:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("precision,tol", [("FP64", 1e-12), ("FP32", 1e-5)])
def test_deterministic_mode_meets_the_oracle(oracle_mod, amd, precision, tol):
    c = L.small_fsi()
    o = oracle_mod.from_config(c, extended=(precision == "FP64"))
    s = amd.solver_from_config(c, precision=getattr(amd, precision))
    s.set_deterministic(True)
    o.step(120)
    s.step(120)
    s.sync()
    _compare(o, s, c["flags"], tol)
    Do, _ = o.displacement()
    X = s.read_wall()["X"]
    e_x = rel_l2(X - c["mesh"]["X0"], Do)
    floor = np.finfo(float).eps * np.linalg.norm(X) / np.linalg.norm(Do)
    assert e_x <= wall_bar(precision, tol, 120) + floor, (e_x, floor)
    s.close()


@pytest.mark.parametrize("precision,nee", [("FP32", 0), ("FP16S", 0), ("FP32", 1)])
def test_stream_orders_agree_bitwise(amd, precision, nee):
    """With deterministic spreading every kernel of a step is deterministic,
    so the step's three orders must give bitwise equal states: the replayed
    graph (0D reductions on the second stream beside the band moments and the
    wall exchange, membrane and 0D-plane tiles there beside the bulk
    collide), the same launches without a graph, and the timed step (every
    launch in sequence on one stream).  A missing wait between the streams
    would show here as a difference.  nee = 1: the normal-neighbour build,
    whose 0D-plane tiles have a launch of their own (on the second stream)."""
    c = dict(L.small_fsi(), nee_variant=nee)
    out = []
    for mode in ("graph", "eager", "sequential"):
        s = amd.solver_from_config(c, precision=getattr(amd, precision))
        s.set_deterministic(True)
        if mode == "eager":
            s.set_graph(False)
        if mode == "sequential":
            s.set_timing(True)
        s.step(150)
        s.sync()
        w = s.read_wall()
        out.append((s.read_populations(), s.waveforms(), w["X"], w["F"]))
        s.close()
    for o in out[1:]:
        for a, b in zip(out[0], o):
            assert np.array_equal(a, b)
