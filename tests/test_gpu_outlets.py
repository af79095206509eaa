"""Several outlets, each with its own 3-element Windkessel (Sec. 2.1.2), on
the GPU against the oracle: the rigid branched duct of
lbm_inputs.branched_duct (one inlet, a septum splitting the duct into two
branches, outlet 0 and outlet 1 with different distal resistances), with
the pressure-in / flux-out and the flux-in / pressure-out couplings, and a
batch of two ducts of different sizes whose outlets all differ.  Fields,
the main waveform record and every outlet's flux, pressure and Windkessel
pressure; bars FP64 1e-12 (against the long-double oracle), FP32 1e-5."""
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


def _duct(mode, nx=14, ny=10, nz=40):
    if mode == 1:
        c = L.branched_duct(nx=nx, ny=ny, nz=nz, Rd=(0.6, 1.8), Rp=0.05, C=50.0)
    else:
        c = L.branched_duct(nx=nx, ny=ny, nz=nz, Rd=(0.15, 0.45), Rp=0.005, C=300.0)
        c["outlets"] = [(L.BC_WINDKESSEL3, [0.005, 300.0, r, 0.0], [c["p_init"]]) for r in (0.15, 0.45)]
    return c


def _compare(o, s, c, tol, inst=0):
    po, uo = o.fields()
    ps, us = s.fields(inst)
    fl = c["flags"] == L.FLUID
    wo, ws = o.waveforms(), s.waveforms(inst)
    oo, os_ = o.outlet_waveforms(), s.outlet_waveforms(inst)
    assert ws.shape == wo.shape and os_.shape == oo.shape
    e = {"u": rel(us[fl], uo[fl]), "p": rel(ps[fl], po[fl]),
         "wave": rel(ws[:, 1:5], wo[:, 1:5]),
         "outlet_Q": rel(os_[:, :2, 0], oo[:, :2, 0]), "outlet_p": rel(os_[:, :2, 1], oo[:, :2, 1]),
         "outlet_Pw": rel(os_[:, :2, 2], oo[:, :2, 2])}
    print({k: f"{v:.1e}" for k, v in e.items()}, flush=True)
    assert np.all(os_[:, 2:, :] == 0.0)
    for k, v in e.items():
        assert v <= tol, (k, v)


@pytest.mark.parametrize("mode", [1, 0])
@pytest.mark.parametrize("precision,tol", [("FP64", 1e-12), ("FP32", 1e-5)])
def test_branched_duct_two_windkessels(oracle_mod, amd, mode, precision, tol):
    c = _duct(mode)
    o = oracle_mod.from_config(c, extended=(precision == "FP64"))
    s = amd.solver_from_config(c, precision=getattr(amd, precision))
    o.step(401)
    s.step(401)
    s.sync()
    _compare(o, s, c, tol)
    # the branch with the lower distal resistance draws more
    q = s.outlet_waveforms()[-1, :2, 0]
    assert q[0] > q[1] > 0
    s.close()


def test_batched_ducts_keep_their_own_outlets(oracle_mod, amd):
    cs = [_duct(1), _duct(0, nx=18, ny=12, nz=36)]
    s = amd.solver_from_configs(cs, precision=amd.FP64)
    s.step(300)
    s.sync()
    for k, c in enumerate(cs):
        o = oracle_mod.from_config(c, extended=True)
        o.step(300)
        _compare(o, s, c, 1e-12, inst=k)
    s.close()


def test_outlet_index_only_on_outlet_ghosts(amd):
    c = _duct(1)
    bad = c["flags"].copy()
    bad[0][bad[0] == L.INLET] = L.INLET | (1 << 5)     # an index on an INLET ghost
    with pytest.raises(amd.LbmError):
        amd.solver_from_config(dict(c, flags=bad), precision=amd.FP32)
    with pytest.raises(amd.LbmError):                   # boundary ids stop at 2 + 7
        amd.solver_from_config(dict(c, outlets=[(L.BC_PRESSURE_CONST, [0.0], [])] * 9), precision=amd.FP32)
