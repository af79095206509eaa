"""The wall-shear-stress diagnostic (lbm_wall_shear_stress) against the
oracle's (same definition, written separately): the small elastic tube after
a run of 240 steps with the LV inlet and Windkessel outlet, every wall
point; FP64 1e-12 (long-double oracle), FP32 1e-5 relative L2, and the two
parities of the AA layout (an even and an odd step count)."""
import numpy as np
import pytest

import lbm_inputs as L

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def amd():
    import paper_2112_05258_amd as amd
    amd.lib()
    return amd


@pytest.mark.parametrize("steps", [240, 241])
@pytest.mark.parametrize("precision,tol", [("FP64", 1e-12), ("FP32", 1e-5)])
def test_wall_shear_stress_matches_oracle(oracle_mod, amd, precision, tol, steps):
    c = L.small_fsi()
    o = oracle_mod.from_config(c, extended=(precision == "FP64"))
    s = amd.solver_from_config(c, precision=getattr(amd, precision))
    o.step(steps)
    s.step(steps)
    s.sync()
    for dist in (2.0, 2.5):
        wo, ws = o.wss(dist), s.wall_shear_stress(dist=dist)
        assert np.isfinite(wo).all() and np.isfinite(ws).all()
        e = np.linalg.norm(ws - wo) / np.linalg.norm(wo)
        print({"precision": precision, "steps": steps, "dist": dist, "rel_l2": f"{e:.1e}",
               "range": [float(wo.min()), float(wo.max())]}, flush=True)
        assert e <= tol
    with pytest.raises(amd.LbmError):
        s.wall_shear_stress(dist=0.0)
    s.close()
