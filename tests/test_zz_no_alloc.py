"""The allocation-free inference entry point (lbm_sur_predict_static) against
lbm_sur_predict of a context holding the same network, through the C
interface: two calls in a row, the second with fewer rows, each equal bit
for bit (same kernel, same FP32 values, same fragment-order BF16 weights).
The network is the trained surrogate; the inputs are seeded draws from its
parameter box.  Also: the shapes the fused kernel does not take and a row
count past the limit are refused without a launch."""
import ctypes as C
import os

import numpy as np
import pytest

import lbm_inputs as L

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sur():
    import torch
    from paper_2112_05258_amd import surrogate as S
    s = S.Surrogate.load(os.path.join(ROOT, "paper_2112_05258_amd", "surrogate_weights.npz"), max_batch=4096)
    d = np.load(os.path.join(ROOT, "paper_2112_05258_amd", "surrogate_weights.npz"))
    dev = torch.device("cuda:0")
    f32 = lambda a: torch.as_tensor(np.asarray(a, np.float64), device=dev).to(torch.float32).contiguous()
    arrs = dict(theta=f32(d["theta"]), lo=f32(d["lo"]), hi=f32(d["hi"]), mu=f32(d["mu"]), sigma=f32(d["sigma"]))
    yield s, arrs
    s.close()


def _static(s, arrs, x, y, m=None):
    import torch
    p = lambda t: C.c_void_p(t.data_ptr())
    cfg = s.cfg
    st = s.L.lbm_sur_predict_static(C.byref(cfg), p(arrs["theta"]), p(arrs["lo"]), p(arrs["hi"]), p(arrs["mu"]),
                                    p(arrs["sigma"]), p(x), x.shape[0] if m is None else m, p(y),
                                    C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


def test_static_inference_matches_the_context_call(sur):
    import torch
    s, arrs = sur
    for m, seed in ((3000, 5), (77, 6)):       # second call smaller than the first
        print("rows", m, flush=True)
        x = s._dev(L.surrogate_params(m, seed=seed))
        want = s.predict(x).cpu().numpy()
        y = torch.full((m, s.cfg.n_out), float("nan"), dtype=torch.float32, device="cuda:0")
        assert _static(s, arrs, x, y) == 0
        torch.cuda.synchronize()
        got = y.cpu().numpy()
        assert np.isfinite(got).all()
        assert np.array_equal(got, want), np.abs(got - want).max()


def test_static_inference_refusals(sur):
    import torch
    from paper_2112_05258_amd import SurConfig
    s, arrs = sur
    x = s._dev(L.surrogate_params(8, seed=1))
    y = torch.zeros((8, s.cfg.n_out), dtype=torch.float32, device="cuda:0")
    assert _static(s, arrs, x, y, m=(1 << 22) + 1) == -1
    assert _static(s, arrs, x, y, m=-1) == -1
    assert _static(s, arrs, x, y, m=0) == 0
    narrow = SurConfig(7, 256, 4, 512, 64, 256)
    st = s.L.lbm_sur_predict_static(C.byref(narrow), *[C.c_void_p(arrs[k].data_ptr()) for k in
                                                       ("theta", "lo", "hi", "mu", "sigma")],
                                    C.c_void_p(x.data_ptr()), 8, C.c_void_p(y.data_ptr()), None)
    assert st == -1
    assert b"width 512" in s.L.lbm_sur_last_error(None)
    torch.cuda.synchronize()
    assert float(y.abs().sum()) == 0.0         # nothing was launched
