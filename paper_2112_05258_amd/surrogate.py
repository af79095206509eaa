"""Learned surrogate of the coupled solver (binding of include/lbm_surrogate.h).

The network maps the 7 parameters (Emax, Emin, HR, Z, C, R, k) of the
LV-elastance inlet, the Windkessel outlet and the wall to one beat of inlet
pressure and inlet flow at 256 phases each.  Its forward and backward passes
and the Adam update run in the library's kernels (BF16 matrix cores, FP32
master weights); this module marshals arguments and drives the loops.

Training data come from the batched solver: for each parameter vector an
elastic tube of fixed geometry is run for three beats and the third beat is
sampled.  The solver is the judge of the network's error and the fallback
for parameters outside the training box (predict_or_solve).

Command line:
    python -m paper_2112_05258_amd.surrogate data  --n 4096 --seed 11 --out F.npz
    python -m paper_2112_05258_amd.surrogate train --data F.npz --test T.npz --weights W.npz
"""
from __future__ import annotations

import argparse
import ctypes as C
import math
import sys
import time

import numpy as np

from . import LbmError, SurConfig, lib, solver_from_configs, FP32

N_PHASE = 256


def _chk(L, ctx, st):
    if st != 0:
        raise LbmError(st, (L.lbm_sur_last_error(ctx) or b"").decode())


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class Surrogate:
    """MLP n_in -> [width, GELU] x n_hidden -> n_out on the current GPU."""

    def __init__(self, n_in=7, width=512, n_hidden=4, n_out=2 * N_PHASE, max_batch=65536, train_batch=256,
                 device="cuda:0"):
        import torch
        self.torch = torch
        self.L = lib()
        self.device = torch.device(device)
        self.cfg = SurConfig(n_in, width, n_hidden, n_out, max_batch, train_batch)
        self.n_params = int(self.L.lbm_sur_num_params(C.byref(self.cfg)))
        if self.n_params < 0:
            raise LbmError(-1, "unsupported network configuration")
        nb = C.c_size_t()
        _chk(self.L, None, self.L.lbm_sur_query_sizes(C.byref(self.cfg), C.byref(nb)))
        self.mem = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        off = (-self.mem.data_ptr()) % 256
        self.stream = torch.cuda.Stream(device=self.device)
        self.ctx = C.c_void_p()
        with torch.cuda.device(self.device):
            _chk(self.L, None, self.L.lbm_sur_init(C.byref(self.cfg), C.c_void_p(self.mem.data_ptr() + off),
                                                   nb.value, C.c_void_p(self.stream.cuda_stream),
                                                   C.byref(self.ctx)))
        self.box = None

    # ---- parameters and scaling ------------------------------------------
    def set_params(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        _chk(self.L, self.ctx, self.L.lbm_sur_set_params(self.ctx, th.ctypes.data_as(C.POINTER(C.c_double)),
                                                         th.size))

    def params(self):
        th = np.empty(self.n_params)
        _chk(self.L, self.ctx, self.L.lbm_sur_get_params(self.ctx, th.ctypes.data_as(C.POINTER(C.c_double)),
                                                         th.size))
        return th

    def set_scaling(self, lo, hi, mu, sigma):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (lo, hi, mu, sigma)]
        _chk(self.L, self.ctx, self.L.lbm_sur_set_scaling(self.ctx, *[a.ctypes.data_as(C.POINTER(C.c_double))
                                                                       for a in arrs]))
        self.box = (arrs[0].copy(), arrs[1].copy())
        self.mu, self.sigma = arrs[2].copy(), arrs[3].copy()

    def _dev(self, a, dtype=None):
        t = self.torch
        if isinstance(a, t.Tensor):
            a = a.to(self.device)
        else:
            a = t.as_tensor(np.ascontiguousarray(a), device=self.device)
        return a.to(dtype or t.float32).contiguous()

    # ---- passes ------------------------------------------------------------
    def grad(self, x, t, idx=None):
        """(gradient as a device FP32 tensor, loss) on one batch."""
        x, t = self._dev(x), self._dev(t)
        ix = self._dev(idx, self.torch.int32) if idx is not None else None
        m = ix.numel() if ix is not None else x.shape[0]
        g = self.torch.empty(self.n_params, dtype=self.torch.float32, device=self.device)
        loss = C.c_double()
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        _chk(self.L, self.ctx, self.L.lbm_sur_grad(self.ctx, _ptr(x), _ptr(t), x.shape[0], _ptr(ix), m, _ptr(g),
                                                   C.byref(loss)))
        return g, loss.value

    def train_step(self, x, t, idx, lr, b1=0.9, b2=0.999, eps=1e-8, want_loss=False):
        loss = C.c_double()
        _chk(self.L, self.ctx, self.L.lbm_sur_train_step(self.ctx, _ptr(x), _ptr(t), x.shape[0], _ptr(idx),
                                                         idx.numel() if idx is not None else x.shape[0],
                                                         lr, b1, b2, eps, C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def predict(self, x):
        """Physical outputs (device tensor m x n_out) for rows of x."""
        x = self._dev(x)
        m = x.shape[0]
        y = self.torch.empty((m, self.cfg.n_out), dtype=self.torch.float32, device=self.device)
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        for r0 in range(0, m, self.cfg.max_batch):
            r1 = min(m, r0 + self.cfg.max_batch)
            _chk(self.L, self.ctx, self.L.lbm_sur_predict(self.ctx, C.c_void_p(x[r0:].data_ptr()), r1 - r0,
                                                          C.c_void_p(y[r0:].data_ptr())))
        self.sync()
        return y

    def predict_into(self, x, y):
        """Enqueue inference of device rows x (m <= max_batch) into device y
        on the context's stream, without waiting."""
        _chk(self.L, self.ctx, self.L.lbm_sur_predict(self.ctx, _ptr(x), x.shape[0], _ptr(y)))

    def sync(self):
        _chk(self.L, self.ctx, self.L.lbm_sur_sync(self.ctx))

    def set_timing(self, on):
        _chk(self.L, self.ctx, self.L.lbm_sur_set_timing(self.ctx, 1 if on else 0))

    def gemm_time(self):
        """(launches, total ms, FLOP) of the matrix products since set_timing."""
        n, ms, fl = C.c_int64(), C.c_double(), C.c_double()
        _chk(self.L, self.ctx, self.L.lbm_sur_gemm_time(self.ctx, C.byref(n), C.byref(ms), C.byref(fl)))
        return n.value, ms.value, fl.value

    # ---- training loop -----------------------------------------------------
    def fit(self, X, T, epochs=2000, batch=None, lr=1e-3, lr_min=1e-5, seed=0, log=None, log_every=200):
        """Adam over shuffled mini-batches with a cosine learning-rate decay.
        Input box and output standardisation come from the training set."""
        torch = self.torch
        X = np.asarray(X, np.float64)
        T = np.asarray(T, np.float64)
        lo, hi = X.min(axis=0), X.max(axis=0)
        mu, sd = T.mean(axis=0), T.std(axis=0)
        sd = np.maximum(sd, 1e-6 * np.abs(T).max())
        if self.box is None:
            self.set_scaling(lo, hi, mu, sd)
        xd, td = self._dev(X), self._dev(T)
        n = X.shape[0]
        b = batch or self.cfg.train_batch
        rng = np.random.default_rng(seed)
        per_epoch = n // b
        total = epochs * per_epoch
        hist = []
        k = 0
        # every epoch's shuffle uploaded once, before the library's stream
        # starts reading them
        perms = self._dev(np.stack([rng.permutation(n)[:per_epoch * b] for _ in range(epochs)]).astype(np.int32),
                          torch.int32)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        for ep in range(epochs):
            perm = perms[ep]
            for s in range(per_epoch):
                rate = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * k / total))
                want = (k % log_every == 0) or k == total - 1
                loss = self.train_step(xd, td, perm[s * b:(s + 1) * b], rate, want_loss=want)
                if want:
                    hist.append((k, loss))
                    if log:
                        log(f"step {k}/{total} lr {rate:.2e} loss {loss:.4e}")
                k += 1
        self.sync()
        return hist

    def save(self, path):
        np.savez_compressed(path, theta=self.params().astype(np.float32), lo=self.box[0], hi=self.box[1],
                            mu=self.mu, sigma=self.sigma,
                            shape=np.array([self.cfg.n_in, self.cfg.width, self.cfg.n_hidden, self.cfg.n_out]))

    @classmethod
    def load(cls, path, max_batch=65536, train_batch=256, device="cuda:0"):
        d = np.load(path)
        n_in, width, n_hidden, n_out = (int(v) for v in d["shape"])
        s = cls(n_in, width, n_hidden, n_out, max_batch=max_batch, train_batch=train_batch, device=device)
        s.set_params(d["theta"].astype(np.float64))
        s.set_scaling(d["lo"], d["hi"], d["mu"], d["sigma"])
        return s

    def inside(self, X):
        lo, hi = self.box
        X = np.asarray(X, np.float64)
        return np.all((X >= lo) & (X <= hi), axis=1)

    def predict_or_solve(self, X, log=None):
        """Outputs for every row of X: the network inside its training box,
        the solver (three beats of the batched tube model) outside it.
        Returns (outputs, mask of rows the solver produced)."""
        X = np.asarray(X, np.float64)
        out = np.empty((X.shape[0], self.cfg.n_out))
        ins = self.inside(X)
        if ins.any():
            out[ins] = self.predict(X[ins]).cpu().numpy()
        if (~ins).any():
            out[~ins] = lb_waveforms(X[~ins], log=log)
        return out, ~ins

    def close(self):
        if self.ctx:
            self.L.lbm_sur_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------
# training data from the batched solver
# ----------------------------------------------------------------------------

def phase_sample(w, beat, n_phase=N_PHASE, sc=None):
    """Inlet pressure (mmHg) and flow (ml/s) of the third beat at n_phase
    phases from the beat start, linearly interpolated in the per-step record
    w (columns: step, Q_in, P_in, ...)."""
    t = 2.0 * beat + beat * np.arange(n_phase) / n_phase
    P = np.interp(t, w[:, 0], w[:, 2])
    Q = np.interp(t, w[:, 0], w[:, 1])
    if sc is not None:
        P = P / sc["sigma_P"]
        Q = Q * sc["sigma_t"] / sc["sigma_V"]
    return np.concatenate([P, Q])


def lb_waveforms(X, batch=512, precision=FP32, log=None):
    """Solver outputs (pressure then flow phases, physical units) for each
    parameter vector in X, run in batches of instances on the GPU."""
    import lbm_inputs as L
    X = np.asarray(X, np.float64)
    out = np.empty((X.shape[0], 2 * N_PHASE))
    for b0 in range(0, X.shape[0], batch):
        cfgs = [L.surrogate_config(p) for p in X[b0:b0 + batch]]
        steps = max(c["steps"] for c in cfgs)
        t0 = time.time()
        if log:
            log(f"  instances {b0}..{b0 + len(cfgs) - 1}: setting up")
        s = solver_from_configs(cfgs, precision=precision, wave_cap=steps)
        done = 0
        while done < steps:
            k = min(1000, steps - done)
            s.step(k)
            done += k
            s.sync()
            if log:
                log(f"  instances {b0}..{b0 + len(cfgs) - 1}: step {done}/{steps} ({time.time() - t0:.1f} s)")
        for k, c in enumerate(cfgs):
            out[b0 + k] = phase_sample(s.waveforms(k), c["beat"], sc=c["scales"])
        s.close()
    return out


def rel_errors(Y, Yref, p0_mmHg=80.0):
    """Per-sample relative L2 errors of the pressure pulse (P - P0) and of
    the flow waveform."""
    n = Y.shape[1] // 2
    dP = np.linalg.norm(Y[:, :n] - Yref[:, :n], axis=1) / np.linalg.norm(Yref[:, :n] - p0_mmHg, axis=1)
    dQ = np.linalg.norm(Y[:, n:] - Yref[:, n:], axis=1) / np.linalg.norm(Yref[:, n:], axis=1)
    return dP, dQ


def _main(argv=None):
    import lbm_inputs as L
    ap = argparse.ArgumentParser(prog="python -m paper_2112_05258_amd.surrogate")
    sub = ap.add_subparsers(dest="cmd", required=True)
    d = sub.add_parser("data", help="solver runs for n parameter draws")
    d.add_argument("--n", type=int, default=4096)
    d.add_argument("--seed", type=int, default=11)
    d.add_argument("--batch", type=int, default=512)
    d.add_argument("--out", required=True)
    t = sub.add_parser("train", help="train on a data file, evaluate on another, save the weights")
    t.add_argument("--data", required=True)
    t.add_argument("--test", required=True)
    t.add_argument("--weights", required=True)
    t.add_argument("--epochs", type=int, default=1500)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--batch", type=int, default=256)
    t.add_argument("--seed", type=int, default=0)
    a = ap.parse_args(argv)

    def log(m):
        print(m, flush=True)

    if a.cmd == "data":
        X = L.surrogate_params(a.n, a.seed)
        t0 = time.time()
        Y = lb_waveforms(X, batch=a.batch, log=log)
        np.savez_compressed(a.out, X=X, Y=Y)
        log(f"wrote {a.out}: {a.n} runs in {time.time() - t0:.1f} s, finite {bool(np.isfinite(Y).all())}")
    else:
        D, E = np.load(a.data), np.load(a.test)
        s = Surrogate(train_batch=a.batch)
        s.set_params(L.mlp_init([7] + [512] * 4 + [512], seed=a.seed))
        # the training box is the sampling box of the parameter draws
        Yd = np.asarray(D["Y"], np.float64)
        s.set_scaling(L.SURROGATE_LO, L.SURROGATE_HI, Yd.mean(axis=0),
                      np.maximum(Yd.std(axis=0), 1e-6 * np.abs(Yd).max()))
        t0 = time.time()
        s.fit(D["X"], D["Y"], epochs=a.epochs, lr=a.lr, seed=a.seed, log=log, log_every=2000)
        log(f"trained in {time.time() - t0:.1f} s")
        s.save(a.weights)
        Yp = s.predict(E["X"]).cpu().numpy()
        dP, dQ = rel_errors(Yp, E["Y"])
        log(f"held-out {len(dP)}: pressure pulse rel-L2 mean {dP.mean():.4f} max {dP.max():.4f}; "
            f"flow rel-L2 mean {dQ.mean():.4f} max {dQ.max():.4f}")
        Yt = s.predict(D["X"]).cpu().numpy()
        tP, tQ = rel_errors(Yt, D["Y"])
        log(f"training set: pressure {tP.mean():.4f}, flow {tQ.mean():.4f}")
    return 0


if __name__ == "__main__":
    sys.exit(_main())
