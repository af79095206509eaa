"""MI355X-native 0D-3D coupled lattice Boltzmann / immersed-boundary solver.

Python binding of ``liblbm0d3d.so`` (C interface in ``include/lbm0d3d.h``).
This module only marshals arguments: every step of the method runs in the
library's HIP kernels.  torch supplies device memory and the stream.  There
is no CPU fallback: if the library is missing, importing ``lib()`` raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm0d3d.so")
NQ = 19
NREC = 14
NOUT = 8          # outlets per instance (index in bits 5-7 of an OUTLET ghost's cell type)
FP64, FP32, FP16S, BF16S = 0, 1, 2, 3
KERNEL_COLLIDE, KERNEL_REDUCE, KERNEL_BAND, KERNEL_WALL = 0, 1, 2, 3

STATUS = {0: "OK", -1: "E_INVAL", -2: "E_DEVICE", -3: "E_UNSTABLE", -4: "E_STATE",
          -5: "E_UNSUPPORTED", -6: "E_BAND"}


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("tau", C.c_double),
                ("precision", C.c_int32), ("store_scale", C.c_double),
                ("flags", C.POINTER(C.c_uint8)), ("wave_cap", C.c_int32), ("p_ref", C.c_double),
                ("nee_variant", C.c_int32)]


class Buffers(C.Structure):
    _fields_ = [("pop", C.c_void_p), ("pop_bytes", C.c_size_t),
                ("work", C.c_void_p), ("work_bytes", C.c_size_t)]


class WallDesc(C.Structure):
    _fields_ = [("n_theta", C.c_int32), ("n_z", C.c_int32), ("X0_host", C.POINTER(C.c_double)),
                ("ds_theta", C.c_double), ("ds_z", C.c_double), ("area", C.c_double),
                ("k_stretch", C.c_double), ("ei_bend", C.c_double), ("mass", C.c_double),
                ("alpha", C.c_double), ("beta", C.c_double), ("band_margin", C.c_int32),
                ("kernel", C.c_int32), ("mode", C.c_int32), ("shell", C.c_int32), ("poisson", C.c_double)]


class Launch(C.Structure):
    _fields_ = [("block", C.c_int32), ("cells_per_lane", C.c_int32), ("wall_tile_theta", C.c_int32),
                ("wall_tile_z", C.c_int32)]


SYMBOLS = {
    "lbm_query_sizes": (C.c_int, [C.POINTER(Config), C.c_int32, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "lbm_init": (C.c_int, [C.POINTER(Config), C.c_int32, C.POINTER(Buffers), C.c_void_p, C.POINTER(C.c_void_p)]),
    "lbm_step": (C.c_int, [C.c_void_p, C.c_int64]),
    "lbm_couple_0d": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_double), C.c_int32,
                                C.POINTER(C.c_double), C.c_int32]),
    "lbm_get_0d": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_double)]),
    "lbm_fsi_query_sizes": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(WallDesc), C.POINTER(C.c_size_t)]),
    "lbm_fsi_exchange": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(WallDesc), C.c_void_p, C.c_size_t]),
    "lbm_read_wall": (C.c_int, [C.c_void_p, C.c_int32] + [C.POINTER(C.c_double)] * 5),
    "lbm_set_wall": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "lbm_wall_shear_stress": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.POINTER(C.c_double)]),
    "lbm_write_populations": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double)]),
    "lbm_set_rest": (C.c_int, [C.c_void_p, C.c_int32, C.c_double]),
    "lbm_read_populations": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double)]),
    "lbm_read_fields": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "lbm_read_waveforms": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.c_int64,
                                     C.POINTER(C.c_int64)]),
    "lbm_read_outlet_waveforms": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.c_int64,
                                            C.POINTER(C.c_int64)]),
    "lbm_sync": (C.c_int, [C.c_void_p]),
    "lbm_instance_status": (C.c_int, [C.c_void_p, C.c_int32]),
    "lbm_steps": (C.c_int64, [C.c_void_p]),
    "lbm_set_timing": (C.c_int, [C.c_void_p, C.c_int32]),
    "lbm_kernel_time": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
    "lbm_set_graph": (C.c_int, [C.c_void_p, C.c_int32]),
    "lbm_set_overlap": (C.c_int, [C.c_void_p, C.c_int32]),
    "lbm_set_deterministic": (C.c_int, [C.c_void_p, C.c_int32]),
    "lbm_debug_slot_writes": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_uint32)]),
    "lbm_set_band_check": (C.c_int, [C.c_void_p, C.c_int32]),
    "lbm_num_classes": (C.c_int32, [C.c_void_p]),
    "lbm_class_info": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                 C.POINTER(C.c_int64)]),
    "lbm_get_launch": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Launch)]),
    "lbm_set_launch": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Launch)]),
    "lbm_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64)]),
    "lbm_save": (C.c_int, [C.c_void_p, C.c_char_p]),
    "lbm_load": (C.c_int, [C.c_void_p, C.c_char_p]),
    "lbm_last_error": (C.c_char_p, [C.c_void_p]),
    "lbm_destroy": (None, [C.c_void_p]),
    "lbm_num_cells": (C.c_int64, [C.c_void_p, C.c_int32]),
    "lbm_bytes_per_population": (C.c_int32, [C.c_void_p]),
}



class SurConfig(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("width", C.c_int32), ("n_hidden", C.c_int32), ("n_out", C.c_int32),
                ("max_batch", C.c_int32), ("train_batch", C.c_int32)]


# learned surrogate (include/lbm_surrogate.h)
SUR_SYMBOLS = {
    "lbm_sur_num_params": (C.c_int64, [C.POINTER(SurConfig)]),
    "lbm_sur_query_sizes": (C.c_int, [C.POINTER(SurConfig), C.POINTER(C.c_size_t)]),
    "lbm_sur_init": (C.c_int, [C.POINTER(SurConfig), C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]),
    "lbm_sur_set_params": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_int64]),
    "lbm_sur_get_params": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_int64]),
    "lbm_sur_set_scaling": (C.c_int, [C.c_void_p] + [C.POINTER(C.c_double)] * 4),
    "lbm_sur_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p,
                               C.POINTER(C.c_double)]),
    "lbm_sur_train_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32,
                                     C.c_double, C.c_double, C.c_double, C.c_double, C.POINTER(C.c_double)]),
    "lbm_sur_predict": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "lbm_sur_predict_static": (C.c_int, [C.POINTER(SurConfig)] + [C.c_void_p] * 6 + [C.c_int32, C.c_void_p,
                                                                                    C.c_void_p]),
    "lbm_sur_set_timing": (C.c_int, [C.c_void_p, C.c_int32]),
    "lbm_sur_gemm_time": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                    C.POINTER(C.c_double)]),
    "lbm_sur_sync": (C.c_int, [C.c_void_p]),
    "lbm_sur_last_error": (C.c_char_p, [C.c_void_p]),
    "lbm_sur_destroy": (C.c_int, [C.c_void_p]),
}

class AxiConfig(C.Structure):
    _fields_ = [("nx", C.c_int32), ("nr", C.c_int32), ("tau", C.c_double), ("precision", C.c_int32),
                ("flags", C.POINTER(C.c_uint8)), ("periodic_x", C.c_int32), ("wave_cap", C.c_int32),
                ("p_ref", C.c_double)]


# axisymmetric solver (include/lbm_axi.h)
AXI_SYMBOLS = {
    "lbm_axi_query_size": (C.c_int, [C.POINTER(AxiConfig), C.POINTER(C.c_size_t)]),
    "lbm_axi_init": (C.c_int, [C.POINTER(AxiConfig), C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]),
    "lbm_axi_couple_0d": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_double), C.c_int32,
                                    C.POINTER(C.c_double), C.c_int32]),
    "lbm_axi_set_body_force": (C.c_int, [C.c_void_p, C.c_double, C.c_double]),
    "lbm_axi_set_rest": (C.c_int, [C.c_void_p, C.c_double]),
    "lbm_axi_write_populations": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "lbm_axi_read_populations": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "lbm_axi_step": (C.c_int, [C.c_void_p, C.c_int64]),
    "lbm_axi_read_fields": (C.c_int, [C.c_void_p] + [C.POINTER(C.c_double)] * 3),
    "lbm_axi_read_waveforms": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_int64, C.POINTER(C.c_int64)]),
    "lbm_axi_sync": (C.c_int, [C.c_void_p]),
    "lbm_axi_last_error": (C.c_char_p, [C.c_void_p]),
    "lbm_axi_destroy": (C.c_int, [C.c_void_p]),
}

_lib = None


def lib():
    """Load liblbm0d3d.so (built by paper_2112_05258_amd.build); raise if absent."""
    global _lib
    if _lib is None:
        # torch first: its bundled HIP runtime must be the one the library
        # binds to (same SONAME), so that one runtime owns the device, the
        # torch-allocated buffers and the streams.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run python -m paper_2112_05258_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in list(SYMBOLS.items()) + list(SUR_SYMBOLS.items()) + list(AXI_SYMBOLS.items()):
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


class Solver:
    """One context over one or more lattice instances on the current GPU.

    boxes: list of dicts with nx, ny, nz, tau, flags (uint8 (nz, ny, nx)).
    """

    def __init__(self, boxes, precision=FP32, store_scale=0.0, wave_cap=4096, device="cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        if isinstance(boxes, dict):
            boxes = [boxes]
        self.boxes = boxes
        self.n = len(boxes)
        self._flags = [np.ascontiguousarray(b["flags"], dtype=np.uint8) for b in boxes]
        cfgs = (Config * self.n)()
        for k, b in enumerate(boxes):
            cfgs[k] = Config(b["nx"], b["ny"], b["nz"], float(b["tau"]), precision, float(store_scale),
                             self._flags[k].ctypes.data_as(C.POINTER(C.c_uint8)), wave_cap,
                             float(b.get("p_ref", 0.0)), int(b.get("nee_variant", 0)))
        self._cfgs = cfgs
        pb, wb = C.c_size_t(), C.c_size_t()
        self._check(lib().lbm_query_sizes(cfgs, self.n, C.byref(pb), C.byref(wb)), None)
        self.pop = torch.empty(pb.value, dtype=torch.uint8, device=self.device)
        self.work = torch.empty(wb.value, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.Stream(device=self.device)
        buf = Buffers(self.pop.data_ptr(), pb.value, self.work.data_ptr(), wb.value)
        h = C.c_void_p()
        self._check(lib().lbm_init(cfgs, self.n, C.byref(buf), C.c_void_p(self.stream.cuda_stream), C.byref(h)), None)
        self.h = h
        self.fsi = {}
        self.precision = precision

    # ------------------------------------------------------------------
    def _check(self, code, h="self"):
        if code != 0:
            hh = self.h if h == "self" else h
            msg = lib().lbm_last_error(hh).decode()
            raise LbmError(code, msg)

    def close(self):
        if getattr(self, "h", None):
            lib().lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------
    def step(self, n=1):
        self._check(lib().lbm_step(self.h, int(n)))

    @property
    def t(self):
        return lib().lbm_steps(self.h)

    def sync(self):
        self._check(lib().lbm_sync(self.h))

    def instance_status(self, inst):
        """0 while instance inst runs, else the lbm_status it failed with
        (it is then frozen)."""
        code = lib().lbm_instance_status(self.h, int(inst))
        if code == -1:
            self._check(code)
        return code

    def failed(self):
        """Indices of the instances that have failed and been frozen."""
        return [k for k in range(self.n) if self.instance_status(k) != 0]

    def save(self, path):
        """Checkpoint of the whole state to a file (lbm_save)."""
        self._check(lib().lbm_save(self.h, os.fsencode(path)))

    def load(self, path):
        """Restore a checkpoint into this solver, built like the saved one
        (lbm_load)."""
        self._check(lib().lbm_load(self.h, os.fsencode(path)))

    def couple_0d(self, inst, boundary, kind, params, state=()):
        p = np.ascontiguousarray(params, dtype=np.float64)
        s = np.ascontiguousarray(state, dtype=np.float64) if len(state) else None
        self._check(lib().lbm_couple_0d(self.h, inst, boundary, kind, _dp(p), len(p), _dp(s),
                                        0 if s is None else len(s)))

    def get_0d(self, inst, boundary):
        out = np.zeros(8)
        self._check(lib().lbm_get_0d(self.h, inst, boundary, _dp(out)))
        return dict(vmode=int(out[0]), pstar=out[1], S=out[2], Pv=out[3], Pw=out[4],
                    open=int(out[5]), Td=int(out[6]), vz=out[7])

    def _wall_desc(self, mesh, k, ei, mass, alpha, beta, margin, kernel=0, mode=0, shell=0, poisson=0.5):
        X0 = np.ascontiguousarray(mesh["X0"], dtype=np.float64).reshape(-1)
        d = WallDesc(mesh["n_theta"], mesh["n_z"], _dp(X0), mesh["ds_theta"], mesh["ds_z"], mesh["area"],
                     k, ei, mass, alpha, beta, margin, kernel, mode, int(shell), float(poisson))
        return d, X0

    def fsi_exchange(self, inst, mesh, k, ei, mass, alpha, beta, margin=2, kernel=0, mode=0,
                     shell=0, poisson=0.5):
        """Attach the wall of instance inst: kernel 0 Peskin 4-point / 1
        cosine; mode 0 built-in membrane / 1 external solid (set_wall);
        shell 1 adds the off-diagonal terms of the wall model (Poisson's
        ratio poisson)."""
        d, X0 = self._wall_desc(mesh, k, ei, mass, alpha, beta, margin, kernel, mode, shell, poisson)
        nb = C.c_size_t()
        self._check(lib().lbm_fsi_query_sizes(self.h, inst, C.byref(d), C.byref(nb)))
        buf = self.torch.empty(nb.value, dtype=self.torch.uint8, device=self.device)
        self._check(lib().lbm_fsi_exchange(self.h, inst, C.byref(d), C.c_void_p(buf.data_ptr()), nb.value))
        self.fsi[inst] = (buf, mesh["n_theta"] * mesh["n_z"])

    def set_wall(self, X, V, inst=0):
        """External solid: positions (n, 3) now and velocities (lu / step)."""
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1)
        V = np.ascontiguousarray(V, dtype=np.float64).reshape(-1)
        n = self.fsi[inst][1]
        if X.size != 3 * n or V.size != 3 * n:
            raise ValueError("set_wall needs (n_points, 3) positions and velocities")
        self._check(lib().lbm_set_wall(self.h, inst, _dp(X), _dp(V)))

    def read_wall(self, inst=0):
        n = self.fsi[inst][1]
        out = [np.zeros((n, 3)) for _ in range(5)]
        self._check(lib().lbm_read_wall(self.h, inst, *[_dp(o) for o in out]))
        return dict(X=out[0], Xprev=out[1], slip=out[2], Vf=out[3], F=out[4])

    def wall_shear_stress(self, inst=0, dist=2.0):
        """Wall shear stress at every wall point (lbm_wall_shear_stress)."""
        out = np.zeros(self.fsi[inst][1])
        self._check(lib().lbm_wall_shear_stress(self.h, inst, float(dist), _dp(out)))
        return out

    def ncell(self, inst=0):
        return lib().lbm_num_cells(self.h, inst)

    def write_populations(self, g, inst=0):
        g = np.ascontiguousarray(g, dtype=np.float64).reshape(-1)
        self._check(lib().lbm_write_populations(self.h, inst, _dp(g)))

    def set_rest(self, p, inst=0):
        self._check(lib().lbm_set_rest(self.h, inst, float(p)))

    def read_populations(self, inst=0):
        g = np.zeros((self.ncell(inst), NQ))
        self._check(lib().lbm_read_populations(self.h, inst, _dp(g)))
        return g

    def fields(self, inst=0):
        """(gauge pressure (nz,ny,nx), first moment sum e g (nz,ny,nx,3))."""
        b = self.boxes[inst]
        nc = self.ncell(inst)
        p = np.zeros(nc)
        u = np.zeros((nc, 3))
        self._check(lib().lbm_read_fields(self.h, inst, _dp(p), _dp(u)))
        return p.reshape(b["nz"], b["ny"], b["nx"]), u.reshape(b["nz"], b["ny"], b["nx"], 3)

    def waveforms(self, inst=0, cap=1 << 30):
        cap = min(cap, self.t)
        out = np.zeros((max(cap, 1), NREC))
        n = C.c_int64()
        self._check(lib().lbm_read_waveforms(self.h, inst, _dp(out), cap, C.byref(n)))
        return out[: n.value]

    def outlet_waveforms(self, inst=0, cap=1 << 30):
        """(steps, NOUT, 3): flux, mean gauge pressure and Windkessel Pw of
        each outlet per step."""
        cap = min(cap, self.t)
        out = np.zeros((max(cap, 1), NOUT * 3))
        n = C.c_int64()
        self._check(lib().lbm_read_outlet_waveforms(self.h, inst, _dp(out), cap, C.byref(n)))
        return out[: n.value].reshape(-1, NOUT, 3)

    def set_timing(self, on):
        self._check(lib().lbm_set_timing(self.h, 1 if on else 0))

    def kernel_time(self, kernel):
        n = C.c_int64()
        ms = C.c_double()
        self._check(lib().lbm_kernel_time(self.h, kernel, C.byref(n), C.byref(ms)))
        return n.value, ms.value

    def set_graph(self, on):
        self._check(lib().lbm_set_graph(self.h, 1 if on else 0))

    def set_overlap(self, on):
        self._check(lib().lbm_set_overlap(self.h, 1 if on else 0))

    def debug_slot_writes(self, parity):
        """Store counts per population slot of one collide-stream pass of the
        given parity, shape (19, total cells), populations left unchanged
        (lbm_debug_slot_writes; FP32 contexts)."""
        n = sum(self.ncell(k) for k in range(self.n))
        out = np.zeros((NQ, n), dtype=np.uint32)
        self._check(lib().lbm_debug_slot_writes(self.h, int(parity), out.ctypes.data_as(C.POINTER(C.c_uint32))))
        return out

    def set_deterministic(self, on):
        """Wall tiles launched colour by colour (lbm_set_deterministic)."""
        self._check(lib().lbm_set_deterministic(self.h, 1 if on else 0))

    def set_band_check(self, every):
        self._check(lib().lbm_set_band_check(self.h, int(every)))

    # ---- launch shapes per size class (autotuner) ----------------------
    def classes(self):
        """Per size class: dict(instances, cells, wall_points, block,
        cells_per_lane, wall_tile_theta, wall_tile_z)."""
        out = []
        for q in range(lib().lbm_num_classes(self.h)):
            ni, nc, npt = C.c_int32(), C.c_int64(), C.c_int64()
            self._check(lib().lbm_class_info(self.h, q, C.byref(ni), C.byref(nc), C.byref(npt)))
            la = Launch()
            self._check(lib().lbm_get_launch(self.h, q, C.byref(la)))
            out.append(dict(instances=ni.value, cells=nc.value, wall_points=npt.value, block=la.block,
                            cells_per_lane=la.cells_per_lane, wall_tile_theta=la.wall_tile_theta,
                            wall_tile_z=la.wall_tile_z))
        return out

    def set_launch(self, cls, block, cells_per_lane, wall_tile_theta, wall_tile_z=0):
        """wall_tile_z = 0: the 256-point tile, 256 / wall_tile_theta along z."""
        la = Launch(block, cells_per_lane, wall_tile_theta, wall_tile_z)
        self._check(lib().lbm_set_launch(self.h, cls, C.byref(la)))

    def _class_keys(self):
        """Cache key of each size class: GPU, storage precision, and the
        class's mean cells and wall points per instance (powers of two)."""
        arch = self.torch.cuda.get_device_properties(self.device).gcnArchName.split(":")[0]
        keys = []
        for c in self.classes():
            n = max(c["instances"], 1)
            cb = int(round(np.log2(max(c["cells"] / n, 1))))
            pb = int(round(np.log2(c["wall_points"] / n))) if c["wall_points"] else -1
            keys.append(f"{arch}|p{self.precision}|cells2^{cb}|wall2^{pb}")
        return keys

    def autotune(self, trial_steps=8, cache=None):
        """Launch shapes per size class: taken from the JSON file cache when
        it holds every class's key, else measured by the library's autotuner
        (which advances the state by ordinary steps) and written back.
        Returns the number of steps taken."""
        import json
        import os
        keys = self._class_keys()
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f).get("classes", {})
        if keys and all(k in table for k in keys):
            for q, k in enumerate(keys):
                e = table[k]
                self.set_launch(q, e["block"], e["cells_per_lane"], e["wall_tile_theta"], e.get("wall_tile_z", 0))
            return 0
        adv = C.c_int64()
        self._check(lib().lbm_autotune(self.h, int(trial_steps), C.byref(adv)))
        # classes with the same key take the shapes of the largest of them
        # (small classes time noisily), so that the cache reproduces them
        cls = self.classes()
        pick = {}
        for q, (k, c) in enumerate(zip(keys, cls)):
            if k not in pick or c["cells"] > cls[pick[k]]["cells"]:
                pick[k] = q
        for q, k in enumerate(keys):
            c = cls[pick[k]]
            if pick[k] != q:
                self.set_launch(q, c["block"], c["cells_per_lane"], c["wall_tile_theta"], c["wall_tile_z"])
            table[k] = {a: c[a] for a in ("block", "cells_per_lane", "wall_tile_theta", "wall_tile_z")}
        if cache:
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump({"version": 1, "classes": table}, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return adv.value


def _couple_all(s, k, cfg):
    """0D models of a workload dict: inlet, outlet (outlet 0), exterior, and
    an optional list `outlets` of (kind, params, state) for outlets 0, 1, ..."""
    for b, key in ((0, "inlet"), (1, "outlet"), (2, "exterior")):
        if key in cfg:
            s.couple_0d(k, b, cfg[key][0], cfg[key][1], cfg.get(key + "_state", ()))
    for q, (kind, par, st) in enumerate(cfg.get("outlets", ())):
        s.couple_0d(k, 1 if q == 0 else 2 + q, kind, par, st)


def solver_from_config(cfg, precision=FP32, pops=None, store_scale=0.0, wave_cap=4096):
    """Solver for one workload dict (see lbm_inputs): box, 0D models, initial
    state and wall are passed through the C interface unchanged."""
    s = Solver(dict(nx=cfg["nx"], ny=cfg["ny"], nz=cfg["nz"], tau=cfg["tau"], flags=cfg["flags"],
                    p_ref=cfg.get("p_ref", 0.0), nee_variant=cfg.get("nee_variant", 0)),
               precision=precision, store_scale=store_scale, wave_cap=wave_cap)
    _couple_all(s, 0, cfg)
    if pops is not None:
        s.write_populations(pops)
    elif cfg.get("p_init", 0.0) != 0.0:
        s.set_rest(cfg["p_init"])
    if "mesh" in cfg:
        s.fsi_exchange(0, cfg["mesh"], cfg["k"], cfg["ei"], cfg["mass"], cfg["alpha"], cfg["beta"],
                       margin=cfg.get("band_margin", 2), kernel=cfg.get("kernel", 0), mode=cfg.get("wall_mode", 0),
                       shell=cfg.get("shell", 0), poisson=cfg.get("poisson", 0.5))
    return s


def solver_from_configs(cfgs, precision=FP32, store_scale=0.0, wave_cap=4096):
    """One batched context over several workload dicts (the ensemble): one
    launch per kernel per step advances every instance."""
    boxes = [dict(nx=c["nx"], ny=c["ny"], nz=c["nz"], tau=c["tau"], flags=c["flags"],
                  p_ref=c.get("p_ref", 0.0), nee_variant=c.get("nee_variant", 0)) for c in cfgs]
    s = Solver(boxes, precision=precision, store_scale=store_scale, wave_cap=wave_cap)
    for k, cfg in enumerate(cfgs):
        _couple_all(s, k, cfg)
        if cfg.get("p_init", 0.0) != 0.0:
            s.set_rest(cfg["p_init"], inst=k)
        if "mesh" in cfg:
            s.fsi_exchange(k, cfg["mesh"], cfg["k"], cfg["ei"], cfg["mass"], cfg["alpha"], cfg["beta"],
                           margin=cfg.get("band_margin", 2), kernel=cfg.get("kernel", 0),
                           mode=cfg.get("wall_mode", 0), shell=cfg.get("shell", 0),
                           poisson=cfg.get("poisson", 0.5))
    return s


# ----------------------------------------------------------------------------
# axisymmetric solver
# ----------------------------------------------------------------------------

class AxiSolver:
    """Axisymmetric D2Q9 context (include/lbm_axi.h) on the current GPU: node
    types (nr, nx), row j at r = j + 1/2; boundaries 0 (inlet) and 1 (outlet)."""

    def __init__(self, flags, tau, precision=FP64, periodic_x=False, wave_cap=4096, p_ref=0.0, device="cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self._flags = np.ascontiguousarray(flags, dtype=np.uint8)
        self.nr, self.nx = self._flags.shape
        self.cfg = AxiConfig(self.nx, self.nr, float(tau), precision,
                             self._flags.ctypes.data_as(C.POINTER(C.c_uint8)), 1 if periodic_x else 0, wave_cap,
                             float(p_ref))
        self.h = None
        nb = C.c_size_t()
        self._check(lib().lbm_axi_query_size(C.byref(self.cfg), C.byref(nb)))
        self.buf = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.Stream(device=self.device)
        h = C.c_void_p()
        self._check(lib().lbm_axi_init(C.byref(self.cfg), C.c_void_p(self.buf.data_ptr()), nb.value,
                                       C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self.t = 0

    def _check(self, code):
        if code != 0:
            raise LbmError(code, lib().lbm_axi_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib().lbm_axi_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def couple_0d(self, boundary, kind, params, state=()):
        p = np.ascontiguousarray(params, dtype=np.float64)
        st = np.ascontiguousarray(state, dtype=np.float64) if len(state) else None
        self._check(lib().lbm_axi_couple_0d(self.h, boundary, kind, _dp(p), len(p), _dp(st),
                                            0 if st is None else len(st)))

    def set_body_force(self, G0, omega=0.0):
        self._check(lib().lbm_axi_set_body_force(self.h, float(G0), float(omega)))

    def set_rest(self, p):
        self._check(lib().lbm_axi_set_rest(self.h, float(p)))

    def write_populations(self, g):
        g = np.ascontiguousarray(g, dtype=np.float64)
        if g.size != self.nr * self.nx * 9:
            raise ValueError("populations must be (nr * nx, 9)")
        self._check(lib().lbm_axi_write_populations(self.h, _dp(g)))

    def read_populations(self):
        g = np.zeros((self.nr * self.nx, 9))
        self._check(lib().lbm_axi_read_populations(self.h, _dp(g)))
        return g

    def step(self, n):
        self._check(lib().lbm_axi_step(self.h, int(n)))
        self.t += int(n)

    def sync(self):
        self._check(lib().lbm_axi_sync(self.h))

    def fields(self):
        """Gauge pressure and forced velocity (u_x, u_r), each (nr, nx)."""
        out = [np.zeros((self.nr, self.nx)) for _ in range(3)]
        self._check(lib().lbm_axi_read_fields(self.h, *[_dp(o) for o in out]))
        return out[0], out[1], out[2]

    def waveforms(self, cap=1 << 30):
        m = min(cap, self.t, self.cfg.wave_cap if self.cfg.wave_cap > 0 else 4096)
        out = np.zeros((m, 14))
        n = C.c_int64()
        self._check(lib().lbm_axi_read_waveforms(self.h, _dp(out), m, C.byref(n)))
        return out[:n.value]


def axi_solver_from_config(cfg, precision=FP64, wave_cap=None):
    """Axisymmetric context for a workload dict of lbm_inputs (axi_* builders)."""
    s = AxiSolver(cfg["flags"], cfg["tau"], precision=precision, periodic_x=cfg.get("periodic_x", False),
                  wave_cap=wave_cap or max(4096, int(cfg.get("steps", 0)) + 1),
                  p_ref=cfg.get("p_ref", cfg.get("p_init", 0.0)))
    for b, key in ((0, "inlet"), (1, "outlet")):
        if key in cfg:
            kind, par = cfg[key][0], cfg[key][1]
            st = cfg[key][2] if len(cfg[key]) > 2 else ()
            s.couple_0d(b, kind, par, st)
    if cfg.get("body_force"):
        s.set_body_force(*cfg["body_force"])
    if cfg.get("p_init", 0.0):
        s.set_rest(cfg["p_init"])
    return s
