"""Plain CPU oracle (FP64; long-double build as the FP64-bar reference) of the
0D-3D coupled LB / IB method (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It is the reference the HIP path is
checked against and shares no code with it: ``lbm_oracle.c`` (built here with
gcc) is the solver, ``brute.py`` an independent numpy re-derivation used to
pin it on tiny lattices.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "axi_oracle.c")]   # the 3D solver, the axisymmetric one
_LIBS = {False: os.path.join(_HERE, "liblbm_oracle.so"),       # real = double
         True: os.path.join(_HERE, "liblbm_oracle_ext.so")}    # real = long double
NREC = 14
NOUT = 8          # outlets per box (index in bits 5-7 of an OUTLET ghost's cell type)
Q = 19


def build(force=True):
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math), in FP64 and
    in extended precision (long double, the reference for the FP64 bar)."""
    for ext, path in _LIBS.items():
        if not force and os.path.exists(path) and os.path.getmtime(path) >= max(map(os.path.getmtime, _SRCS)):
            continue
        tmp = path + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-Wno-unused-function", "-o", tmp] + _SRCS + ["-lm"]
        if ext:
            cmd.insert(1, "-DORC_EXTENDED")
        subprocess.check_call(cmd)
        os.replace(tmp, path)
    return _LIBS[False]


_lib = {}


def lib(extended=False):
    if extended not in _lib:
        build(force=False)
        L = C.CDLL(_LIBS[extended])
        vp, dp, ip, u8p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_uint8)
        L.orc_create.restype = vp
        L.orc_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, u8p, C.c_int, C.c_int, C.c_int]
        L.orc_destroy.argtypes = [vp]
        L.orc_set_bc.argtypes = [vp, C.c_int, C.c_int, dp, C.c_int, dp, C.c_int]
        L.orc_set_body_force.argtypes = [vp, C.c_double, C.c_double, C.c_double, C.c_double]
        L.orc_set_pops.argtypes = [vp, dp]
        L.orc_get_pops.argtypes = [vp, dp]
        L.orc_set_rest.argtypes = [vp, C.c_double]
        L.orc_set_membrane.argtypes = [vp, C.c_int, C.c_int, dp, C.c_double, C.c_double, C.c_double,
                                       C.c_double, C.c_double, C.c_double, C.c_double, C.c_double]
        L.orc_get_lagrangian.argtypes = [vp, dp, dp, dp, dp, dp]
        L.orc_get_displacement.argtypes = [vp, dp, dp]
        L.orc_ib_interp.argtypes = [vp, C.c_long, dp, dp, dp]
        L.orc_ib_spread.argtypes = [vp, C.c_long, dp, dp, C.c_double, dp]
        L.orc_membrane_force.argtypes = [vp, dp, dp]
        L.orc_step.argtypes = [vp, C.c_long]
        L.orc_get_fields.argtypes = [vp, dp, dp]
        L.orc_get_force.argtypes = [vp, dp]
        L.orc_get_waveforms.restype = C.c_long
        L.orc_get_waveforms.argtypes = [vp, dp, C.c_long]
        L.orc_wss.argtypes = [vp, C.c_double, dp]
        L.orc_get_outlet_waveforms.restype = C.c_long
        L.orc_get_outlet_waveforms.argtypes = [vp, dp, C.c_long]
        L.orc_get_step.restype = C.c_long
        L.orc_get_step.argtypes = [vp]
        L.orc_smooth_S.restype = C.c_double
        L.orc_smooth_S.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_elastance.argtypes = [dp, C.c_double, dp, dp]
        L.orc_phi4.restype = C.c_double
        L.orc_phi4.argtypes = [C.c_double]
        L.orc_phicos.restype = C.c_double
        L.orc_phicos.argtypes = [C.c_double]
        L.orc_set_wall_options.argtypes = [vp, C.c_int, C.c_int]
        L.orc_set_shell.argtypes = [vp, C.c_int, C.c_double]
        L.orc_set_nee_variant.argtypes = [vp, C.c_int]
        L.orc_set_wall.argtypes = [vp, dp, dp]
        L.orc_lattice.argtypes = [ip, dp]
        L.orc_feq.argtypes = [C.c_double, dp, dp]
        L.orc_forcing.argtypes = [C.c_double, dp, dp, dp]
        L.orc_bc_new.restype = vp
        L.orc_bc_new.argtypes = [C.c_int, C.c_int, dp, C.c_int, dp, C.c_int]
        L.orc_bc_free.argtypes = [vp]
        L.orc_bc_update.argtypes = [vp, C.c_long, C.c_double, C.c_double, dp]
        L.orc_filament_force.argtypes = [C.c_int, dp, C.c_double, C.c_double, C.c_double, dp]
        L.orc_num_threads.restype = C.c_int
        L.orc_is_extended.restype = C.c_int
        L.axo_create.restype = vp
        L.axo_create.argtypes = [C.c_int, C.c_int, C.c_double, u8p, C.c_int]
        L.axo_destroy.argtypes = [vp]
        L.axo_set_bc.argtypes = [vp, C.c_int, C.c_int, dp, C.c_int, dp, C.c_int]
        L.axo_set_body_force.argtypes = [vp, C.c_double, C.c_double]
        L.axo_set_rest.argtypes = [vp, C.c_double]
        L.axo_set_pops.argtypes = [vp, dp]
        L.axo_get_pops.argtypes = [vp, dp]
        L.axo_step.argtypes = [vp, C.c_long]
        L.axo_get_fields.argtypes = [vp, dp, dp, dp]
        L.axo_get_waveforms.restype = C.c_long
        L.axo_get_waveforms.argtypes = [vp, dp, C.c_long]
        _lib[extended] = L
    return _lib[extended]


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _dn(a):
    if a is None:
        return None, None
    return _d(a)


# ----------------------------------------------------------------------------
# single-node formulas (exported for the pin tests)
# ----------------------------------------------------------------------------

def lattice():
    e = np.zeros(57, dtype=np.int32)
    w = np.zeros(19)
    lib().orc_lattice(e.ctypes.data_as(C.POINTER(C.c_int)), w.ctypes.data_as(C.POINTER(C.c_double)))
    return e.reshape(19, 3), w


def feq(p_gauge, v):
    out = np.zeros(19)
    v, vp = _d(v)
    lib().orc_feq(p_gauge, vp, out.ctypes.data_as(C.POINTER(C.c_double)))
    return out


def forcing(tau, v, b):
    out = np.zeros(19)
    v, vp = _d(v)
    b, bp = _d(b)
    lib().orc_forcing(tau, vp, bp, out.ctypes.data_as(C.POINTER(C.c_double)))
    return out


def smooth_S(t, t0, Ls):
    return lib().orc_smooth_S(float(t), float(t0), float(Ls))


def elastance(par, t):
    par, pp = _d(par)
    E = C.c_double(); dE = C.c_double()
    lib().orc_elastance(pp, float(t), C.byref(E), C.byref(dE))
    return E.value, dE.value


def phi4(r):
    return lib().orc_phi4(float(r))


def phicos(r):
    return lib().orc_phicos(float(r))


def filament_force(X, ds, Eh, EI):
    X, xp = _d(X)
    m = X.shape[0]
    F = np.zeros((m, 3))
    lib().orc_filament_force(m, xp, ds, Eh, EI, F.ctypes.data_as(C.POINTER(C.c_double)))
    return F


class ZeroD:
    """One 0D boundary model advanced by hand (unit tests of the ODEs)."""

    def __init__(self, boundary, kind, par, state=()):
        par, pp = _d(par)
        st = np.asarray(state, float) if len(state) else np.zeros(1)
        st, sp = _d(st)
        self._keep = (par, st)
        self.h = lib().orc_bc_new(boundary, kind, pp, len(par), sp, len(state))

    def update(self, n, Qp, Pbar):
        out = np.zeros(8)
        lib().orc_bc_update(self.h, n, Qp, Pbar, out.ctypes.data_as(C.POINTER(C.c_double)))
        return dict(vmode=int(out[0]), pstar=out[1], S=out[2], Pv=out[3], Pw=out[4],
                    open=int(out[5]), snap=int(out[6]), Td=int(out[7]))

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_bc_free(self.h)
            self.h = None


# ----------------------------------------------------------------------------
# the solver
# ----------------------------------------------------------------------------

class Oracle:
    """Two-lattice pull solver (FP64, or long double with extended=True).
    flags: uint8 array (nz, ny, nx)."""

    def __init__(self, flags, tau, periodic=(0, 0, 0), extended=False):
        flags = np.ascontiguousarray(flags, dtype=np.uint8)
        self.nz, self.ny, self.nx = flags.shape
        self.ncell = flags.size
        self.flags = flags
        self.tau = tau
        self.L = lib(extended)
        self.h = self.L.orc_create(self.nx, self.ny, self.nz, tau,
                                   flags.ctypes.data_as(C.POINTER(C.c_uint8)), *periodic)
        self.np = 0

    def __del__(self):
        if getattr(self, "h", None):
            self.L.orc_destroy(self.h)
            self.h = None

    def set_bc(self, boundary, kind, par, state=()):
        par, pp = _d(par)
        st = np.asarray(state, float) if len(state) else np.zeros(1)
        st, sp = _d(st)
        self.L.orc_set_bc(self.h, boundary, kind, pp, len(par), sp, len(state))

    def set_body_force(self, b, omega=0.0):
        self.L.orc_set_body_force(self.h, float(b[0]), float(b[1]), float(b[2]), float(omega))

    def set_pops(self, g):
        g, gp = _d(np.asarray(g).reshape(self.ncell, 19))
        self.L.orc_set_pops(self.h, gp)

    def get_pops(self):
        g = np.zeros((self.ncell, 19))
        self.L.orc_get_pops(self.h, g.ctypes.data_as(C.POINTER(C.c_double)))
        return g

    def set_rest(self, p_gauge):
        self.L.orc_set_rest(self.h, float(p_gauge))

    def set_membrane(self, mesh, k, ei, mass, alpha, beta):
        X0, xp = _d(mesh["X0"])
        self.np = X0.shape[0]
        self.L.orc_set_membrane(self.h, mesh["n_theta"], mesh["n_z"], xp, mesh["ds_theta"],
                               mesh["ds_z"], mesh["area"], k, ei, mass, alpha, beta)

    def set_nee_variant(self, v):
        """0: x_f = x + e_i (literal, default); 1: the ghost's normal neighbour."""
        self.L.orc_set_nee_variant(self.h, int(v))

    def set_wall_options(self, kernel=0, external=False):
        """Delta kernel (0 Peskin 4-point, 1 cosine) and external-solid mode."""
        self.L.orc_set_wall_options(self.h, int(kernel), 1 if external else 0)

    def set_shell(self, shell=True, poisson=0.5):
        """Shell model: also the off-diagonal terms of Eq. structure (in-plane
        shear with phi_12 = 1 / (2 (1 + poisson)), mixed bending)."""
        self.L.orc_set_shell(self.h, 1 if shell else 0, float(poisson))

    def set_wall(self, X, V):
        """External-solid mode: positions at t_n and velocities (lu/step)."""
        X, xp = _d(X)
        V, vp = _d(V)
        self.L.orc_set_wall(self.h, xp, vp)

    def lagrangian(self):
        out = [np.zeros((self.np, 3)) for _ in range(5)]
        ptrs = [o.ctypes.data_as(C.POINTER(C.c_double)) for o in out]
        self.L.orc_get_lagrangian(self.h, *ptrs)
        return dict(X=out[0], Xprev=out[1], slip=out[2], Vf=out[3], F=out[4])

    def displacement(self):
        """(D^n, D^{n-1}) = wall positions minus the rest shape."""
        out = [np.zeros((self.np, 3)) for _ in range(2)]
        self.L.orc_get_displacement(self.h, *[o.ctypes.data_as(C.POINTER(C.c_double)) for o in out])
        return out

    def ib_interp(self, X, u):
        X, xp = _d(X)
        u, up = _d(np.asarray(u).reshape(self.ncell, 3))
        V = np.zeros((X.shape[0], 3))
        self.L.orc_ib_interp(self.h, X.shape[0], xp, up, V.ctypes.data_as(C.POINTER(C.c_double)))
        return V

    def ib_spread(self, X, F, area):
        X, xp = _d(X)
        F, fp = _d(F)
        b = np.zeros((self.ncell, 3))
        self.L.orc_ib_spread(self.h, X.shape[0], xp, fp, float(area), b.ctypes.data_as(C.POINTER(C.c_double)))
        return b

    def membrane_force(self, X):
        X, xp = _d(X)
        F = np.zeros_like(X)
        self.L.orc_membrane_force(self.h, xp, F.ctypes.data_as(C.POINTER(C.c_double)))
        return F

    def wss(self, dist=2.0):
        """Wall shear stress at every wall point: mu times the axial velocity
        difference between the fluid at dist along the inward normal and the
        wall, over dist."""
        out = np.zeros(self.np)
        self.L.orc_wss(self.h, float(dist), out.ctypes.data_as(C.POINTER(C.c_double)))
        return out

    def step(self, n=1):
        self.L.orc_step(self.h, int(n))

    @property
    def t(self):
        return self.L.orc_get_step(self.h)

    def fields(self):
        """(gauge pressure (nz,ny,nx), first moment sum e g (nz,ny,nx,3))."""
        p = np.zeros(self.ncell)
        u = np.zeros((self.ncell, 3))
        self.L.orc_get_fields(self.h, p.ctypes.data_as(C.POINTER(C.c_double)),
                             u.ctypes.data_as(C.POINTER(C.c_double)))
        return p.reshape(self.nz, self.ny, self.nx), u.reshape(self.nz, self.ny, self.nx, 3)

    def force(self):
        b = np.zeros((self.ncell, 3))
        self.L.orc_get_force(self.h, b.ctypes.data_as(C.POINTER(C.c_double)))
        return b

    def waveforms(self):
        n = self.L.orc_get_waveforms(self.h, None, 0)
        out = np.zeros((n, NREC))
        self.L.orc_get_waveforms(self.h, out.ctypes.data_as(C.POINTER(C.c_double)), n)
        return out

    def outlet_waveforms(self):
        """(steps, NOUT, 3): flux, mean gauge pressure and Windkessel Pw of
        each outlet per step."""
        n = self.L.orc_get_outlet_waveforms(self.h, None, 0)
        out = np.zeros((n, NOUT, 3))
        self.L.orc_get_outlet_waveforms(self.h, out.ctypes.data_as(C.POINTER(C.c_double)), n)
        return out


def num_threads():
    return lib().orc_num_threads()


def from_config(cfg, pops=None, extended=False):
    """Oracle set up from one of the lbm_inputs workload dicts."""
    o = Oracle(cfg["flags"], cfg["tau"], extended=extended)
    o.set_nee_variant(cfg.get("nee_variant", 0))
    if "inlet" in cfg:
        o.set_bc(0, cfg["inlet"][0], cfg["inlet"][1], cfg.get("inlet_state", ()))
    if "outlet" in cfg:
        o.set_bc(1, cfg["outlet"][0], cfg["outlet"][1], cfg.get("outlet_state", ()))
    for k, (kind, par, st) in enumerate(cfg.get("outlets", ())):   # outlet k: boundary 1 or 2 + k
        o.set_bc(1 if k == 0 else 2 + k, kind, par, st)
    if "exterior" in cfg:
        o.set_bc(2, cfg["exterior"][0], cfg["exterior"][1])
    if pops is not None:
        o.set_pops(pops)
    elif cfg.get("p_init", 0.0) != 0.0:
        o.set_rest(cfg["p_init"])
    if "mesh" in cfg:
        o.set_membrane(cfg["mesh"], cfg["k"], cfg["ei"], cfg["mass"], cfg["alpha"], cfg["beta"])
        o.set_wall_options(cfg.get("kernel", 0), cfg.get("wall_mode", 0) == 1)
        if cfg.get("shell", 0):
            o.set_shell(True, cfg.get("poisson", 0.5))
    return o


# ----------------------------------------------------------------------------
# axisymmetric D2Q9 solver (axi_oracle.c)
# ----------------------------------------------------------------------------

class Axi:
    """Axisymmetric D2Q9 oracle on an nr x nx grid of node types (row j at
    r = j + 1/2, the axis half way below row 0, rows past nr-1 wall; column 0
    INLET ghosts, column nx-1 OUTLET ghosts, or periodic along x)."""

    def __init__(self, flags, tau, periodic_x=False, extended=False):
        self.L = lib(extended)
        self.flags = np.ascontiguousarray(flags, dtype=np.uint8)
        self.nr, self.nx = self.flags.shape
        self.h = self.L.axo_create(self.nx, self.nr, float(tau),
                                   self.flags.ctypes.data_as(C.POINTER(C.c_uint8)), 1 if periodic_x else 0)

    def __del__(self):
        if getattr(self, "h", None):
            self.L.axo_destroy(self.h)
            self.h = None

    def set_bc(self, boundary, kind, par, state=()):
        par, pp = _d(np.asarray(par, dtype=np.float64))
        st, sp = _dn(np.asarray(state, dtype=np.float64) if len(state) else None)
        self.L.axo_set_bc(self.h, boundary, kind, pp, len(par), sp, 0 if st is None else len(st))

    def set_body_force(self, G0, omega=0.0):
        self.L.axo_set_body_force(self.h, float(G0), float(omega))

    def set_rest(self, p):
        self.L.axo_set_rest(self.h, float(p))

    def set_pops(self, g):
        g, gp = _d(g)
        self.L.axo_set_pops(self.h, gp)

    def get_pops(self):
        g = np.zeros((self.nr * self.nx, 9))
        self.L.axo_get_pops(self.h, g.ctypes.data_as(C.POINTER(C.c_double)))
        return g

    def step(self, n):
        self.L.axo_step(self.h, int(n))

    def fields(self):
        """Gauge pressure and the forced velocity (u_x, u_r), each (nr, nx)."""
        out = [np.zeros((self.nr, self.nx)) for _ in range(3)]
        self.L.axo_get_fields(self.h, *[o.ctypes.data_as(C.POINTER(C.c_double)) for o in out])
        return out[0], out[1], out[2]

    def waveforms(self):
        n = self.L.axo_get_waveforms(self.h, None, 0)
        out = np.zeros((n, NREC))
        self.L.axo_get_waveforms(self.h, out.ctypes.data_as(C.POINTER(C.c_double)), n)
        return out


def axi_from_config(cfg, extended=False):
    """Axisymmetric oracle for a workload dict of lbm_inputs (axi_* builders)."""
    o = Axi(cfg["flags"], cfg["tau"], periodic_x=cfg.get("periodic_x", False), extended=extended)
    for b, key in ((0, "inlet"), (1, "outlet")):
        if key in cfg:
            kind, par = cfg[key][0], cfg[key][1]
            st = cfg[key][2] if len(cfg[key]) > 2 else ()
            o.set_bc(b, kind, par, st)
    if cfg.get("body_force"):
        o.set_body_force(*cfg["body_force"])
    if cfg.get("p_init", 0.0):
        o.set_rest(cfg["p_init"])
    return o
