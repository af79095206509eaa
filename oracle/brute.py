"""Brute-force numpy re-derivation of one lattice Boltzmann / IB / 0D step.

Test infrastructure: it pins the C oracle (``lbm_oracle.c``) on tiny
lattices.  It is written independently of that file -- unshifted populations
f_i, push streaming with ``np.roll``, the velocity set generated from its
definition, the 0D models and wall forces re-derived from the paper's
equations -- so that a slip in either (a wrong sign, index, weight or a
dropped term) shows up as a mismatch.

Equations (arXiv 2112.05258): Eq. fi (BGK step), Eq. feq (incompressible
equilibrium), Eq. f (forcing), Eqs. rho / v (moments), flux integral of
Sec. 2.1.2, Eqs. LVE, rightbc, rightQ (0D models), Eq. Non-equilibrium3 with
the pressure/velocity couplings of Sec. 2.2, Eqs. SmoothFunction / vnew,
Eqs. LagForce / interpolation / EulForce (immersed boundary), Eqs. tension /
bending (wall).
"""
from __future__ import annotations

import math
import numpy as np

# interface order of the 19 velocities (documented in include/lbm0d3d.h)
ORDER = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
         (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1),
         (1, 0, -1), (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]


def velocity_set():
    """D3Q19: all e in {-1,0,1}^3 with |e|^2 <= 2; w = 1/3, 1/18, 1/36 by |e|^2."""
    gen = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)
           if a * a + b * b + c * c <= 2]
    assert sorted(gen) == sorted(ORDER)
    e = np.array(ORDER, dtype=np.int64)
    n2 = (e * e).sum(1)
    w = np.where(n2 == 0, 1.0 / 3.0, np.where(n2 == 1, 1.0 / 18.0, 1.0 / 36.0))
    opp = np.array([ORDER.index((-a, -b, -c)) for (a, b, c) in ORDER])
    return e, w, opp


E, W, OPP = velocity_set()
CS2 = 1.0 / 3.0
FLUID, SOLID, INLET, OUTLET, EXTP = 0, 1, 2, 3, 4


def f_eq(P, v):
    """Eq. feq; P shape (...), v shape (..., 3) -> (19, ...)."""
    ev = np.einsum("ia,...a->i...", E.astype(float), v)
    vv = (v * v).sum(-1)
    return (W[:, None] * (P / CS2).reshape(1, -1) +
            W[:, None] * (ev.reshape(19, -1) * 3.0 + 4.5 * ev.reshape(19, -1) ** 2 -
                          1.5 * vv.reshape(1, -1))).reshape((19,) + np.shape(P))


def force_term(tau, v, b):
    """Eq. f -> (19, ...)."""
    Ef = E.astype(float)
    ev = np.einsum("ia,...a->i...", Ef, v)
    eb = np.einsum("ia,...a->i...", Ef, b)
    vb = (v * b).sum(-1)
    return (1.0 - 0.5 / tau) * W.reshape((19,) + (1,) * vb.ndim) * (3.0 * (eb - vb[None]) + 9.0 * ev * eb)


def smooth(t, t0, L):
    if t < t0:
        return 1.0
    if t > t0 + L:
        return 0.0
    u = (t - t0) / L
    if u == 0.0:
        return 1.0
    if u == 1.0:
        return 0.0
    return math.exp(2.0 * math.exp(-1.0 / u) / (u - 1.0))


def elastance(p, t):
    Emax, Emin, Tc, Tmax, Ped, NS, k, a1, n1, a2, n2 = p[:11]
    x = t / Tmax
    h1 = (x / a1) ** n1 / (1.0 + (x / a1) ** n1)
    h2 = 1.0 / (1.0 + (x / a2) ** n2)
    # derivative by the quotient rule, written out separately
    d1 = 0.0 if x == 0 else (n1 / a1) * (x / a1) ** (n1 - 1) / (1.0 + (x / a1) ** n1) ** 2
    d2 = 0.0 if x == 0 else -(n2 / a2) * (x / a2) ** (n2 - 1) / (1.0 + (x / a2) ** n2) ** 2
    return (Emax - Emin) * k * h1 * h2 + Emin, (Emax - Emin) * k * (d1 * h2 + h1 * d2) / Tmax


def phi(r):
    r = abs(r)
    if r <= 1.0:
        return 0.125 * (3.0 - 2.0 * r + math.sqrt(1.0 + 4.0 * r - 4.0 * r * r))
    if r < 2.0:
        return 0.125 * (5.0 - 2.0 * r - math.sqrt(-7.0 + 12.0 * r - 4.0 * r * r))
    return 0.0


class Boundary:
    def __init__(self, which, kind=0, par=(0.0,), state=()):
        self.which, self.kind, self.par = which, kind, list(par) + [0.0] * 16
        self.Pw = state[0] if (kind == 2 and len(state)) else 0.0
        self.Pv = (state[0] if len(state) else self.par[4]) if kind == 3 else 0.0
        self.open, self.inflow, self.Td, self.cycle = False, False, -1, 0
        self.mode, self.pstar, self.vc, self.S, self.snap, self.area = 0, 0.0, 0.0, 1.0, False, 1.0

    def advance(self, n, Qp, Pbar):
        self.snap = False
        k, p = self.kind, self.par
        if k == 0:
            self.mode, self.pstar = 0, p[0]
        elif k == 1:
            self.mode, self.vc = 1, p[0]
        elif k == 2:
            Z, C, R = p[0], p[1], p[2]
            if p[3] == 0.0:
                Qo = -Qp if self.which == 0 else Qp
                # C dPw/dt = Q - Pw/R  (rightbc after substituting rightQ)
                self.Pw += (Qo - self.Pw / R) / C
                self.mode, self.pstar = 0, self.Pw + Z * Qo
            else:
                self.Pw += (Pbar - self.Pw) / (C * Z) - self.Pw / (C * R)
                Qo = (Pbar - self.Pw) / Z
                target = -Qo if self.which == 0 else Qo
                self.mode, self.vc = 1, (target - Qp) / self.area
        elif k == 3:
            Tc, NS = p[2], p[5]
            cyc = int(math.floor(n / Tc))
            if cyc != self.cycle:
                self.cycle, self.Pv, self.open, self.inflow, self.Td = cyc, p[4], False, False, -1
            Ev, dEv = elastance(p, n - cyc * Tc)
            # closes once inflow, having started, turns negative
            if self.open and self.inflow and Qp < 0.0:
                self.open, self.Td, self.snap = False, n, True
            elif self.open:
                self.inflow = self.inflow or Qp > 0.0
            elif self.Td < 0 and self.Pv > Pbar:
                self.open, self.inflow = True, False
            Q = Qp if self.open else 0.0
            # dPv/dt = (E'/E) Pv - E Q  (Eq. LVE with C_v = 1/E)
            self.Pv = self.Pv + (dEv / Ev) * self.Pv - Ev * Q
            if self.open:
                self.mode, self.pstar = 0, self.Pv
            else:
                self.mode = 1
                self.S = 0.0 if self.Td < 0 else smooth(n + 1, self.Td, NS)


class Brute:
    """Unshifted-population reference for tiny boxes (no periodic axes)."""

    def __init__(self, flags, tau):
        self.t = np.asarray(flags, dtype=np.uint8)
        self.nz, self.ny, self.nx = self.t.shape
        self.tau = tau
        self.f = np.where(self.t[None] == FLUID, W.reshape(19, 1, 1, 1), 0.0)
        self.bc = [Boundary(0), Boundary(1), Boundary(2)]
        self.v0 = np.zeros((self.ny, self.nx, 3))
        self.mesh = None
        self.n = 0
        self.records = []
        self.nee_normal = False    # True: Eq. Non-equilibrium3 at the ghost's normal neighbour

    def set_pops(self, g):
        g = np.asarray(g).reshape(self.nz, self.ny, self.nx, 19)
        self.f = np.where(self.t[None] == FLUID, np.moveaxis(g, -1, 0) + W.reshape(19, 1, 1, 1), 0.0)

    def pops(self):
        g = np.where(self.t[None] == FLUID, self.f - W.reshape(19, 1, 1, 1), 0.0)
        return np.moveaxis(g, 0, -1).reshape(-1, 19)

    def set_membrane(self, mesh, k, ei, mass, alpha, beta):
        m = dict(mesh)
        m.update(k=k, ei=ei, mass=mass, alpha=alpha, beta=beta)
        m["X"] = np.array(mesh["X0"], float)
        m["Xp"] = m["X"].copy()
        m["slip"] = np.zeros_like(m["X"])
        self.mesh = m

    # ------------------------------------------------------------------
    def _stencil(self, X):
        """[(z, y, x, weight)] over the 4x4x4 nodes of point X, FLUID only."""
        out = []
        b = [int(math.floor(c)) - 1 for c in X]
        for dz in range(4):
            for dy in range(4):
                for dx in range(4):
                    x, y, z = b[0] + dx, b[1] + dy, b[2] + dz
                    if not (0 <= x < self.nx and 0 <= y < self.ny and 0 <= z < self.nz):
                        continue
                    if self.t[z, y, x] != FLUID:
                        continue
                    out.append((z, y, x, phi(x - X[0]) * phi(y - X[1]) * phi(z - X[2])))
        return out

    def wall_force(self, X):
        m = self.mesh
        nth, nzl = m["n_theta"], m["n_z"]
        X = X.reshape(nzl, nth, 3)
        Y = X - m["X0"].reshape(nzl, nth, 3)
        F = np.zeros_like(X)

        def tension(d, ds):
            L = np.linalg.norm(d / ds, axis=-1, keepdims=True)
            return m["k"] * (L - 1.0) * d / ds

        # around the ring (periodic)
        tp = tension(np.roll(X, -1, axis=1) - X, m["ds_theta"])
        F += (tp - np.roll(tp, 1, axis=1)) / m["ds_theta"]
        kt = (np.roll(Y, -1, axis=1) - 2 * Y + np.roll(Y, 1, axis=1)) / m["ds_theta"] ** 2
        F -= m["ei"] * (np.roll(kt, -1, axis=1) - 2 * kt + np.roll(kt, 1, axis=1)) / m["ds_theta"] ** 2
        # along the tube: interior rings only, curvature 0 on the end rings
        tz = tension(X[1:] - X[:-1], m["ds_z"])                 # edges k+1/2, k = 0..nzl-2
        kz = np.zeros_like(Y)
        kz[1:-1] = (Y[2:] - 2 * Y[1:-1] + Y[:-2]) / m["ds_z"] ** 2
        F[1:-1] += (tz[1:] - tz[:-1]) / m["ds_z"]
        F[1:-1] -= m["ei"] * (kz[2:] - 2 * kz[1:-1] + kz[:-2]) / m["ds_z"] ** 2
        return F.reshape(-1, 3)

    def _normal_neighbours(self):
        """Flat index of the cell one step inwards from each cell along the
        normal of the box face it lies on (z faces before x before y), -1
        for cells on no face."""
        z, y, x = np.meshgrid(np.arange(self.nz), np.arange(self.ny), np.arange(self.nx), indexing="ij")
        dz = np.where(z == 0, 1, np.where(z == self.nz - 1, -1, 0))
        onz = dz != 0
        dx = np.where(onz, 0, np.where(x == 0, 1, np.where(x == self.nx - 1, -1, 0)))
        onx = dx != 0
        dy = np.where(onz | onx, 0, np.where(y == 0, 1, np.where(y == self.ny - 1, -1, 0)))
        q = ((z + dz) * self.ny + (y + dy)) * self.nx + (x + dx)
        return np.where((dx != 0) | (dy != 0) | (dz != 0), q, -1)

    # ------------------------------------------------------------------
    def step(self):
        t, tau, n = self.t, self.tau, self.n
        fl = t == FLUID
        f = self.f
        rho = f.sum(0)                       # sum f = P / c_s^2
        P = CS2 * rho
        j = np.einsum("ia,izyx->zyxa", E.astype(float), f)

        # flux and mean pressure on the first layer of each 0D plane
        Qs, Ps = [], []
        for zl, zg, code in ((1, 0, INLET), (self.nz - 2, self.nz - 1, OUTLET)):
            m = fl[zl] & (t[zg] == code)
            Qs.append(float((j[zl, :, :, 2][m] / rho[zl][m]).sum()))
            Ps.append(float((P[zl] - CS2)[m].mean()) if m.any() else 0.0)
            self.bc[len(Qs) - 1].area = float(m.sum())
        self.bc[0].advance(n, Qs[0], Ps[0])
        self.bc[1].advance(n, Qs[1], Ps[1])
        self.bc[2].advance(n, 0.0, 0.0)
        if self.bc[0].snap:
            self.v0 = np.where(fl[1][..., None], j[1], 0.0)

        # immersed boundary
        b = np.zeros(j.shape)
        m = self.mesh
        if m is not None:
            npt = m["X"].shape[0]
            Fp = np.zeros((npt, 3))
            for p in range(npt):
                st = self._stencil(m["X"][p])
                Vf = sum((w * j[z, y, x] for (z, y, x, w) in st), np.zeros(3))
                d = Vf - (m["X"][p] - m["Xp"][p])
                m["slip"][p] += d
                Fp[p] = m["alpha"] * m["slip"][p] + m["beta"] * d
            for p in range(npt):
                for (z, y, x, w) in self._stencil(m["X"][p]):
                    b[z, y, x] += Fp[p] * m["area"] * w

        v = j + 0.5 * b
        feq = f_eq(P, v)
        Fi = force_term(tau, v, b)
        fs = f - (f - feq) / tau + Fi
        fs = np.where(fl[None], fs, 0.0)

        fn = np.zeros_like(f)
        idx = np.arange(t.size).reshape(t.shape)
        nn = self._normal_neighbours().ravel() if self.nee_normal else None
        for i in range(19):
            ex, ey, ez = E[i]
            pulled = np.roll(fs[i], shift=(ez, ey, ex), axis=(0, 1, 2))   # fs_i(x - e_i)
            src = np.roll(t, shift=(ez, ey, ex), axis=(0, 1, 2))
            val = np.where(src == FLUID, pulled, 0.0)
            val = np.where(src == SOLID, fs[OPP[i]], val)
            # x_f: the receiving cell itself, or the ghost's normal neighbour
            xf = idx
            if nn is not None:
                q = nn[np.roll(idx, shift=(ez, ey, ex), axis=(0, 1, 2))]
                ok = (q >= 0) & (t.ravel()[np.maximum(q, 0)] == FLUID)
                xf = np.where(ok, q, idx)
            at = lambda a: a.ravel()[xf]                                   # noqa: E731
            vf = v.reshape(-1, 3)[xf]
            for code, bc in ((INLET, self.bc[0]), (OUTLET, self.bc[1]), (EXTP, self.bc[2])):
                sel = src == code
                if not sel.any():
                    continue
                if bc.mode == 0:
                    Pst = np.full(P.shape, CS2 + bc.pstar)
                    vst = vf
                else:
                    Pst = at(P)
                    if bc.kind == 3:
                        v0 = self.v0.reshape(-1, 3)[xf % (self.nx * self.ny)]
                        vst = v0 * bc.S
                    elif bc.kind == 2:
                        vst = vf.copy()
                        vst[..., 2] += bc.vc
                    else:
                        vst = np.zeros_like(v)
                        vst[..., 2] = bc.vc
                nee = f_eq(Pst, vst)[i] + (1.0 - 1.0 / tau) * (at(f[i]) - at(feq[i])) + at(Fi[i])
                val = np.where(sel, nee, val)
            fn[i] = np.where(fl, val, 0.0)
        self.f = fn

        if m is not None:
            Fel = self.wall_force(m["X"])
            nth = m["n_theta"]
            ring = np.arange(m["X"].shape[0]) // nth
            fixed = (ring == 0) | (ring == m["n_z"] - 1)
            Xn = 2 * m["X"] - m["Xp"] + (Fel - Fp) / m["mass"]
            Xn[fixed] = m["X"][fixed]
            m["Xp"], m["X"] = m["X"], Xn

        self.records.append([n, Qs[0], Ps[0], Qs[1], Ps[1]])
        self.n += 1

    def fields(self):
        g = self.f - W.reshape(19, 1, 1, 1)
        g = np.where(self.t[None] == FLUID, g, 0.0)
        p = CS2 * g.sum(0)
        u = np.einsum("ia,izyx->zyxa", E.astype(float), g)
        return p, u
