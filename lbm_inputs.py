"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and bench.py.

This module only *generates inputs*: cell-type masks, Lagrangian rest meshes,
random populations and the parameter sets of the standard workloads.  It holds
none of the method's arithmetic (no equilibrium, collision, streaming, 0D model
or delta kernel); both the plain CPU oracle and the HIP path consume what it
returns, and neither imports the other.

Conventions (they are part of the library interface, `include/lbm0d3d.h`):

* cell (x, y, z) has linear index x + nx*(y + ny*z); arrays are shaped
  (nz, ny, nx) in numpy;
* cell types: FLUID 0, SOLID 1 (halfway bounce-back wall), INLET 2 and OUTLET 3
  (ghost nodes of the 0D-coupled boundary, planes z = 0 and z = nz-1), EXTP 4
  (ghost node held at the exterior reference pressure);
* all pressures are gauge pressures p = P - c_s^2 in lattice units, so that the
  population sum is 1 + 3p;
* time is counted in lattice steps (dt = 1), lengths in lattice units (dx = 1).

Physical 0D parameters (mmHg, ml, s) are mapped to lattice units with three
scales: sigma_t steps per second, sigma_V lattice volumes per ml and sigma_P
lattice pressure per mmHg.  Then E_lu = E * sP/sV, R_lu = R * sP*st/sV,
C_lu = C * sV/sP, Q_lu = Q * sV/st.
"""
from __future__ import annotations

import math
import numpy as np

FLUID, SOLID, INLET, OUTLET, EXTP = 0, 1, 2, 3, 4

# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------

def tube_flags(nx, ny, nz, cx, cy, r, elastic=False):
    """Straight tube along z with the lumen (x-cx)^2 + (y-cy)^2 < r^2.

    rigid (elastic=False): every cell outside the lumen is SOLID, the lumen
    cells of z = 0 / z = nz-1 are INLET / OUTLET ghosts.
    elastic=True: the whole box interior is fluid (the wall is an immersed
    membrane); the box side faces are SOLID; on the end planes the lumen is
    INLET / OUTLET and the rest EXTP (exterior fluid at a reference pressure).
    """
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    lumen = (x - cx) ** 2 + (y - cy) ** 2 < r * r
    side = (x == 0) | (x == nx - 1) | (y == 0) | (y == ny - 1)
    f = np.full((nz, ny, nx), FLUID, dtype=np.uint8)
    if elastic:
        ends = (z == 0) | (z == nz - 1)
        f[ends] = EXTP
        f[(z == 0) & lumen] = INLET
        f[(z == nz - 1) & lumen] = OUTLET
        f[side] = SOLID
    else:
        f[~lumen] = SOLID
        f[(z == 0) & lumen] = INLET
        f[(z == nz - 1) & lumen] = OUTLET
        f[side] = SOLID
    return f


def closed_box_flags(nx, ny, nz):
    """Box whose six faces are SOLID walls (no open boundary)."""
    f = np.full((nz, ny, nx), FLUID, dtype=np.uint8)
    f[0, :, :] = f[-1, :, :] = SOLID
    f[:, 0, :] = f[:, -1, :] = SOLID
    f[:, :, 0] = f[:, :, -1] = SOLID
    return f


def random_flags(nx, ny, nz, seed, solid_frac=0.15, extp=True):
    """Random geometry for brute-force and parity checks.

    Side faces SOLID; end planes a random mix of INLET/OUTLET, EXTP and SOLID;
    interior cells SOLID with probability solid_frac, otherwise FLUID.
    """
    rng = np.random.default_rng(seed)
    f = np.where(rng.random((nz, ny, nx)) < solid_frac, SOLID, FLUID).astype(np.uint8)
    for zz, code in ((0, INLET), (nz - 1, OUTLET)):
        u = rng.random((ny, nx))
        plane = np.full((ny, nx), code, dtype=np.uint8)
        if extp:
            plane[u < 0.25] = EXTP
        plane[u > 0.85] = SOLID
        f[zz] = plane
    f[:, 0, :] = f[:, -1, :] = SOLID
    f[:, :, 0] = f[:, :, -1] = SOLID
    return f


def cylinder_mesh(cx, cy, r, z0, z1, h):
    """Structured Lagrangian mesh of a cylinder wall.

    n_theta points around (periodic), n_z rings from z0 to z1 inclusive
    (rings 0 and n_z-1 are the fixed ends).  Point index p = j + n_theta*k.
    Returns dict with X0 (n, 3) float64, n_theta, n_z, ds_theta (rest chord
    between ring neighbours), ds_z, area (wall area carried by one point).
    """
    n_theta = max(3, int(round(2.0 * math.pi * r / h)))
    n_z = int(round((z1 - z0) / h)) + 1
    ds_z = (z1 - z0) / (n_z - 1)
    th = 2.0 * math.pi * np.arange(n_theta) / n_theta
    zz = z0 + ds_z * np.arange(n_z)
    X0 = np.empty((n_z, n_theta, 3))
    X0[:, :, 0] = cx + r * np.cos(th)[None, :]
    X0[:, :, 1] = cy + r * np.sin(th)[None, :]
    X0[:, :, 2] = zz[:, None]
    ds_theta = 2.0 * r * math.sin(math.pi / n_theta)
    area = (2.0 * math.pi * r / n_theta) * ds_z
    return dict(X0=X0.reshape(-1, 3), n_theta=n_theta, n_z=n_z,
                ds_theta=ds_theta, ds_z=ds_z, area=area)


# ----------------------------------------------------------------------------
# random states
# ----------------------------------------------------------------------------

def random_populations(ncell, seed, amp=1e-3, q=19):
    """Shifted populations g[cell][i] ~ amp * U(-1, 1), AoS (ncell, q) float64."""
    rng = np.random.default_rng(seed)
    return amp * (2.0 * rng.random((ncell, q)) - 1.0)


def random_points(n, lo, hi, seed):
    rng = np.random.default_rng(seed)
    lo = np.asarray(lo, float); hi = np.asarray(hi, float)
    return lo + (hi - lo) * rng.random((n, 3))


# ----------------------------------------------------------------------------
# 0D parameter sets (lattice units)
# ----------------------------------------------------------------------------

# boundary kinds (same codes as the C interface)
BC_PRESSURE_CONST, BC_VELOCITY_CONST, BC_WINDKESSEL3, BC_LV_ELASTANCE = 0, 1, 2, 3

# double-Hill elastance shape constants (published fit used for the LV
# compliance curve): alpha1, n1, alpha2, n2 and the normalisation k
HILL = dict(a1=0.7, n1=1.9, a2=1.17, n2=21.9, k=1.55)


def scales(sigma_t=25000.0, sigma_V=8000.0, sigma_P=2.5e-6):
    return dict(sigma_t=sigma_t, sigma_V=sigma_V, sigma_P=sigma_P)


def lv_params(Emax, Emin, HR, P_ed_mmHg, Ls_seconds, sc):
    """LV-elastance parameter vector in lattice units.

    Layout: [Emax, Emin, Tc, Tmax, P_ed, N_S, k, a1, n1, a2, n2]
    (Emax/Emin in mmHg/ml, HR in beats/min, P_ed in mmHg, Ls in s).
    T_max = (0.2 + 0.15 * T_c[s]) seconds, the published double-Hill timing.
    """
    st, sV, sP = sc["sigma_t"], sc["sigma_V"], sc["sigma_P"]
    Tc_s = 60.0 / HR
    Tmax_s = 0.2 + 0.15 * Tc_s
    return [Emax * sP / sV, Emin * sP / sV, Tc_s * st, Tmax_s * st,
            P_ed_mmHg * sP, round(Ls_seconds * st), HILL["k"],
            HILL["a1"], HILL["n1"], HILL["a2"], HILL["n2"]]


def wk_params(Z, C, R, sc, coupling=0.0):
    """3-element Windkessel [Rp, C, Rd, coupling] in lattice units from
    (mmHg s/ml, ml/mmHg).  coupling 0: flux in, pressure out; 1: mean
    pressure in, outflow out."""
    st, sV, sP = sc["sigma_t"], sc["sigma_V"], sc["sigma_P"]
    return [Z * sP * st / sV, C * sV / sP, R * sP * st / sV, coupling]


# ----------------------------------------------------------------------------
# standard workloads
# ----------------------------------------------------------------------------

def cfg0():
    """Rigid tube r = 8 in 24x24x64, tau 0.8, FP64, constant inlet with
    population sum 1.001, 3-element Windkessel outlet Rp 0.05, C 50, Rd 1.0
    (lattice units), 1000 steps, starting at rest at the inlet pressure."""
    nx, ny, nz = 24, 24, 64
    return dict(
        name="cfg0_rigid_tube_24x24x64",
        nx=nx, ny=ny, nz=nz, tau=0.8,
        flags=tube_flags(nx, ny, nz, 11.5, 11.5, 8.0, elastic=False),
        inlet=(BC_PRESSURE_CONST, [0.001 / 3.0]),
        p_ref=0.001 / 3.0,            # storage reference (exact change of variables)
        # Rp = 0.05 is ~18x the tube's acoustic impedance rho c_s / A, so the
        # Windkessel is coupled in the direction that is stable there: mean
        # outlet pressure in, outflow out (coupling flag 1).
        outlet=(BC_WINDKESSEL3, [0.05, 50.0, 1.0, 1.0]),
        # the paper's initialisation U0 = 0, Q0 = 0, P0 != 0: fluid at rest at
        # the inlet pressure, Windkessel chamber at the same pressure (no
        # initial outflow)
        p_init=0.001 / 3.0,
        outlet_state=[0.001 / 3.0],
        steps=1000,
    )


def _elastic_tube(nx, ny, nz, r, h, k, ei, sc, tau, Emax=2.0, Emin=0.06, HR=75.0,
                  Z=0.05, C=1.5, R=1.0, P0_mmHg=80.0, mass=2.0,
                  alpha=-0.05, beta=-0.5, nee=0, p_ext=None):
    """Elastic tube workload.  The tube and the box start at rest at P0; the
    exterior ghosts hold p_ext (None: P0, so that the wall starts in
    equilibrium) and nee selects the extrapolation variant at the 0D planes
    (0 literal x_f = x + e_i, 1 the ghost's normal neighbour)."""
    cx, cy = (nx - 1) / 2.0, (ny - 1) / 2.0
    mesh = cylinder_mesh(cx, cy, r, 2.0, nz - 3.0, h)
    p0 = P0_mmHg * sc["sigma_P"]
    return dict(
        nx=nx, ny=ny, nz=nz, tau=tau,
        flags=tube_flags(nx, ny, nz, cx, cy, r, elastic=True),
        inlet=(BC_LV_ELASTANCE, lv_params(Emax, Emin, HR, 8.0, 0.075, sc)),
        outlet=(BC_WINDKESSEL3, wk_params(Z, C, R, sc)),
        outlet_state=[p0],            # Windkessel chamber starts at P0
        exterior=(BC_PRESSURE_CONST, [p0 if p_ext is None else p_ext]),
        p_init=p0,                    # uniform initial gauge pressure P0 != 0
        p_ref=p0,                     # storage reference (exact change of variables)
        mesh=mesh, k=k, ei=ei, mass=mass, alpha=alpha, beta=beta,
        scales=sc, nee_variant=nee,
    )


def cfg1(h=0.5, tau=0.5085, sigma_P=5e-7):
    """Elastic tube r = 48 in 128x128x512 (8.4 M cells), FP32, spring k 0.05,
    bending 1e-3, Peskin 4-point kernel, LV-elastance inlet (Emax 2.0, Emin
    0.06 mmHg/ml, HR 75) and Windkessel outlet (Z 0.05, C 1.5, R 1.0), one
    cardiac cycle = 20 000 steps.  tau = 0.5085 gives the Womersley number 16
    of the paper's aorta at r = 48 and 20 000 steps a beat.  The 0D planes
    take the normal-neighbour extrapolation (the literal per-direction form
    feeds each inlet-layer cell's own velocity back into it and runs away
    under strong inflow) and the exterior sits at gauge pressure 0, so the
    tube is always inflated (with the exterior at the diastolic-range P0 the
    thin wall buckles when the tube pressure falls below it)."""
    sc = scales(25000.0, 8000.0, sigma_P)
    c = _elastic_tube(128, 128, 512, 48.0, h, 0.05, 1e-3, sc, tau=tau, nee=1, p_ext=0.0)
    c.update(name="cfg1_fsi_tube_128x128x512", steps=20000)
    return c


def cfg2(beats=1):
    """cfg1's construction at 64x64x256 (r = 24, 0.5 lu wall spacing,
    302 x 503 points), tau 0.6, over `beats` cardiac cycles of 20 000 steps.
    One beat by default: in the second beat a wall mode grows next to the
    fixed end rings at peak flow and the run diverges before the third ends,
    in every variant tried (exterior at P0 or 0, axial pre-stretch, wall
    reaching closer to the end planes, bending 1e-2)."""
    sc = scales(25000.0, 8000.0 * (24.0 / 48.0) ** 2, 5e-7)
    c = _elastic_tube(64, 64, 256, 24.0, 0.5, 0.05, 1e-3, sc, tau=0.6, nee=1, p_ext=0.0)
    c.update(name="cfg2_fsi_tube_64x64x256", steps=20000 * beats)
    return c


def precision_study(r=12.0):
    """Workload of the 16-bit storage study: elastic tube r = 12 in a
    32 x 32 x 128 box with the cfg1 boundary models, three beats of 1600
    steps (sigma_t = 2000 /s at 75 bpm; sigma_V keeps the peak velocities of
    the large tube).  tau = 0.6: at tau = 0.52 the pressure-type inlet
    becomes unstable late in systole on this compressed time scale, when the
    ventricle pressure falls under the downstream pressure while the valve
    is still open.  Bending stiffness 1e-2 (not 1e-3): in diastole the tube
    pressure drops under the exterior's P0 and a thinner wall buckles inwards
    a little further every beat."""
    st = 2000.0
    sc = scales(st, 8000.0 * (r / 48.0) ** 2 * (st / 25000.0), 2.5e-6)
    n = int(round(8 * r / 3))
    nz = int(round(32 * r / 3))
    c = _elastic_tube(n, n, nz, r, 0.5, 0.05, 1e-2, sc, tau=0.6)
    c.update(name=f"precision_study_{n}x{n}x{nz}", steps=3 * int(round(60.0 / 75.0 * st)))
    return c


def outlet_flag(k):
    """Cell-type byte of an OUTLET ghost of outlet k (index in bits 5-7)."""
    return OUTLET | (k << 5)


def branched_duct(nx=14, ny=10, nz=40, septum_from=None, Rd=(1.0, 2.0), Rp=0.05, C=50.0, tau=1.0,
                  p_in=1e-3 / 3.0):
    """Rigid rectangular duct with one inlet and two outlets: the lumen is the
    box interior, a 2-cell SOLID septum (x = nx/2 - 1, nx/2) divides its last
    part into two mirror-image branches, and the OUTLET ghosts of the left
    branch are outlet 0, those of the right branch outlet 1.  Constant
    inlet pressure; each outlet drives its own 3-element Windkessel (Rp, C,
    Rd[k]; pressure in, outflow out, as for the small rigid tube)."""
    f = tube_flags(nx, ny, nz, (nx - 1) / 2, (ny - 1) / 2, 1e9)   # the whole interior is lumen
    z0 = nz // 2 if septum_from is None else septum_from
    xs = (nx // 2 - 1, nx // 2)
    f[z0:, 1:ny - 1, xs[0]:xs[1] + 1] = SOLID
    out = f[nz - 1]
    out[(out == OUTLET)] = outlet_flag(0)
    right = np.zeros_like(out, dtype=bool)
    right[:, xs[1] + 1:] = True
    out[right & (out == outlet_flag(0))] = outlet_flag(1)
    return dict(name=f"branched_duct_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, tau=tau, flags=f,
                inlet=(BC_PRESSURE_CONST, [p_in]), p_ref=p_in, p_init=p_in,
                outlets=[(BC_WINDKESSEL3, [Rp, C, Rd[k], 1.0], [p_in]) for k in range(2)])


def small_fsi(nx=24, ny=24, nz=40, r=7.0, h=0.7, tau=0.6, seed=None):
    """Small elastic tube with the cfg1 boundary models, for parity tests."""
    sc = scales(2500.0, 8000.0 * (r / 48.0) ** 2, 2.5e-6)
    c = _elastic_tube(nx, ny, nz, r, h, 0.05, 1e-3, sc, tau=tau)
    c.update(name=f"small_fsi_{nx}x{ny}x{nz}")
    return c


def inflating_tube():
    """A soft elastic tube (r = 7, k = 0.002, areal mass 0.5) in a 30 x 30 x 40
    box whose exterior is held 200 mmHg below the tube's pressure: the wall
    moves outwards by almost three lattice units within 600 steps, past the
    default band margin (the bulge next to the fixed end rings stays clear
    of the box ends until then)."""
    n, nz, r = 30, 40, 7.0
    sc = scales(2500.0, 8000.0 * (r / 48.0) ** 2, 2.5e-6)
    c = _elastic_tube(n, n, nz, r, 0.7, 0.002, 1e-3, sc, tau=0.6, mass=0.5)
    p0 = c["p_init"]
    c.update(name="inflating_tube_30x30x40", inlet=(BC_PRESSURE_CONST, [p0]), outlet=(BC_PRESSURE_CONST, [p0]),
             exterior=(BC_PRESSURE_CONST, [p0 - 200 * sc["sigma_P"]]), steps=600)
    c.pop("outlet_state")
    return c


def ensemble(n=256, seed=3):
    """Parameter draws of the batched ensemble (radius, length, LV, WK, wall):
    r ~ U[6, 16] lu and L ~ U[48, 160] lu (rounded), Emax ~ U[1.5, 3.0],
    Emin ~ U[0.04, 0.08] mmHg/ml, HR ~ U[60, 100] bpm, Windkessel Z, C, R
    each the reference set (Z 0.05, C 1.5, R 1.0) times U[0.7, 1.3],
    membrane stiffness k ~ U[0.02, 0.1]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        r = int(round(rng.uniform(6.0, 16.0)))
        L = int(round(rng.uniform(48.0, 160.0)))
        out.append(dict(
            r=r, L=L,
            Emax=rng.uniform(1.5, 3.0), Emin=rng.uniform(0.04, 0.08),
            HR=rng.uniform(60.0, 100.0),
            Z=0.05 * rng.uniform(0.7, 1.3), C=1.5 * rng.uniform(0.7, 1.3),
            R=1.0 * rng.uniform(0.7, 1.3), k=rng.uniform(0.02, 0.1)))
    return out


def ensemble_config(p, h=0.5, tau=0.6, sigma_P=5e-7):
    """Workload dict of one ensemble member: an elastic tube of radius r in a
    (2r + 8)^2 x (L + 2) box with the member's LV, Windkessel and wall.
    Volume scale sigma_V ~ r^2 keeps peak velocities near the large tube's."""
    r, L = p["r"], p["L"]
    n = 2 * r + 8
    sc = scales(25000.0, 8000.0 * (r / 48.0) ** 2, sigma_P)
    c = _elastic_tube(n, n, L + 2, float(r), h, p["k"], 1e-3, sc, tau=tau, Emax=p["Emax"], Emin=p["Emin"],
                      HR=p["HR"], Z=p["Z"], C=p["C"], R=p["R"], nee=1, p_ext=0.0)
    c.update(name=f"ensemble_r{r}_L{L}")
    return c


# ----------------------------------------------------------------------------
# learned surrogate: parameter draws and initial weights
# ----------------------------------------------------------------------------

# the 7 surrogate inputs and the box they are drawn from (the ensemble's
# ranges): Emax, Emin (mmHg/ml), HR (bpm), Windkessel Z, C, R (the reference
# set 0.05, 1.5, 1.0 times U[0.7, 1.3]) and the membrane stiffness k
SURROGATE_NAMES = ("Emax", "Emin", "HR", "Z", "C", "R", "k")
SURROGATE_LO = np.array([1.5, 0.04, 60.0, 0.05 * 0.7, 1.5 * 0.7, 1.0 * 0.7, 0.02])
SURROGATE_HI = np.array([3.0, 0.08, 100.0, 0.05 * 1.3, 1.5 * 1.3, 1.0 * 1.3, 0.1])


def surrogate_params(n, seed, lo=SURROGATE_LO, hi=SURROGATE_HI):
    """n parameter vectors drawn uniformly from the box [lo, hi]."""
    rng = np.random.default_rng(seed)
    return lo + (hi - lo) * rng.random((n, len(lo)))


def surrogate_config(p, r=11, L=104, st=2000.0):
    """Elastic tube of fixed geometry (r = 11, length 104: the midpoints of
    the ensemble's ranges) driven by the parameter vector p (the 7 inputs),
    with the 16-bit study's time scale and wall (tau 0.6, bending 1e-2).
    steps: three beats at the vector's heart rate."""
    Emax, Emin, HR, Z, C, R, k = (float(v) for v in p)
    n = 2 * r + 8
    sc = scales(st, 8000.0 * (r / 48.0) ** 2 * (st / 25000.0), 2.5e-6)
    c = _elastic_tube(n, n, L + 2, float(r), 0.5, k, 1e-2, sc, tau=0.6, Emax=Emax, Emin=Emin, HR=HR,
                      Z=Z, C=C, R=R)
    beat = 60.0 / HR * st
    c.update(name=f"surrogate_r{r}_L{L}", beat=beat, steps=int(math.ceil(3 * beat)) + 1)
    return c


def mlp_init(dims, seed):
    """Flat FP64 initial parameters of an MLP with layer widths dims: for each
    layer W (out x in, row-major) then b, both U(-1/sqrt(in), 1/sqrt(in))."""
    rng = np.random.default_rng(seed)
    parts = []
    for k in range(len(dims) - 1):
        fan_in, fan_out = dims[k], dims[k + 1]
        a = 1.0 / np.sqrt(fan_in)
        parts.append(rng.uniform(-a, a, fan_out * fan_in))
        parts.append(rng.uniform(-a, a, fan_out))
    return np.concatenate(parts)


# ----------------------------------------------------------------------------
# axisymmetric workloads (D2Q9 in (x, r); node (i, j) at x = i, r = j + 1/2)
# ----------------------------------------------------------------------------

def axi_pipe(nr, nx, periodic=False, stenosis=None):
    """Node types (nr rows, nx columns) of a straight rigid pipe of radius nr:
    every node fluid, the wall half way past the last row, INLET ghosts in
    column 0 and OUTLET ghosts in column nx-1 unless periodic along x.
    stenosis = (i0, i1, jtop): SOLID nodes in rows >= jtop of columns i0..i1-1
    (the lumen narrows to radius jtop there)."""
    f = np.full((nr, nx), FLUID, np.uint8)
    if not periodic:
        f[:, 0] = INLET
        f[:, -1] = OUTLET
    if stenosis is not None:
        i0, i1, jt = stenosis
        f[jt:, i0:i1] = SOLID
    return f


AXI_D_REF = 20


def axi_aorta(D=20, beats=4, Wo=16.0, tau20=0.51, length_D=25, Z=0.005):
    """The straight-aorta refinement workload: a rigid axisymmetric tube of
    diameter D cells and length 25 D between an LV-elastance inlet (E_es 2.2,
    E_min 0.06 mmHg/ml, HR 60, P_ed 8 mmHg) and a flux-driven Windkessel outlet
    (Z, C 1.5, R 1.0), Womersley number 16.  Every resolution is the same
    continuous problem under acoustic scaling from D = 20 (dx and dt both
    ~ 1/D, so the lattice's sound speed, its Mach number and its pressures
    stay what they are at D = 20, and nu grows with D): with s = D / 20,
    tau = 1/2 + (tau20 - 1/2) s, the beat takes T_20 s steps, 1 ml is
    0.7 s^3 cells and 1 mmHg is 1e-4 in lattice pressure; T_20 =
    2 pi R^2 / (Wo^2 nu) at R = 10.  The rigid tube's only compliance is the
    lattice's own compressibility (sound speed c_s), part of the problem
    being refined.  The flows are slow (Reynolds number ~ 3: the
    physiological ~4 000 with Wo = 16 is beyond BGK at D = 20), and
    Z = 0.005 mmHg s/ml keeps the flux-driven Windkessel coupling inside its
    stable range at every resolution."""
    if D % 2:
        raise ValueError("D must be even")
    R = D // 2
    s = D / AXI_D_REF
    nu20 = (tau20 - 0.5) / 3.0
    T20 = 2.0 * math.pi * (AXI_D_REF / 2) ** 2 / (Wo * Wo * nu20)
    tau = 0.5 + (tau20 - 0.5) * s
    sc = scales(T20 * s, 0.7 * s ** 3, 1e-4)
    nx = length_D * D + 2
    p0 = 80.0 * sc["sigma_P"]
    return dict(
        name=f"axi_aorta_D{D}", nr=R, nx=nx, tau=tau, flags=axi_pipe(R, nx),
        inlet=(BC_LV_ELASTANCE, lv_params(2.2, 0.06, 60.0, 8.0, 0.075, sc)),
        outlet=(BC_WINDKESSEL3, wk_params(Z, 1.5, 1.0, sc, coupling=0.0), [p0]),
        p_init=p0, scales=sc, beat=T20 * s, steps=int(math.ceil(beats * T20 * s)), D=D)
