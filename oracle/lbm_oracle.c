/*
 * lbm_oracle.c -- plain FP64 CPU reference of the 0D-3D coupled lattice
 * Boltzmann / immersed-boundary method (Wei, Amlani & Pahlevan, "Direct 0D-3D
 * coupling of a lattice Boltzmann methodology for fluid-structure
 * hemodynamics simulations", arXiv 2112.05258).
 *
 * TEST INFRASTRUCTURE.  This file is the oracle the HIP path is checked
 * against; it is not part of the product.  Only the tests, the smoke check and
 * the CPU-baseline leg of the benchmark load it.  It shares no code, header,
 * table or helper with the HIP library: it keeps its own D3Q19 tables, stores
 * populations array-of-structures in two lattices and streams by pulling,
 * and evaluates every equation in the order and form the paper writes it.
 *
 * What one step computes (Algorithm 1 of the paper, Sec. 2.3):
 *   1. moments P = c_s^2 sum f_i, j = sum e_i f_i          (Eqs. rho, v)
 *   2. flux Q and mean pressure on the layer next to each 0D plane
 *      (Sec. 2.1.2, flux integral)
 *   3. 0D models advanced one step by forward Euler: LV elastance with valve
 *      switching and C-infinity smoothing (Eqs. LVE, SmoothFunction, vnew),
 *      3-element Windkessel (Eqs. rightbc, rightQ)
 *   4. immersed boundary: interpolate (Eq. interpolation), penalty force
 *      (Eq. LagForce), spread (Eq. EulForce)
 *   5. BGK collision with the incompressible equilibrium and the forcing term
 *      (Eqs. fi, feq, f)
 *   6. streaming; halfway bounce-back at SOLID cells; non-equilibrium
 *      extrapolation from 0D ghost nodes (Eq. Non-equilibrium3 with the
 *      pressure- or velocity-type coupling of Sec. 2.2)
 *   7. wall update by the staggered finite-difference operators
 *      (Eqs. tension, bending; central difference in time), optionally with
 *      the off-diagonal shear and mixed-bending terms of Eq. structure.
 *
 * Populations are stored shifted, g_i = f_i - w_i (an exact change of
 * variables: the equilibrium is linear in P and equals w_i at rest).  All
 * pressures handed in or out are gauge, p = P - c_s^2.  rho_0 = 1.
 *
 * Arithmetic type: `real` is double; the same source built with
 * -DORC_EXTENDED uses long double (x87, 64-bit significand) and serves as
 * the reference for the FP64 bar, where double rounding of the oracle itself
 * (~1e-12 relative on slow flows) would be as large as the bar.  Values
 * cross the interface as double either way.
 *
 * The wall is carried as displacement D = X - X0 from its rest shape (an
 * exact change of variables that keeps wall velocities X^n - X^{n-1} free of
 * the rounding of absolute positions).
 *
 * Parity status: every function here is pinned by a test that does not
 * re-use it (independent numpy brute force, closed forms, conservation laws,
 * Poiseuille / Womersley / Windkessel / Laplace-law checks, the paper's
 * manufactured-solution filament).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <tgmath.h>

#ifdef ORC_EXTENDED
typedef long double real;
#else
typedef double real;
#endif
#ifdef _OPENMP
#include <omp.h>
#endif

#define NQ 19
#define NREC 14
/* Outlets: the OUTLET ghosts of one instance may form up to NOUT separate
 * outlets, each with its own 0D model (the paper's several outlets, each with
 * a Windkessel, Sec. 2.1.2); the cell-type byte of an OUTLET ghost carries
 * its outlet index k in bits 5-7.  Boundary records: 0 inlet, 1 outlet 0,
 * 2 exterior, 2 + k outlet k >= 1. */
#define NOUT 8
#define NBC (3 + NOUT - 1)

/* D3Q19 velocities: rest, 6 faces, 12 edges (weights 1/3, 1/18, 1/36). */
static const int EV[NQ][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static real WT[NQ];
static real CS2;  /* c_s^2 = 1/3 with dx/dt = 1 (Eq. tau) */
static real PI;
static const real RHO0 = 1;

static void init_constants(void) {
  CS2 = (real)1 / 3;
  PI = 4 * atan((real)1);
  for (int i = 0; i < NQ; ++i) {
    int n2 = EV[i][0] * EV[i][0] + EV[i][1] * EV[i][1] + EV[i][2] * EV[i][2];
    WT[i] = n2 == 0 ? (real)1 / 3 : (n2 == 1 ? (real)1 / 18 : (real)1 / 36);
  }
}

enum { T_FLUID = 0, T_SOLID = 1, T_INLET = 2, T_OUTLET = 3, T_EXTP = 4 };
enum { K_PRESSURE = 0, K_VELOCITY = 1, K_WK3 = 2, K_LV = 3 };

static int opp(int i) {
  for (int k = 0; k < NQ; ++k)
    if (EV[k][0] == -EV[i][0] && EV[k][1] == -EV[i][1] && EV[k][2] == -EV[i][2]) return k;
  return -1;
}

/* ------------------------------------------------------------------------ */
/* single-node formulas                                                      */
/* ------------------------------------------------------------------------ */

/* Eq. feq (He & Luo incompressible equilibrium) in the shifted variable:
 * with P / c_s^2 = sum f = 1 + delta, f_eq - w_i = w_i delta + w_i rho0 [..].
 * Working in delta (never adding w_i back) keeps the rounding at the scale of
 * the deviations, not of the weights. */
static real geq(int i, real delta, const real v[3]) {
  real ev = EV[i][0] * v[0] + EV[i][1] * v[1] + EV[i][2] * v[2];
  real vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  return WT[i] * delta + WT[i] * RHO0 * (ev / CS2 + ev * ev / (2 * CS2 * CS2) - vv / (2 * CS2));
}

/* Eq. f (forcing term of He, Shan & Doolen / Guo form). */
static real forcing(int i, real tau, const real v[3], const real b[3]) {
  real ev = EV[i][0] * v[0] + EV[i][1] * v[1] + EV[i][2] * v[2];
  real s = 0;
  for (int a = 0; a < 3; ++a) s += ((EV[i][a] - v[a]) / CS2 + ev * EV[i][a] / (CS2 * CS2)) * b[a];
  return (1 - 1 / (2 * tau)) * WT[i] * s;
}

/* Eq. SmoothFunction: C-infinity step from 1 to 0 over [t0, t0 + Ls]. */
static real smooth_S(real t, real t0, real Ls) {
  if (t < t0) return 1;
  if (t >= t0 + Ls) return 0; /* u = 1: the formula's limit (2/e / 0 -> -inf) */
  real u = (t - t0) / Ls;
  return exp(2 * exp(-1 / u) / (u - 1));
}

/* Double-Hill elastance E(t) and dE/dt (the compliance curve C_v = 1/E).
 * par: [Emax, Emin, Tc, Tmax, P_ed, N_S, k, a1, n1, a2, n2]; t = time within
 * the cycle in steps. */
static void elastance(const real* p, real t, real* E, real* dE) {
  real Emax = p[0], Emin = p[1], Tmax = p[3];
  real k = p[6], a1 = p[7], n1 = p[8], a2 = p[9], n2 = p[10];
  real tn = t / Tmax;
  real A = pow(tn / a1, n1), B = pow(tn / a2, n2);
  real h1 = A / (1 + A), h2 = 1 / (1 + B);
  real dA = tn > 0 ? n1 * pow(tn / a1, n1 - 1) / a1 : 0;
  real dB = tn > 0 ? n2 * pow(tn / a2, n2 - 1) / a2 : 0;
  real dh1 = dA / ((1 + A) * (1 + A));
  real dh2 = -dB / ((1 + B) * (1 + B));
  *E = (Emax - Emin) * k * h1 * h2 + Emin;
  *dE = (Emax - Emin) * k * (dh1 * h2 + h1 * dh2) / Tmax;
}

/* Peskin's 4-point regularised delta (per axis, unit spacing). */
static real phi4(real r) {
  r = fabs(r);
  if (r <= 1) return (3 - 2 * r + sqrt(1 + 4 * r - 4 * r * r)) / 8;
  if (r < 2) return (5 - 2 * r - sqrt(-7 + 12 * r - 4 * r * r)) / 8;
  return 0;
}

/* The 4-point cosine delta, (1 + cos(pi r / 2)) / 4 on |r| < 2: the variant
 * kernel of the wall exchange (same support, partition of unity only). */
static real phicos(real r) {
  r = fabs(r);
  if (r < 2) return (1 + cos(PI * r / 2)) / 4;
  return 0;
}

double orc_smooth_S(double t, double t0, double Ls) {
  init_constants();
  return (double)smooth_S(t, t0, Ls);
}
void orc_elastance(const double* p, double t, double* E, double* dE) {
  real q[11], e, de;
  for (int k = 0; k < 11; ++k) q[k] = p[k];
  elastance(q, t, &e, &de);
  *E = (double)e;
  *dE = (double)de;
}
double orc_phi4(double r) { return (double)phi4(r); }
double orc_phicos(double r) {
  init_constants();
  return (double)phicos(r);
}
void orc_lattice(int* e, double* w) {
  init_constants();
  for (int i = 0; i < NQ; ++i) {
    for (int a = 0; a < 3; ++a) e[3 * i + a] = EV[i][a];
    w[i] = (double)WT[i];
  }
}
void orc_feq(double p_gauge, const double* v, double* g) {
  init_constants();
  real vv[3] = {v[0], v[1], v[2]};
  for (int i = 0; i < NQ; ++i) g[i] = (double)geq(i, (real)p_gauge / CS2, vv);
}
void orc_forcing(double tau, const double* v, const double* b, double* F) {
  init_constants();
  real vv[3] = {v[0], v[1], v[2]}, bb[3] = {b[0], b[1], b[2]};
  for (int i = 0; i < NQ; ++i) F[i] = (double)forcing(i, tau, vv, bb);
}
int orc_is_extended(void) { return sizeof(real) > sizeof(double); }

/* ------------------------------------------------------------------------ */
/* 0D boundary models                                                        */
/* ------------------------------------------------------------------------ */

typedef struct {
  int boundary; /* 0 inlet (z = 0), 1 outlet 0 (z = nz-1), 2 exterior, 2 + k outlet k */
  int kind;
  real par[16];
  real area;      /* number of layer cells of the boundary (flux -> velocity) */
  /* state */
  real Pw, Pv;
  int open;
  int inflow;     /* inflow (Q > 0) seen since the valve opened */
  long Td, cycle;
  /* result of the last update */
  int vmode;      /* 0: pressure-type coupling, 1: velocity-type */
  real pstar;     /* gauge P* (pressure type) */
  real vconst;    /* axial v* (constant velocity) or axial correction (WK) */
  real S;         /* smoothing factor (LV, velocity type) */
  int snap;       /* 1 on the step the valve closes */
} orc_bc;

static void bc_init(orc_bc* c, int boundary, int kind, const double* par, int npar,
                    const double* st, int nst) {
  memset(c, 0, sizeof *c);
  c->boundary = boundary;
  c->kind = kind;
  for (int k = 0; k < npar && k < 16; ++k) c->par[k] = par[k];
  c->Td = -1;
  c->cycle = 0;
  if (kind == K_WK3) c->Pw = nst > 0 ? (real)st[0] : 0;
  if (kind == K_LV) c->Pv = nst > 0 ? (real)st[0] : c->par[4];
}

/* Advance the 0D model of one boundary from t_n to t_{n+1}.  Qp is the flux
 * through the boundary's layer in +z, Pbar its mean gauge pressure. */
static void bc_update(orc_bc* c, long n, real Qp, real Pbar) {
  c->snap = 0;
  switch (c->kind) {
    case K_PRESSURE:
      c->vmode = 0;
      c->pstar = c->par[0];
      break;
    case K_VELOCITY:
      c->vmode = 1;
      c->vconst = c->par[0];
      c->S = 1;
      break;
    case K_WK3: {
      /* Eqs. rightbc / rightQ with Z = Rp, R = Rd, C = C, marched by forward
       * Euler.  par[3] selects the direction of the explicit coupling:
       *  0  pressure type: the 3D side hands over the flux Q leaving the
       *     domain, the boundary pressure follows from rightQ, P = Pw + Z Q;
       *  1  velocity type (the input/output direction the two equations are
       *     written in): the 3D side hands over the mean boundary pressure P,
       *     rightQ gives the outflow Q = (P - Pw)/Z, imposed as a plug
       *     velocity Q / A over the boundary layer. */
      real Z = c->par[0], C = c->par[1], R = c->par[2];
      if (c->par[3] == 0) {
        real Q = (c->boundary == 0) ? -Qp : Qp;
        real P = c->Pw + Z * Q;
        real dPw = P / (C * Z) - (R + Z) / (C * R * Z) * c->Pw;
        c->Pw = c->Pw + dPw;
        c->vmode = 0;
        c->pstar = c->Pw + Z * Q; /* P_0D(t_{n+1}) */
      } else {
        real P = Pbar;
        real dPw = P / (C * Z) - (R + Z) / (C * R * Z) * c->Pw;
        c->Pw = c->Pw + dPw;
        real Q = (P - c->Pw) / Z; /* outflow the 0D model asks for */
        /* v* = v(x_f) + dv e_z: the profile is the fluid's, the flux the
         * model's; dv spreads the flux deficit evenly over the layer. */
        real want = (c->boundary == 0) ? -Q : Q; /* as a +z flux */
        c->vmode = 1;
        c->vconst = (want - Qp) / (c->area > 0 ? c->area : 1);
      }
      break;
    }
    case K_LV: {
      const real* p = c->par;
      real Tc = p[2], NS = p[5];
      long cyc = (long)floor((real)n / Tc);
      if (cyc != c->cycle) { /* new beat: ventricle back at end-diastole */
        c->cycle = cyc;
        c->Pv = p[4];
        c->open = 0;
        c->inflow = 0;
        c->Td = -1;
      }
      real E, dE;
      elastance(p, (real)n - (real)cyc * Tc, &E, &dE);
      real Cv = 1 / E, dCv = -dE / (E * E);
      /* The valve closes when the inflow, after ejection has begun, drops
       * below zero; the flux of the first steps after opening still carries
       * the closed valve's small residual (either sign), which does not
       * count as the inflow reaching zero. */
      if (c->open && c->inflow && Qp < 0) { /* inflow reached zero: valve closes */
        c->open = 0;
        c->Td = n;
        c->snap = 1;
      } else if (c->open) {
        if (Qp > 0) c->inflow = 1;
      } else if (c->Td < 0 && c->Pv > Pbar) { /* P_v above aortic */
        c->open = 1;
        c->inflow = 0;
      }
      real Q = c->open ? Qp : 0;
      /* Eq. LVE, forward Euler */
      c->Pv = c->Pv - (dCv * c->Pv + Q) / Cv;
      if (c->open) {
        c->vmode = 0;
        c->pstar = c->Pv;
      } else {
        c->vmode = 1;
        c->S = (c->Td < 0) ? 0 : smooth_S((real)(n + 1), (real)c->Td, NS);
      }
      break;
    }
  }
}

/* standalone 0D object for unit tests of the ODE models */
void* orc_bc_new(int boundary, int kind, const double* par, int npar, const double* st, int nst) {
  init_constants();
  orc_bc* c = (orc_bc*)malloc(sizeof(orc_bc));
  bc_init(c, boundary, kind, par, npar, st, nst);
  return c;
}
void orc_bc_free(void* c) { free(c); }
/* out: [vmode, pstar, S, Pv, Pw, open, snap, Td] */
void orc_bc_update(void* cv, long n, double Qp, double Pbar, double* out) {
  orc_bc* c = (orc_bc*)cv;
  bc_update(c, n, Qp, Pbar);
  out[0] = c->vmode; out[1] = (double)c->pstar; out[2] = (double)c->S; out[3] = (double)c->Pv;
  out[4] = (double)c->Pw; out[5] = c->open; out[6] = c->snap; out[7] = (double)c->Td;
}

/* v* of a velocity-type update: the constant axial velocity, or the axial
 * correction dv of the pressure-driven Windkessel */
double orc_bc_vconst(void* cv) { return (double)((orc_bc*)cv)->vconst; }
/* boundary area (cells, or the summed ring areas of an axisymmetric layer)
 * that turns the pressure-driven Windkessel's flux deficit into dv */
void orc_bc_set_area(void* cv, double area) { ((orc_bc*)cv)->area = area; }

/* ------------------------------------------------------------------------ */
/* wall (membrane) finite-difference operators                               */
/* ------------------------------------------------------------------------ */

/* Tension vector on the half edge with edge vector d (= X_b - X_a)
 * (Eq. tension): T D0 X with T = Eh (|D0 X| - 1), D0 X = d / ds. */
static void edge_tension(const real d[3], real ds, real Eh, real out[3]) {
  real t[3] = {d[0] / ds, d[1] / ds, d[2] / ds};
  real T = Eh * (sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]) - 1);
  for (int k = 0; k < 3; ++k) out[k] = T * t[k];
}

/* 1D filament forces: points X[0..m-1] (stride 3), the first and last two are
 * given (boundary/ghost) points; forces on points 2..m-3 are
 *   D0(T D0 X) - D+D-(EI D+D- X)   (Eqs. tension and bending).
 * F receives m*3 values (zero at the four given points). */
void orc_filament_force(int m, const double* X, double ds, double Eh, double EI, double* F) {
  memset(F, 0, sizeof(double) * 3 * m);
  real* kap = (real*)calloc((size_t)3 * m, sizeof(real));
  for (int s = 1; s < m - 1; ++s)
    for (int k = 0; k < 3; ++k)
      kap[3 * s + k] = ((real)X[3 * (s + 1) + k] - 2 * (real)X[3 * s + k] + X[3 * (s - 1) + k]) / ((real)ds * ds);
  for (int s = 2; s < m - 2; ++s) {
    real dp[3], dm[3], tp[3], tm[3];
    for (int k = 0; k < 3; ++k) {
      dp[k] = (real)X[3 * (s + 1) + k] - X[3 * s + k];
      dm[k] = (real)X[3 * s + k] - X[3 * (s - 1) + k];
    }
    edge_tension(dp, ds, Eh, tp);
    edge_tension(dm, ds, Eh, tm);
    for (int k = 0; k < 3; ++k) {
      real ten = (tp[k] - tm[k]) / ds;
      real ben = -EI * (kap[3 * (s + 1) + k] - 2 * kap[3 * s + k] + kap[3 * (s - 1) + k]) / ((real)ds * ds);
      F[3 * s + k] = (double)(ten + ben);
    }
  }
  free(kap);
}

/* ------------------------------------------------------------------------ */
/* solver state                                                              */
/* ------------------------------------------------------------------------ */

typedef struct {
  int nx, ny, nz;
  long ncell;
  real tau;
  int per[3];
  uint8_t* type;           /* cell type (low 3 bits of the cell-type byte) */
  uint8_t* oid;            /* outlet index of an OUTLET ghost (bits 5-7) */
  real *g, *gs, *gn;       /* [cell][19] */
  real *D, *j, *v, *b;     /* moments delta = sum g, j = sum e g; v; force */
  real *v0;                /* inlet-layer snapshot, nx*ny*3 */
  orc_bc bc[NBC];
  real body[3], body_omega;
  /* membrane: rest shape X0 and displacements D = X - X0 */
  int nth, nzl;
  long np;
  real *X0, *Dn, *Dp, *slip, *Vf, *F;
  real ds_th, ds_z, area, ks, ei, mass, alpha, beta;
  int nee_normal;          /* 1: NEE from the ghost's normal neighbour */
  int kernel;              /* 0 Peskin 4-point, 1 cosine 4-point */
  int external;            /* 1: the caller moves the points (no membrane forces) */
  int shell;               /* 1: the off-diagonal (i != j) terms of Eq. structure too */
  real phi12;              /* phi_12 = 1 / (2 (1 + Poisson's ratio)) */
  /* waveforms; per outlet k: flux, mean gauge pressure, Windkessel Pw */
  double* rec;
  double* orec;            /* [step][NOUT][3] */
  long nrec, caprec;
  long step;
} orc_t;

static long cidx(const orc_t* o, int x, int y, int z) {
  return (long)x + (long)o->nx * ((long)y + (long)o->ny * z);
}

/* The neighbour of ghost cell s one cell inwards along the normal of the box
 * face it lies on (z faces first, then x, then y): 0 for a cell on no face. */
static int normal_neighbour(const orc_t* o, long s, long* q) {
  const int x = (int)(s % o->nx), y = (int)((s / o->nx) % o->ny), z = (int)(s / ((long)o->nx * o->ny));
  int dx = 0, dy = 0, dz = 0;
  if (z == 0) dz = 1;
  else if (z == o->nz - 1) dz = -1;
  else if (x == 0) dx = 1;
  else if (x == o->nx - 1) dx = -1;
  else if (y == 0) dy = 1;
  else if (y == o->ny - 1) dy = -1;
  else return 0;
  *q = cidx(o, x + dx, y + dy, z + dz);
  return 1;
}

/* Non-equilibrium extrapolation variant: 0 literal x_f = x + e_i (default),
 * 1 the ghost's normal neighbour (Guo, Zheng & Shi 2002). */
void orc_set_nee_variant(void* ov, int v) { ((orc_t*)ov)->nee_normal = v == 1; }

void* orc_create(int nx, int ny, int nz, double tau, const uint8_t* flags, int px, int py, int pz) {
  init_constants();
  orc_t* o = (orc_t*)calloc(1, sizeof(orc_t));
  o->nx = nx; o->ny = ny; o->nz = nz; o->tau = tau;
  o->per[0] = px; o->per[1] = py; o->per[2] = pz;
  o->ncell = (long)nx * ny * nz;
  o->type = (uint8_t*)malloc(o->ncell);
  o->oid = (uint8_t*)malloc(o->ncell);
  for (long c = 0; c < o->ncell; ++c) {
    o->type[c] = flags[c] & 7;
    o->oid[c] = o->type[c] == T_OUTLET ? flags[c] >> 5 : 0;
  }
  o->g = (real*)calloc((size_t)o->ncell * NQ, sizeof(real));
  o->gs = (real*)calloc((size_t)o->ncell * NQ, sizeof(real));
  o->gn = (real*)calloc((size_t)o->ncell * NQ, sizeof(real));
  o->D = (real*)calloc((size_t)o->ncell, sizeof(real));
  o->j = (real*)calloc((size_t)o->ncell * 3, sizeof(real));
  o->v = (real*)calloc((size_t)o->ncell * 3, sizeof(real));
  o->b = (real*)calloc((size_t)o->ncell * 3, sizeof(real));
  o->v0 = (real*)calloc((size_t)nx * ny * 3, sizeof(real));
  double zero = 0.0;
  for (int k = 0; k < NBC; ++k) bc_init(&o->bc[k], k, K_PRESSURE, &zero, 1, NULL, 0);
  return o;
}

void orc_destroy(void* ov) {
  orc_t* o = (orc_t*)ov;
  if (!o) return;
  free(o->type); free(o->oid); free(o->g); free(o->gs); free(o->gn);
  free(o->D); free(o->j); free(o->v); free(o->b); free(o->v0);
  free(o->X0); free(o->Dn); free(o->Dp); free(o->slip); free(o->Vf); free(o->F);
  free(o->rec); free(o->orec);
  free(o);
}

/* boundary: 0 inlet, 1 outlet 0, 2 exterior, 2 + k outlet k (k = 1..NOUT-1) */
void orc_set_bc(void* ov, int boundary, int kind, const double* par, int npar,
                const double* st, int nst) {
  orc_t* o = (orc_t*)ov;
  if (boundary < 0 || boundary >= NBC) return;
  bc_init(&o->bc[boundary], boundary, kind, par, npar, st, nst);
}

void orc_set_body_force(void* ov, double bx, double by, double bz, double omega) {
  orc_t* o = (orc_t*)ov;
  o->body[0] = bx; o->body[1] = by; o->body[2] = bz; o->body_omega = omega;
}

/* g (AoS, [cell][19]) for FLUID cells; other cells are ignored. */
void orc_set_pops(void* ov, const double* g) {
  orc_t* o = (orc_t*)ov;
  for (long c = 0; c < o->ncell; ++c)
    for (int i = 0; i < NQ; ++i) o->g[c * NQ + i] = (o->type[c] == T_FLUID) ? (real)g[c * NQ + i] : 0;
}
void orc_get_pops(void* ov, double* g) {
  orc_t* o = (orc_t*)ov;
  for (long k = 0; k < NQ * o->ncell; ++k) g[k] = (double)o->g[k];
}
/* uniform rest state at gauge pressure p: f_i = f_i^eq(P = c_s^2 + p, v = 0) */
void orc_set_rest(void* ov, double p) {
  orc_t* o = (orc_t*)ov;
  real v[3] = {0, 0, 0};
  for (long c = 0; c < o->ncell; ++c)
    for (int i = 0; i < NQ; ++i) o->g[c * NQ + i] = (o->type[c] == T_FLUID) ? geq(i, (real)p / CS2, v) : 0;
}

int orc_set_membrane(void* ov, int nth, int nzl, const double* X0, double ds_th, double ds_z,
                     double area, double ks, double ei, double mass, double alpha, double beta) {
  orc_t* o = (orc_t*)ov;
  o->nth = nth; o->nzl = nzl; o->np = (long)nth * nzl;
  size_t n3 = (size_t)o->np * 3;
  o->X0 = (real*)malloc(n3 * sizeof(real));
  o->Dn = (real*)calloc(n3, sizeof(real));
  o->Dp = (real*)calloc(n3, sizeof(real));
  o->slip = (real*)calloc(n3, sizeof(real));
  o->Vf = (real*)calloc(n3, sizeof(real));
  o->F = (real*)calloc(n3, sizeof(real));
  for (size_t k = 0; k < n3; ++k) o->X0[k] = X0[k];
  o->ds_th = ds_th; o->ds_z = ds_z; o->area = area;
  o->ks = ks; o->ei = ei; o->mass = mass; o->alpha = alpha; o->beta = beta;
  return 0;
}

/* Wall options: delta kernel (0 Peskin 4-point, 1 cosine) and external-solid
 * mode (1: the points are moved by the caller through orc_set_wall; between
 * calls they keep their velocity, X^{n+1} = 2 X^n - X^{n-1}; no membrane
 * forces act and the force on the solid is only reported). */
void orc_set_wall_options(void* ov, int kernel, int external) {
  orc_t* o = (orc_t*)ov;
  o->kernel = kernel;
  o->external = external;
}

/* Shell model: with shell = 1 the membrane force takes the i != j terms of
 * Eq. structure as well (in-plane shear with phi_12 = 1 / (2 (1 + nu)) and
 * the mixed bending with gamma_12 = 1); 0 keeps the two coordinate
 * directions only. */
void orc_set_shell(void* ov, int shell, double poisson) {
  orc_t* o = (orc_t*)ov;
  o->shell = shell;
  o->phi12 = 1 / (2 * (1 + (real)poisson));
}

/* Positions X (np*3) at t_n and velocities V (lattice units per step) of the
 * points: D^n = X - X0, D^{n-1} = D^n - V. */
void orc_set_wall(void* ov, const double* X, const double* V) {
  orc_t* o = (orc_t*)ov;
  for (long k = 0; k < 3 * o->np; ++k) {
    o->Dn[k] = (real)X[k] - o->X0[k];
    o->Dp[k] = o->Dn[k] - (real)V[k];
  }
}

/* X, Xprev, slip integral, interpolated fluid velocity, force on the fluid:
 * each np*3 (any pointer may be NULL). */
void orc_get_lagrangian(void* ov, double* X, double* Xp, double* slip, double* Vf, double* F) {
  orc_t* o = (orc_t*)ov;
  for (long k = 0; k < 3 * o->np; ++k) {
    if (X) X[k] = (double)(o->X0[k] + o->Dn[k]);
    if (Xp) Xp[k] = (double)(o->X0[k] + o->Dp[k]);
    if (slip) slip[k] = (double)o->slip[k];
    if (Vf) Vf[k] = (double)o->Vf[k];
    if (F) F[k] = (double)o->F[k];
  }
}
/* displacement of the wall from its rest shape, now and one step earlier */
void orc_get_displacement(void* ov, double* Dn, double* Dp) {
  orc_t* o = (orc_t*)ov;
  for (long k = 0; k < 3 * o->np; ++k) {
    if (Dn) Dn[k] = (double)o->Dn[k];
    if (Dp) Dp[k] = (double)o->Dp[k];
  }
}

/* ------------------------------------------------------------------------ */
/* immersed-boundary transfer (Eqs. interpolation and EulForce)              */
/* ------------------------------------------------------------------------ */

static real delta(const orc_t* o, real r) { return o->kernel == 1 ? phicos(r) : phi4(r); }

/* V(X) = sum over the 4x4x4 stencil of u(node) phi phi phi, FLUID nodes only,
 * for the point X = x0 + d; u is a dense [cell][3] field. */
/* The stencil of the point X = x0 + d: the 4 x 4 x 4 nodes from
 * base = floor(X) - 1, and the kernel's value along each axis at each of its
 * 4 node offsets (phi(x - X) per axis; a node's weight is their product). */
static void ib_stencil(const orc_t* o, const real* x0, const real* d, int base[3], real phi[3][4]) {
  for (int a = 0; a < 3; ++a) {
    base[a] = (int)floor(x0[a] + d[a]) - 1;
    for (int m = 0; m < 4; ++m) phi[a][m] = delta(o, ((base[a] + m) - x0[a]) - d[a]);
  }
}

/* V(X) = sum over the 4x4x4 stencil of u(node) phi phi phi, FLUID nodes only,
 * for the point X = x0 + d; u is a dense [cell][3] field. */
static void ib_interp_one(const orc_t* o, const real* x0, const real* d, const real* u, real V[3]) {
  int base[3];
  real phi[3][4];
  ib_stencil(o, x0, d, base, phi);
  V[0] = V[1] = V[2] = 0;
  for (int c = 0; c < 4; ++c)
    for (int bb = 0; bb < 4; ++bb)
      for (int a = 0; a < 4; ++a) {
        int x = base[0] + a, y = base[1] + bb, z = base[2] + c;
        if (x < 0 || y < 0 || z < 0 || x >= o->nx || y >= o->ny || z >= o->nz) continue;
        long id = cidx(o, x, y, z);
        if (o->type[id] != T_FLUID) continue;
        real w = phi[0][a] * phi[1][bb] * phi[2][c];
        for (int k = 0; k < 3; ++k) V[k] += u[3 * id + k] * w;
      }
}

/* b(node) += F area phi phi phi, FLUID nodes only, for the nodes of the
 * stencil with zlo <= z < zhi. */
static void ib_spread_one(const orc_t* o, const real* x0, const real* d, const real F[3], real area, real* b,
                          int zlo, int zhi) {
  int base[3];
  real phi[3][4];
  ib_stencil(o, x0, d, base, phi);
  for (int c = 0; c < 4; ++c)
    for (int bb = 0; bb < 4; ++bb)
      for (int a = 0; a < 4; ++a) {
        int x = base[0] + a, y = base[1] + bb, z = base[2] + c;
        if (x < 0 || y < 0 || z < zlo || x >= o->nx || y >= o->ny || z >= zhi) continue;
        long id = cidx(o, x, y, z);
        if (o->type[id] != T_FLUID) continue;
        real w = phi[0][a] * phi[1][bb] * phi[2][c];
        for (int k = 0; k < 3; ++k) b[3 * id + k] += F[k] * area * w;
      }
}

/* b = sum over all points, in index order, of their spread force.  Each
 * thread owns a range of z planes and adds only into its own cells while it
 * walks every point in order, so each cell receives its terms in the same
 * order whatever the thread count. */
static void ib_spread_all(const orc_t* o, long np, const real* X0, const real* Dn, const real* F, real area,
                          real* b) {
#pragma omp parallel
  {
    int nt = 1, t = 0;
#ifdef _OPENMP
    nt = omp_get_num_threads();
    t = omp_get_thread_num();
#endif
    const int zlo = (int)((long)o->nz * t / nt), zhi = (int)((long)o->nz * (t + 1) / nt);
    for (long p = 0; p < np; ++p) {
      const real* x0 = &X0[3 * p];
      const real* d = Dn ? &Dn[3 * p] : NULL;
      const int zb = (int)floor(x0[2] + (d ? d[2] : 0)) - 1;
      if (zb + 3 < zlo || zb >= zhi) continue;
      const real zero[3] = {0, 0, 0};
      ib_spread_one(o, x0, d ? d : zero, &F[3 * p], area, b, zlo, zhi);
    }
  }
}

void orc_ib_interp(void* ov, long np, const double* X, const double* u, double* V) {
  orc_t* o = (orc_t*)ov;
  real* uu = (real*)malloc(sizeof(real) * 3 * o->ncell);
  for (long k = 0; k < 3 * o->ncell; ++k) uu[k] = u[k];
  for (long p = 0; p < np; ++p) {
    real x0[3] = {X[3 * p], X[3 * p + 1], X[3 * p + 2]}, d[3] = {0, 0, 0}, v[3];
    ib_interp_one(o, x0, d, uu, v);
    for (int a = 0; a < 3; ++a) V[3 * p + a] = (double)v[a];
  }
  free(uu);
}
void orc_ib_spread(void* ov, long np, const double* X, const double* F, double area, double* b) {
  orc_t* o = (orc_t*)ov;
  real* bb = (real*)calloc((size_t)3 * o->ncell, sizeof(real));
  real* xx = (real*)malloc(sizeof(real) * 3 * np + 1);
  real* ff = (real*)malloc(sizeof(real) * 3 * np + 1);
  for (long k = 0; k < 3 * np; ++k) { xx[k] = X[k]; ff[k] = F[k]; }
  ib_spread_all(o, np, xx, NULL, ff, area, bb);
  for (long k = 0; k < 3 * o->ncell; ++k) b[k] = (double)bb[k];
  free(bb); free(xx); free(ff);
}

/* Membrane force per unit area on every point (Eq. structure along the two
 * coordinate directions, Eqs. tension and bending, plus its off-diagonal
 * terms when the shell model is on): theta periodic, rings
 * 0 and nzl-1 are simply supported fixed ends (curvature zero there).
 * Bending acts on the displacement D from the rest shape X0. */
static void membrane_force(const orc_t* o, const real* D, real* Fel) {
  int nth = o->nth, nzl = o->nzl;
  const real* X0 = o->X0;
  real* kt = (real*)calloc((size_t)3 * o->np, sizeof(real));
  real* kz = (real*)calloc((size_t)3 * o->np, sizeof(real));
  real dt2 = o->ds_th * o->ds_th, dz2 = o->ds_z * o->ds_z;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nzl; ++k)
    for (int jj = 0; jj < nth; ++jj) {
      long p = jj + (long)nth * k;
      long pe = (jj + 1) % nth + (long)nth * k, pw = (jj + nth - 1) % nth + (long)nth * k;
      for (int a = 0; a < 3; ++a) kt[3 * p + a] = (D[3 * pe + a] - 2 * D[3 * p + a] + D[3 * pw + a]) / dt2;
      if (k > 0 && k < nzl - 1) {
        long pn = p + nth, ps = p - nth;
        for (int a = 0; a < 3; ++a) kz[3 * p + a] = (D[3 * pn + a] - 2 * D[3 * p + a] + D[3 * ps + a]) / dz2;
      }
    }
  /* edge vector from point a to point b: (X0_b - X0_a) + (D_b - D_a) */
#define EDGE(a, b, out)                                                          \
  for (int q = 0; q < 3; ++q) out[q] = (X0[3 * (b) + q] - X0[3 * (a) + q]) + (D[3 * (b) + q] - D[3 * (a) + q]);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nzl; ++k)
    for (int jj = 0; jj < nth; ++jj) {
      long p = jj + (long)nth * k;
      real f[3] = {0, 0, 0}, e[3], tp[3], tm[3];
      long pe = (jj + 1) % nth + (long)nth * k, pw = (jj + nth - 1) % nth + (long)nth * k;
      EDGE(p, pe, e);
      edge_tension(e, o->ds_th, o->ks, tp);
      EDGE(pw, p, e);
      edge_tension(e, o->ds_th, o->ks, tm);
      for (int a = 0; a < 3; ++a) {
        f[a] += (tp[a] - tm[a]) / o->ds_th;
        f[a] -= o->ei * (kt[3 * pe + a] - 2 * kt[3 * p + a] + kt[3 * pw + a]) / dt2;
      }
      if (k > 0 && k < nzl - 1) {
        long pn = p + nth, ps = p - nth;
        EDGE(p, pn, e);
        edge_tension(e, o->ds_z, o->ks, tp);
        EDGE(ps, p, e);
        edge_tension(e, o->ds_z, o->ks, tm);
        for (int a = 0; a < 3; ++a) {
          f[a] += (tp[a] - tm[a]) / o->ds_z;
          f[a] -= o->ei * (kz[3 * pn + a] - 2 * kz[3 * p + a] + kz[3 * ps + a]) / dz2;
        }
      }
      for (int a = 0; a < 3; ++a) Fel[3 * p + a] = f[a];
    }
  if (o->shell) {
    /* The i != j terms of Eq. structure.  In-plane shear: the strain
     * S = X_theta . X_z (zero for the rest cylinder), with both tangents
     * taken at the centre of each mesh cell as the mean of its two edges
     * along that direction; the fluxes Eh phi12 S X_z (differentiated along
     * theta) and Eh phi12 S X_theta (along z) live on the cell centres, and
     * their divergence at a point is the difference of the two centre pairs
     * on either side, each pair averaged.  Mixed bending: with gamma_12 =
     * gamma_21 = 1 the two terms add to -2 EI D+D-_z (D+D-_theta D), the
     * theta curvature of the displacement being zero on the end rings
     * (simply supported). */
    long nc = (long)nth * (nzl - 1);
    real* cA = (real*)calloc((size_t)3 * nc + 1, sizeof(real));
    real* cB = (real*)calloc((size_t)3 * nc + 1, sizeof(real));
    real c = o->ks * o->phi12;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nzl - 1; ++k)
      for (int jj = 0; jj < nth; ++jj) {
        long p00 = jj + (long)nth * k, p10 = (jj + 1) % nth + (long)nth * k;
        long p01 = p00 + nth, p11 = p10 + nth;
        real e0[3], e1[3], xt[3], xz[3];
        EDGE(p00, p10, e0);
        EDGE(p01, p11, e1);
        for (int a = 0; a < 3; ++a) xt[a] = (e0[a] + e1[a]) / (2 * o->ds_th);
        EDGE(p00, p01, e0);
        EDGE(p10, p11, e1);
        for (int a = 0; a < 3; ++a) xz[a] = (e0[a] + e1[a]) / (2 * o->ds_z);
        real S = xt[0] * xz[0] + xt[1] * xz[1] + xt[2] * xz[2];
        long q = jj + (long)nth * k;
        for (int a = 0; a < 3; ++a) {
          cA[3 * q + a] = c * S * xz[a];
          cB[3 * q + a] = c * S * xt[a];
        }
      }
#pragma omp parallel for schedule(static)
    for (int k = 1; k < nzl - 1; ++k)
      for (int jj = 0; jj < nth; ++jj) {
        long p = jj + (long)nth * k;
        int jw = (jj + nth - 1) % nth;
        /* centre (j + 1/2, k + 1/2) is entry j + nth k */
        long ne = jj + (long)nth * k, se = jj + (long)nth * (k - 1);
        long nw = jw + (long)nth * k, sw = jw + (long)nth * (k - 1);
        for (int a = 0; a < 3; ++a) {
          real shear = ((cA[3 * ne + a] + cA[3 * se + a]) - (cA[3 * nw + a] + cA[3 * sw + a])) / (2 * o->ds_th) +
                       ((cB[3 * ne + a] + cB[3 * nw + a]) - (cB[3 * se + a] + cB[3 * sw + a])) / (2 * o->ds_z);
          real kn = (k + 1 < nzl - 1) ? kt[3 * (p + nth) + a] : 0;
          real ksth = (k - 1 > 0) ? kt[3 * (p - nth) + a] : 0;
          real mixed = (kn - 2 * kt[3 * p + a] + ksth) / dz2;
          Fel[3 * p + a] += shear - 2 * o->ei * mixed;
        }
      }
    free(cA); free(cB);
  }
#undef EDGE
  free(kt); free(kz);
}

void orc_membrane_force(void* ov, const double* X, double* Fel) {
  orc_t* o = (orc_t*)ov;
  real* D = (real*)calloc((size_t)3 * o->np + 1, sizeof(real));
  real* F = (real*)calloc((size_t)3 * o->np + 1, sizeof(real));
  for (long k = 0; k < 3 * o->np; ++k) D[k] = (real)X[k] - o->X0[k];
  membrane_force(o, D, F);
  for (long k = 0; k < 3 * o->np; ++k) Fel[k] = (double)F[k];
  free(D); free(F);
}

/* ------------------------------------------------------------------------ */
/* one time step                                                             */
/* ------------------------------------------------------------------------ */

static void record(orc_t* o, const double* r, const double* ro) {
  if (o->nrec == o->caprec) {
    o->caprec = o->caprec ? 2 * o->caprec : 1024;
    o->rec = (double*)realloc(o->rec, sizeof(double) * NREC * o->caprec);
    o->orec = (double*)realloc(o->orec, sizeof(double) * 3 * NOUT * o->caprec);
  }
  memcpy(&o->rec[NREC * o->nrec], r, sizeof(double) * NREC);
  memcpy(&o->orec[3 * NOUT * o->nrec], ro, sizeof(double) * 3 * NOUT);
  o->nrec++;
}

/* boundary record of the OUTLET ghost with outlet index k */
static int outlet_bc(int k) { return k == 0 ? 1 : 2 + k; }

static int src_cell(const orc_t* o, int x, int y, int z, int i, long* out) {
  int c[3] = {x - EV[i][0], y - EV[i][1], z - EV[i][2]};
  int n[3] = {o->nx, o->ny, o->nz};
  for (int a = 0; a < 3; ++a) {
    if (c[a] < 0 || c[a] >= n[a]) {
      if (!o->per[a]) return 0;
      c[a] = (c[a] + n[a]) % n[a];
    }
  }
  *out = cidx(o, c[0], c[1], c[2]);
  return 1;
}

static void one_step(orc_t* o) {
  const long n = o->step;
  const int nx = o->nx, ny = o->ny, nz = o->nz;
  const real tau = o->tau;

  /* 1. moments at t_n (Eqs. rho and v without the force half-shift):
   *    sum f = 1 + delta with delta = sum g; sum e f = sum e g. */
#pragma omp parallel for schedule(static)
  for (long c = 0; c < o->ncell; ++c) {
    if (o->type[c] != T_FLUID) continue;
    real s = 0, jx = 0, jy = 0, jz = 0;
    for (int i = 0; i < NQ; ++i) {
      real g = o->g[c * NQ + i];
      s += g;
      jx += EV[i][0] * g; jy += EV[i][1] * g; jz += EV[i][2] * g;
    }
    o->D[c] = s;
    o->j[3 * c] = jx; o->j[3 * c + 1] = jy; o->j[3 * c + 2] = jz;
  }

  /* 2. flux and mean gauge pressure on the first fluid layer next to each
   *    0D plane: the inlet (side 0) and each outlet k (side 1 + k: the cells
   *    of z = nz-2 above an OUTLET ghost of index k) */
  real Qp[1 + NOUT], Pm[1 + NOUT];
  for (int side = 0; side < 1 + NOUT; ++side) {
    int zl = side == 0 ? 1 : nz - 2, zg = side == 0 ? 0 : nz - 1;
    int gt = side == 0 ? T_INLET : T_OUTLET;
    long cnt = 0;
    real q = 0, ps = 0;
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        if (zl < 0 || zl >= nz) continue;
        long c = cidx(o, x, y, zl), gc = cidx(o, x, y, zg);
        if (o->type[c] != T_FLUID || o->type[gc] != gt) continue;
        if (side > 0 && o->oid[gc] != side - 1) continue;
        q += o->j[3 * c + 2] / (1 + o->D[c]); /* sum e f / sum f, dA = 1 */
        ps += CS2 * o->D[c];                    /* P - c_s^2 */
        cnt++;
      }
    Qp[side] = q;
    Pm[side] = cnt ? ps / cnt : 0;
    o->bc[side == 0 ? 0 : outlet_bc(side - 1)].area = (real)cnt;
  }
  /* the same sums on the mid-length plane z = nz/2, over the columns of the
   * inlet's lumen (cells above an INLET ghost): recorded, not coupled */
  real Qmid = 0, Pmid = 0;
  {
    const int zm = nz / 2;
    long cnt = 0;
    real ps = 0;
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        long c = cidx(o, x, y, zm);
        if (o->type[c] != T_FLUID || o->type[cidx(o, x, y, 0)] != T_INLET) continue;
        Qmid += o->j[3 * c + 2] / (1 + o->D[c]);
        ps += CS2 * o->D[c];
        cnt++;
      }
    Pmid = cnt ? ps / cnt : 0;
  }

  /* 3. 0D models to t_{n+1} */
  bc_update(&o->bc[0], n, Qp[0], Pm[0]);
  for (int k = 0; k < NOUT; ++k) bc_update(&o->bc[outlet_bc(k)], n, Qp[1 + k], Pm[1 + k]);
  bc_update(&o->bc[2], n, 0, 0);
  if (o->bc[0].snap) { /* v0(x_f) = v(x_f, T_d) on the inlet layer */
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        long c = cidx(o, x, y, 1);
        for (int a = 0; a < 3; ++a)
          o->v0[3 * ((long)x + (long)nx * y) + a] = (o->type[c] == T_FLUID) ? o->j[3 * c + a] / RHO0 : 0;
      }
  }

  /* 4. immersed boundary force b(t_n) */
  memset(o->b, 0, sizeof(real) * 3 * o->ncell);
  if (o->np > 0) {
    real* u = (real*)malloc(sizeof(real) * 3 * o->ncell);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < 3 * o->ncell; ++c) u[c] = o->j[c] / RHO0;
#pragma omp parallel for schedule(static)
    for (long p = 0; p < o->np; ++p) {
      ib_interp_one(o, &o->X0[3 * p], &o->Dn[3 * p], u, &o->Vf[3 * p]);
      for (int a = 0; a < 3; ++a) {
        real Vs = o->Dn[3 * p + a] - o->Dp[3 * p + a]; /* dX/dt, backward difference */
        real d = o->Vf[3 * p + a] - Vs;
        o->slip[3 * p + a] += d;
        o->F[3 * p + a] = o->alpha * o->slip[3 * p + a] + o->beta * d; /* on the fluid */
      }
    }
    ib_spread_all(o, o->np, o->X0, o->Dn, o->F, o->area, o->b);
    free(u);
  }
  if (o->body[0] != 0 || o->body[1] != 0 || o->body[2] != 0) {
    real cf = cos(o->body_omega * (real)n);
    for (long c = 0; c < o->ncell; ++c)
      if (o->type[c] == T_FLUID)
        for (int a = 0; a < 3; ++a) o->b[3 * c + a] += o->body[a] * cf;
  }

  /* 5. collision (Eq. fi, collision part) */
#pragma omp parallel for schedule(static)
  for (long c = 0; c < o->ncell; ++c) {
    if (o->type[c] != T_FLUID) continue;
    real v[3];
    for (int a = 0; a < 3; ++a) v[a] = o->j[3 * c + a] / RHO0 + o->b[3 * c + a] / (2 * RHO0);
    for (int a = 0; a < 3; ++a) o->v[3 * c + a] = v[a];
    for (int i = 0; i < NQ; ++i) {
      real gi = o->g[c * NQ + i];
      real ge = geq(i, o->D[c], v);
      o->gs[c * NQ + i] = gi - (gi - ge) / tau + forcing(i, tau, v, &o->b[3 * c]);
    }
  }

  /* 6. streaming by pulling; bounce-back; non-equilibrium extrapolation */
#pragma omp parallel for schedule(static)
  for (long c = 0; c < o->ncell; ++c) {
    if (o->type[c] != T_FLUID) continue;
    int z = (int)(c / ((long)nx * ny)), y = (int)((c / nx) % ny), x = (int)(c % nx);
    for (int i = 0; i < NQ; ++i) {
      long s;
      int t = src_cell(o, x, y, z, i, &s) ? o->type[s] : T_SOLID;
      real out;
      if (t == T_FLUID) {
        out = o->gs[s * NQ + i];
      } else if (t == T_SOLID) {
        out = o->gs[c * NQ + opp(i)];
      } else {
        /* Eq. Non-equilibrium3: boundary equilibrium at (P*, v*) plus the
         * relaxed non-equilibrium part and forcing of x_f; x_f = c (the
         * literal x + e_i), or in the normal-neighbour variant the fluid
         * cell next to the ghost along its plane's inward normal. */
        long xf = c;
        if (o->nee_normal) {
          long q;
          if (normal_neighbour(o, s, &q) && o->type[q] == T_FLUID) xf = q;
        }
        const int xfx = (int)(xf % nx), xfy = (int)((xf / nx) % ny);
        const orc_bc* bc = &o->bc[t == T_INLET ? 0 : (t == T_OUTLET ? outlet_bc(o->oid[s]) : 2)];
        real Dst, vst[3]; /* P* / c_s^2 - 1 and v* */
        const real* vf = &o->v[3 * xf];
        if (bc->vmode == 0) { /* pressure type: (P_0D, v(x_f)) */
          Dst = bc->pstar / CS2;
          for (int a = 0; a < 3; ++a) vst[a] = vf[a];
        } else { /* velocity type: (P(x_f), v_0D) */
          Dst = o->D[xf];
          if (bc->kind == K_LV) { /* Eq. vnew: v0(x_f, T_d) S(t_{n+1}) */
            const real* w0 = &o->v0[3 * ((long)xfx + (long)nx * xfy)];
            for (int a = 0; a < 3; ++a) vst[a] = w0[a] * bc->S;
          } else if (bc->kind == K_WK3) {
            vst[0] = vf[0]; vst[1] = vf[1]; vst[2] = vf[2] + bc->vconst;
          } else {
            vst[0] = 0; vst[1] = 0; vst[2] = bc->vconst;
          }
        }
        out = geq(i, Dst, vst) + (1 - 1 / tau) * (o->g[xf * NQ + i] - geq(i, o->D[xf], vf)) +
              forcing(i, tau, vf, &o->b[3 * xf]);
      }
      o->gn[c * NQ + i] = out;
    }
  }
  real* tmp = o->g; o->g = o->gn; o->gn = tmp;

  /* 7. wall position to t_{n+1}: central difference in time */
  if (o->np > 0) {
    real* Fel = (real*)malloc(sizeof(real) * 3 * o->np);
    membrane_force(o, o->Dn, Fel);
#pragma omp parallel for schedule(static)
    for (long p = 0; p < o->np; ++p) {
      long k = p / o->nth;
      for (int a = 0; a < 3; ++a) {
        real dn = o->Dn[3 * p + a];
        real dnew = o->external                  ? 2 * dn - o->Dp[3 * p + a]
                    : (k == 0 || k == o->nzl - 1) ? dn
                    : 2 * dn - o->Dp[3 * p + a] + (Fel[3 * p + a] - o->F[3 * p + a]) / o->mass;
        o->Dp[3 * p + a] = dn;
        o->Dn[3 * p + a] = dnew;
      }
    }
    free(Fel);
  }

  double r[NREC];
  r[0] = (double)n;
  r[1] = (double)Qp[0]; r[2] = (double)Pm[0]; r[3] = (double)Qp[1]; r[4] = (double)Pm[1];
  r[5] = o->bc[0].vmode;
  r[6] = (double)(o->bc[0].vmode == 0 ? o->bc[0].pstar : (o->bc[0].kind == K_LV ? o->bc[0].S : o->bc[0].vconst));
  r[7] = o->bc[1].vmode;
  r[8] = (double)(o->bc[1].vmode == 0 ? o->bc[1].pstar : o->bc[1].vconst);
  r[9] = (double)(o->bc[0].kind == K_LV ? o->bc[0].Pv : 0);
  r[10] = (double)(o->bc[1].kind == K_WK3 ? o->bc[1].Pw : 0);
  r[11] = o->bc[0].kind == K_LV ? (double)o->bc[0].open : 0.0;
  r[12] = (double)Qmid; r[13] = (double)Pmid;
  double ro[3 * NOUT];
  for (int k = 0; k < NOUT; ++k) {
    const orc_bc* b = &o->bc[outlet_bc(k)];
    ro[3 * k] = (double)Qp[1 + k];
    ro[3 * k + 1] = (double)Pm[1 + k];
    ro[3 * k + 2] = b->kind == K_WK3 ? (double)b->Pw : 0.0;
  }
  record(o, r, ro);
  o->step++;
}

void orc_step(void* ov, long nsteps) {
  orc_t* o = (orc_t*)ov;
  for (long k = 0; k < nsteps; ++k) one_step(o);
}

/* Wall shear stress at every wall point (the paper's case study: WSS =
 * mu dv1/dx3, the axial velocity's derivative along the wall normal, taken
 * through the fluid next to the wall).  At point p with position X: the
 * mesh tangents t_theta (central difference over the periodic ring) and t_z
 * (central difference, one-sided on the end rings) give the inward unit
 * normal n = -(t_theta x t_z)/|..| and the axial unit vector a = t_z/|t_z|;
 * the fluid velocity v = sum e g (unforced, rho_0 = 1) is interpolated
 * trilinearly over the FLUID cells among the 8 around Y = X + dist n
 * (weights renormalised, NaN if none is FLUID), and
 *   WSS_p = mu ((v(Y) - V_wall) . a) / dist,  mu = rho_0 (tau - 1/2) / 3,
 * with V_wall = X^n - X^{n-1} the point's velocity. */
void orc_wss(void* ov, double dist, double* out) {
  orc_t* o = (orc_t*)ov;
  const int nth = o->nth, nzl = o->nzl;
  const real mu = RHO0 * (o->tau - (real)0.5) / 3;
  for (long p = 0; p < o->np; ++p) {
    const int jj = (int)(p % nth), k = (int)(p / nth);
    real X[3], tt[3], tz[3], n[3], a[3], Vw[3];
    const long pe = (jj + 1) % nth + (long)nth * k, pw = (jj + nth - 1) % nth + (long)nth * k;
    const long pn = k < nzl - 1 ? p + nth : p, ps = k > 0 ? p - nth : p;
    for (int q = 0; q < 3; ++q) {
      X[q] = o->X0[3 * p + q] + o->Dn[3 * p + q];
      tt[q] = (o->X0[3 * pe + q] + o->Dn[3 * pe + q]) - (o->X0[3 * pw + q] + o->Dn[3 * pw + q]);
      tz[q] = (o->X0[3 * pn + q] + o->Dn[3 * pn + q]) - (o->X0[3 * ps + q] + o->Dn[3 * ps + q]);
      Vw[q] = o->Dn[3 * p + q] - o->Dp[3 * p + q];
    }
    n[0] = -(tt[1] * tz[2] - tt[2] * tz[1]);
    n[1] = -(tt[2] * tz[0] - tt[0] * tz[2]);
    n[2] = -(tt[0] * tz[1] - tt[1] * tz[0]);
    real nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]), na = sqrt(tz[0] * tz[0] + tz[1] * tz[1] + tz[2] * tz[2]);
    for (int q = 0; q < 3; ++q) { n[q] /= nn; a[q] = tz[q] / na; }
    real Y[3], v[3] = {0, 0, 0}, ws = 0;
    int b[3];
    for (int q = 0; q < 3; ++q) { Y[q] = X[q] + (real)dist * n[q]; b[q] = (int)floor(Y[q]); }
    for (int cz = 0; cz < 2; ++cz)
      for (int cy = 0; cy < 2; ++cy)
        for (int cx = 0; cx < 2; ++cx) {
          const int x = b[0] + cx, y = b[1] + cy, z = b[2] + cz;
          if (x < 0 || y < 0 || z < 0 || x >= o->nx || y >= o->ny || z >= o->nz) continue;
          const long c = cidx(o, x, y, z);
          if (o->type[c] != T_FLUID) continue;
          const real w = (cx ? Y[0] - b[0] : 1 - (Y[0] - b[0])) * (cy ? Y[1] - b[1] : 1 - (Y[1] - b[1])) *
                         (cz ? Y[2] - b[2] : 1 - (Y[2] - b[2]));
          real j[3] = {0, 0, 0};
          for (int i = 0; i < NQ; ++i)
            for (int q = 0; q < 3; ++q) j[q] += EV[i][q] * o->g[c * NQ + i];
          for (int q = 0; q < 3; ++q) v[q] += w * j[q] / RHO0;
          ws += w;
        }
    if (ws <= 0) { out[p] = NAN; continue; }
    real s = 0;
    for (int q = 0; q < 3; ++q) s += (v[q] / ws - Vw[q]) * a[q];
    out[p] = (double)(mu * s / (real)dist);
  }
}

/* gauge pressure p = c_s^2 sum g and first moment sum e_i g_i of every cell
 * (0 off-fluid) */
void orc_get_fields(void* ov, double* p, double* u) {
  orc_t* o = (orc_t*)ov;
  for (long c = 0; c < o->ncell; ++c) {
    real s = 0, j[3] = {0, 0, 0};
    if (o->type[c] == T_FLUID)
      for (int i = 0; i < NQ; ++i) {
        real g = o->g[c * NQ + i];
        s += g;
        for (int a = 0; a < 3; ++a) j[a] += EV[i][a] * g;
      }
    if (p) p[c] = (double)(CS2 * s);
    if (u) for (int a = 0; a < 3; ++a) u[3 * c + a] = (double)j[a];
  }
}

/* last Eulerian force field b (dense [cell][3]) */
void orc_get_force(void* ov, double* b) {
  orc_t* o = (orc_t*)ov;
  for (long k = 0; k < 3 * o->ncell; ++k) b[k] = (double)o->b[k];
}

long orc_get_waveforms(void* ov, double* out, long cap) {
  orc_t* o = (orc_t*)ov;
  long n = o->nrec < cap ? o->nrec : cap;
  if (out && n) memcpy(out, o->rec, sizeof(double) * NREC * n);
  return o->nrec;
}

/* per step and outlet k = 0..NOUT-1: flux, mean gauge pressure, Pw */
long orc_get_outlet_waveforms(void* ov, double* out, long cap) {
  orc_t* o = (orc_t*)ov;
  long n = o->nrec < cap ? o->nrec : cap;
  if (out && n) memcpy(out, o->orec, sizeof(double) * 3 * NOUT * n);
  return o->nrec;
}

long orc_get_step(void* ov) { return ((orc_t*)ov)->step; }

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
