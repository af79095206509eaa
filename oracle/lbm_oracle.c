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
 *      (Eqs. tension, bending; central difference in time).
 *
 * Populations are stored shifted, g_i = f_i - w_i (an exact change of
 * variables: the equilibrium is linear in P and equals w_i at rest).  All
 * pressures handed in or out are gauge, p = P - c_s^2.  rho_0 = 1.
 *
 * Parity status: every function here is pinned by a test that does not
 * re-use it (independent numpy brute force, closed forms, conservation laws,
 * Poiseuille / Womersley / Windkessel / Laplace-law checks, the paper's
 * manufactured-solution filament).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NQ 19
#define NREC 12

/* D3Q19 velocities: rest, 6 faces, 12 edges (weights 1/3, 1/18, 1/36). */
static const int EV[NQ][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double WT[NQ] = {
    1.0 / 3.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2 = 1.0 / 3.0; /* c_s^2 with dx/dt = 1 (Eq. tau) */
static const double RHO0 = 1.0;

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
 * Working in delta (never adding w_i back) keeps the FP64 rounding at the
 * scale of the deviations, not of the weights. */
static double geq(int i, double delta, const double v[3]) {
  double ev = EV[i][0] * v[0] + EV[i][1] * v[1] + EV[i][2] * v[2];
  double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  return WT[i] * delta +
         WT[i] * RHO0 * (ev / CS2 + ev * ev / (2.0 * CS2 * CS2) - vv / (2.0 * CS2));
}

/* Eq. f (forcing term of He, Shan & Doolen / Guo form). */
static double forcing(int i, double tau, const double v[3], const double b[3]) {
  double ev = EV[i][0] * v[0] + EV[i][1] * v[1] + EV[i][2] * v[2];
  double s = 0.0;
  for (int a = 0; a < 3; ++a)
    s += ((EV[i][a] - v[a]) / CS2 + ev * EV[i][a] / (CS2 * CS2)) * b[a];
  return (1.0 - 1.0 / (2.0 * tau)) * WT[i] * s;
}

/* Eq. SmoothFunction: C-infinity step from 1 to 0 over [t0, t0 + Ls]. */
double orc_smooth_S(double t, double t0, double Ls) {
  if (t < t0) return 1.0;
  if (t >= t0 + Ls) return 0.0; /* u = 1: the formula's limit (2/e / 0 -> -inf) */
  double u = (t - t0) / Ls;
  return exp(2.0 * exp(-1.0 / u) / (u - 1.0));
}

/* Double-Hill elastance E(t) and dE/dt (the compliance curve C_v = 1/E).
 * par: [Emax, Emin, Tc, Tmax, P_ed, N_S, k, a1, n1, a2, n2]; t = time within
 * the cycle in steps. */
void orc_elastance(const double* p, double t, double* E, double* dE) {
  double Emax = p[0], Emin = p[1], Tmax = p[3];
  double k = p[6], a1 = p[7], n1 = p[8], a2 = p[9], n2 = p[10];
  double tn = t / Tmax;
  double A = pow(tn / a1, n1), B = pow(tn / a2, n2);
  double h1 = A / (1.0 + A), h2 = 1.0 / (1.0 + B);
  double dA = tn > 0.0 ? n1 * pow(tn / a1, n1 - 1.0) / a1 : 0.0;
  double dB = tn > 0.0 ? n2 * pow(tn / a2, n2 - 1.0) / a2 : 0.0;
  double dh1 = dA / ((1.0 + A) * (1.0 + A));
  double dh2 = -dB / ((1.0 + B) * (1.0 + B));
  *E = (Emax - Emin) * k * h1 * h2 + Emin;
  *dE = (Emax - Emin) * k * (dh1 * h2 + h1 * dh2) / Tmax;
}

/* Peskin's 4-point regularised delta (per axis, unit spacing). */
double orc_phi4(double r) {
  r = fabs(r);
  if (r <= 1.0) return (3.0 - 2.0 * r + sqrt(1.0 + 4.0 * r - 4.0 * r * r)) / 8.0;
  if (r < 2.0) return (5.0 - 2.0 * r - sqrt(-7.0 + 12.0 * r - 4.0 * r * r)) / 8.0;
  return 0.0;
}

void orc_lattice(int* e, double* w) {
  for (int i = 0; i < NQ; ++i) {
    for (int a = 0; a < 3; ++a) e[3 * i + a] = EV[i][a];
    w[i] = WT[i];
  }
}
void orc_feq(double p_gauge, const double* v, double* g) {
  for (int i = 0; i < NQ; ++i) g[i] = geq(i, p_gauge / CS2, v);
}
void orc_forcing(double tau, const double* v, const double* b, double* F) {
  for (int i = 0; i < NQ; ++i) F[i] = forcing(i, tau, v, b);
}

/* ------------------------------------------------------------------------ */
/* 0D boundary models                                                        */
/* ------------------------------------------------------------------------ */

typedef struct {
  int boundary; /* 0 inlet (z = 0), 1 outlet (z = nz-1), 2 exterior */
  int kind;
  double par[16];
  double area;    /* number of layer cells of the boundary (flux -> velocity) */
  /* state */
  double Pw, Pv;
  int open;
  long Td, cycle;
  /* result of the last update */
  int vmode;      /* 0: pressure-type coupling, 1: velocity-type */
  double pstar;   /* gauge P* (pressure type) */
  double vconst;  /* axial v* (constant velocity) or axial correction (WK) */
  double S;       /* smoothing factor (LV, velocity type) */
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
  if (kind == K_WK3) c->Pw = nst > 0 ? st[0] : 0.0;
  if (kind == K_LV) c->Pv = nst > 0 ? st[0] : c->par[4];
}

/* Advance the 0D model of one boundary from t_n to t_{n+1}.  Qp is the flux
 * through the boundary's layer in +z, Pbar its mean gauge pressure.
 * rec receives [mode, value, Pv, Pw, valve]. */
static void bc_update(orc_bc* c, long n, double Qp, double Pbar) {
  c->snap = 0;
  switch (c->kind) {
    case K_PRESSURE:
      c->vmode = 0;
      c->pstar = c->par[0];
      break;
    case K_VELOCITY:
      c->vmode = 1;
      c->vconst = c->par[0];
      c->S = 1.0;
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
      double Z = c->par[0], C = c->par[1], R = c->par[2];
      if (c->par[3] == 0.0) {
        double Q = (c->boundary == 0) ? -Qp : Qp;
        double P = c->Pw + Z * Q;
        double dPw = P / (C * Z) - (R + Z) / (C * R * Z) * c->Pw;
        c->Pw = c->Pw + dPw;
        c->vmode = 0;
        c->pstar = c->Pw + Z * Q; /* P_0D(t_{n+1}) */
      } else {
        double P = Pbar;
        double dPw = P / (C * Z) - (R + Z) / (C * R * Z) * c->Pw;
        c->Pw = c->Pw + dPw;
        double Q = (P - c->Pw) / Z; /* outflow the 0D model asks for */
        /* v* = v(x_f) + dv e_z: the profile is the fluid's, the flux the
         * model's; dv spreads the flux deficit evenly over the layer. */
        double want = (c->boundary == 0) ? -Q : Q; /* as a +z flux */
        c->vmode = 1;
        c->vconst = (want - Qp) / (c->area > 0.0 ? c->area : 1.0);
      }
      break;
    }
    case K_LV: {
      const double* p = c->par;
      double Tc = p[2], NS = p[5];
      long cyc = (long)floor((double)n / Tc);
      if (cyc != c->cycle) { /* new beat: ventricle back at end-diastole */
        c->cycle = cyc;
        c->Pv = p[4];
        c->open = 0;
        c->Td = -1;
      }
      double E, dE;
      orc_elastance(p, (double)n - (double)cyc * Tc, &E, &dE);
      double Cv = 1.0 / E, dCv = -dE / (E * E);
      if (c->open && Qp < 0.0) { /* inflow reached zero: valve closes */
        c->open = 0;
        c->Td = n;
        c->snap = 1;
      } else if (!c->open && c->Td < 0 && c->Pv > Pbar) { /* P_v above aortic */
        c->open = 1;
      }
      double Q = c->open ? Qp : 0.0;
      /* Eq. LVE, forward Euler */
      c->Pv = c->Pv - (dCv * c->Pv + Q) / Cv;
      if (c->open) {
        c->vmode = 0;
        c->pstar = c->Pv;
      } else {
        c->vmode = 1;
        c->S = (c->Td < 0) ? 0.0 : orc_smooth_S((double)(n + 1), (double)c->Td, NS);
      }
      break;
    }
  }
}

/* standalone 0D object for unit tests of the ODE models */
void* orc_bc_new(int boundary, int kind, const double* par, int npar, const double* st, int nst) {
  orc_bc* c = (orc_bc*)malloc(sizeof(orc_bc));
  bc_init(c, boundary, kind, par, npar, st, nst);
  return c;
}
void orc_bc_free(void* c) { free(c); }
/* out: [vmode, pstar, S, Pv, Pw, open, snap, Td] */
void orc_bc_update(void* cv, long n, double Qp, double Pbar, double* out) {
  orc_bc* c = (orc_bc*)cv;
  bc_update(c, n, Qp, Pbar);
  out[0] = c->vmode; out[1] = c->pstar; out[2] = c->S; out[3] = c->Pv;
  out[4] = c->Pw; out[5] = c->open; out[6] = c->snap; out[7] = (double)c->Td;
}

/* ------------------------------------------------------------------------ */
/* wall (membrane) finite-difference operators                               */
/* ------------------------------------------------------------------------ */

/* Tension vector on the half edge from a to b (Eq. tension):
 * T D0 X with T = Eh (|D0 X| - 1), D0 X = (b - a)/ds. */
static void half_edge_tension(const double* a, const double* b, double ds, double Eh, double out[3]) {
  double d[3] = {(b[0] - a[0]) / ds, (b[1] - a[1]) / ds, (b[2] - a[2]) / ds};
  double T = Eh * (sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) - 1.0);
  for (int k = 0; k < 3; ++k) out[k] = T * d[k];
}

/* 1D filament forces: points X[0..m-1] (stride 3), the first and last two are
 * given (boundary/ghost) points; forces on points 2..m-3 are
 *   D0(T D0 X) - D+D-(EI D+D- X)   (Eqs. tension and bending).
 * F receives m*3 values (zero at the four given points). */
void orc_filament_force(int m, const double* X, double ds, double Eh, double EI, double* F) {
  memset(F, 0, sizeof(double) * 3 * m);
  double* kap = (double*)calloc((size_t)3 * m, sizeof(double));
  for (int s = 1; s < m - 1; ++s)
    for (int k = 0; k < 3; ++k)
      kap[3 * s + k] = (X[3 * (s + 1) + k] - 2.0 * X[3 * s + k] + X[3 * (s - 1) + k]) / (ds * ds);
  for (int s = 2; s < m - 2; ++s) {
    double tp[3], tm[3];
    half_edge_tension(&X[3 * s], &X[3 * (s + 1)], ds, Eh, tp);
    half_edge_tension(&X[3 * (s - 1)], &X[3 * s], ds, Eh, tm);
    for (int k = 0; k < 3; ++k) {
      double ten = (tp[k] - tm[k]) / ds;
      double ben = -EI * (kap[3 * (s + 1) + k] - 2.0 * kap[3 * s + k] + kap[3 * (s - 1) + k]) / (ds * ds);
      F[3 * s + k] = ten + ben;
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
  double tau;
  int per[3];
  uint8_t* type;
  double *g, *gs, *gn;       /* [cell][19] */
  double *D, *j, *v, *b;      /* moments delta = sum g, j = sum e g; v; force */
  double *v0;                 /* inlet-layer snapshot, nx*ny*3 */
  orc_bc bc[3];
  double body[3], body_omega;
  /* membrane */
  int nth, nzl;
  long np;
  double *X0, *X, *Xp, *slip, *Vf, *F;
  double ds_th, ds_z, area, ks, ei, mass, alpha, beta;
  /* waveforms */
  double* rec;
  long nrec, caprec;
  long step;
  double last_Q[2], last_P[2];
} orc_t;

static long cidx(const orc_t* o, int x, int y, int z) {
  return (long)x + (long)o->nx * ((long)y + (long)o->ny * z);
}

void* orc_create(int nx, int ny, int nz, double tau, const uint8_t* flags, int px, int py, int pz) {
  orc_t* o = (orc_t*)calloc(1, sizeof(orc_t));
  o->nx = nx; o->ny = ny; o->nz = nz; o->tau = tau;
  o->per[0] = px; o->per[1] = py; o->per[2] = pz;
  o->ncell = (long)nx * ny * nz;
  o->type = (uint8_t*)malloc(o->ncell);
  memcpy(o->type, flags, o->ncell);
  o->g = (double*)calloc((size_t)o->ncell * NQ, sizeof(double));
  o->gs = (double*)calloc((size_t)o->ncell * NQ, sizeof(double));
  o->gn = (double*)calloc((size_t)o->ncell * NQ, sizeof(double));
  o->D = (double*)calloc((size_t)o->ncell, sizeof(double));
  o->j = (double*)calloc((size_t)o->ncell * 3, sizeof(double));
  o->v = (double*)calloc((size_t)o->ncell * 3, sizeof(double));
  o->b = (double*)calloc((size_t)o->ncell * 3, sizeof(double));
  o->v0 = (double*)calloc((size_t)nx * ny * 3, sizeof(double));
  double zero = 0.0;
  for (int k = 0; k < 3; ++k) bc_init(&o->bc[k], k, K_PRESSURE, &zero, 1, NULL, 0);
  return o;
}

void orc_destroy(void* ov) {
  orc_t* o = (orc_t*)ov;
  if (!o) return;
  free(o->type); free(o->g); free(o->gs); free(o->gn);
  free(o->D); free(o->j); free(o->v); free(o->b); free(o->v0);
  free(o->X0); free(o->X); free(o->Xp); free(o->slip); free(o->Vf); free(o->F);
  free(o->rec);
  free(o);
}

void orc_set_bc(void* ov, int boundary, int kind, const double* par, int npar,
                const double* st, int nst) {
  orc_t* o = (orc_t*)ov;
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
    for (int i = 0; i < NQ; ++i) o->g[c * NQ + i] = (o->type[c] == T_FLUID) ? g[c * NQ + i] : 0.0;
}
void orc_get_pops(void* ov, double* g) {
  orc_t* o = (orc_t*)ov;
  memcpy(g, o->g, sizeof(double) * NQ * o->ncell);
}
/* uniform rest state at gauge pressure p: f_i = f_i^eq(P = c_s^2 + p, v = 0) */
void orc_set_rest(void* ov, double p) {
  orc_t* o = (orc_t*)ov;
  double v[3] = {0, 0, 0};
  for (long c = 0; c < o->ncell; ++c)
    for (int i = 0; i < NQ; ++i)
      o->g[c * NQ + i] = (o->type[c] == T_FLUID) ? geq(i, p / CS2, v) : 0.0;
}

int orc_set_membrane(void* ov, int nth, int nzl, const double* X0, double ds_th, double ds_z,
                     double area, double ks, double ei, double mass, double alpha, double beta) {
  orc_t* o = (orc_t*)ov;
  o->nth = nth; o->nzl = nzl; o->np = (long)nth * nzl;
  size_t n3 = (size_t)o->np * 3;
  o->X0 = (double*)malloc(n3 * sizeof(double));
  o->X = (double*)malloc(n3 * sizeof(double));
  o->Xp = (double*)malloc(n3 * sizeof(double));
  o->slip = (double*)calloc(n3, sizeof(double));
  o->Vf = (double*)calloc(n3, sizeof(double));
  o->F = (double*)calloc(n3, sizeof(double));
  memcpy(o->X0, X0, n3 * sizeof(double));
  memcpy(o->X, X0, n3 * sizeof(double));
  memcpy(o->Xp, X0, n3 * sizeof(double));
  o->ds_th = ds_th; o->ds_z = ds_z; o->area = area;
  o->ks = ks; o->ei = ei; o->mass = mass; o->alpha = alpha; o->beta = beta;
  return 0;
}

/* X, Xprev, slip integral, interpolated fluid velocity, force on the fluid:
 * each np*3 (any pointer may be NULL). */
void orc_get_lagrangian(void* ov, double* X, double* Xp, double* slip, double* Vf, double* F) {
  orc_t* o = (orc_t*)ov;
  size_t n = sizeof(double) * 3 * o->np;
  if (X) memcpy(X, o->X, n);
  if (Xp) memcpy(Xp, o->Xp, n);
  if (slip) memcpy(slip, o->slip, n);
  if (Vf) memcpy(Vf, o->Vf, n);
  if (F) memcpy(F, o->F, n);
}
void orc_set_lagrangian(void* ov, const double* X, const double* Xp) {
  orc_t* o = (orc_t*)ov;
  size_t n = sizeof(double) * 3 * o->np;
  if (X) memcpy(o->X, X, n);
  if (Xp) memcpy(o->Xp, Xp, n);
}

/* ------------------------------------------------------------------------ */
/* immersed-boundary transfer (Eqs. interpolation and EulForce)              */
/* ------------------------------------------------------------------------ */

/* V(X) = sum over the 4x4x4 stencil of u(node) phi phi phi, FLUID nodes only.
 * u is a dense [cell][3] field. */
static void ib_interp_one(const orc_t* o, const double* Xp, const double* u, double V[3]) {
  int base[3];
  for (int a = 0; a < 3; ++a) base[a] = (int)floor(Xp[a]) - 1;
  V[0] = V[1] = V[2] = 0.0;
  for (int c = 0; c < 4; ++c)
    for (int bb = 0; bb < 4; ++bb)
      for (int a = 0; a < 4; ++a) {
        int x = base[0] + a, y = base[1] + bb, z = base[2] + c;
        if (x < 0 || y < 0 || z < 0 || x >= o->nx || y >= o->ny || z >= o->nz) continue;
        long id = cidx(o, x, y, z);
        if (o->type[id] != T_FLUID) continue;
        double w = orc_phi4(x - Xp[0]) * orc_phi4(y - Xp[1]) * orc_phi4(z - Xp[2]);
        for (int k = 0; k < 3; ++k) V[k] += u[3 * id + k] * w;
      }
}

/* b(node) += F area phi phi phi, FLUID nodes only, points in order. */
static void ib_spread_one(const orc_t* o, const double* Xp, const double F[3], double area, double* b) {
  int base[3];
  for (int a = 0; a < 3; ++a) base[a] = (int)floor(Xp[a]) - 1;
  for (int c = 0; c < 4; ++c)
    for (int bb = 0; bb < 4; ++bb)
      for (int a = 0; a < 4; ++a) {
        int x = base[0] + a, y = base[1] + bb, z = base[2] + c;
        if (x < 0 || y < 0 || z < 0 || x >= o->nx || y >= o->ny || z >= o->nz) continue;
        long id = cidx(o, x, y, z);
        if (o->type[id] != T_FLUID) continue;
        double w = orc_phi4(x - Xp[0]) * orc_phi4(y - Xp[1]) * orc_phi4(z - Xp[2]);
        for (int k = 0; k < 3; ++k) b[3 * id + k] += F[k] * area * w;
      }
}

void orc_ib_interp(void* ov, long np, const double* X, const double* u, double* V) {
  orc_t* o = (orc_t*)ov;
  for (long p = 0; p < np; ++p) ib_interp_one(o, &X[3 * p], u, &V[3 * p]);
}
void orc_ib_spread(void* ov, long np, const double* X, const double* F, double area, double* b) {
  orc_t* o = (orc_t*)ov;
  memset(b, 0, sizeof(double) * 3 * o->ncell);
  for (long p = 0; p < np; ++p) ib_spread_one(o, &X[3 * p], &F[3 * p], area, b);
}

/* Membrane force per unit area on every point (Eq. structure restricted to the
 * two coordinate directions, Eqs. tension and bending): theta periodic, rings
 * 0 and nzl-1 are simply supported fixed ends (curvature zero there).
 * Bending acts on the displacement from the rest shape X0. */
static void membrane_force(const orc_t* o, const double* X, double* Fel) {
  int nth = o->nth, nzl = o->nzl;
  double* Y = (double*)malloc(sizeof(double) * 3 * o->np);
  double* kt = (double*)calloc((size_t)3 * o->np, sizeof(double));
  double* kz = (double*)calloc((size_t)3 * o->np, sizeof(double));
  for (long p = 0; p < 3 * o->np; ++p) Y[p] = X[p] - o->X0[p];
  double dt2 = o->ds_th * o->ds_th, dz2 = o->ds_z * o->ds_z;
  for (int k = 0; k < nzl; ++k)
    for (int jj = 0; jj < nth; ++jj) {
      long p = jj + (long)nth * k;
      long pe = (jj + 1) % nth + (long)nth * k, pw = (jj + nth - 1) % nth + (long)nth * k;
      for (int a = 0; a < 3; ++a) kt[3 * p + a] = (Y[3 * pe + a] - 2.0 * Y[3 * p + a] + Y[3 * pw + a]) / dt2;
      if (k > 0 && k < nzl - 1) {
        long pn = p + nth, ps = p - nth;
        for (int a = 0; a < 3; ++a) kz[3 * p + a] = (Y[3 * pn + a] - 2.0 * Y[3 * p + a] + Y[3 * ps + a]) / dz2;
      }
    }
  for (int k = 0; k < nzl; ++k)
    for (int jj = 0; jj < nth; ++jj) {
      long p = jj + (long)nth * k;
      double f[3] = {0, 0, 0};
      long pe = (jj + 1) % nth + (long)nth * k, pw = (jj + nth - 1) % nth + (long)nth * k;
      double tp[3], tm[3];
      half_edge_tension(&X[3 * p], &X[3 * pe], o->ds_th, o->ks, tp);
      half_edge_tension(&X[3 * pw], &X[3 * p], o->ds_th, o->ks, tm);
      for (int a = 0; a < 3; ++a) {
        f[a] += (tp[a] - tm[a]) / o->ds_th;
        f[a] -= o->ei * (kt[3 * pe + a] - 2.0 * kt[3 * p + a] + kt[3 * pw + a]) / dt2;
      }
      if (k > 0 && k < nzl - 1) {
        long pn = p + nth, ps = p - nth;
        half_edge_tension(&X[3 * p], &X[3 * pn], o->ds_z, o->ks, tp);
        half_edge_tension(&X[3 * ps], &X[3 * p], o->ds_z, o->ks, tm);
        for (int a = 0; a < 3; ++a) {
          f[a] += (tp[a] - tm[a]) / o->ds_z;
          f[a] -= o->ei * (kz[3 * pn + a] - 2.0 * kz[3 * p + a] + kz[3 * ps + a]) / dz2;
        }
      }
      for (int a = 0; a < 3; ++a) Fel[3 * p + a] = f[a];
    }
  free(Y); free(kt); free(kz);
}

void orc_membrane_force(void* ov, const double* X, double* Fel) {
  membrane_force((orc_t*)ov, X, Fel);
}

/* ------------------------------------------------------------------------ */
/* one time step                                                             */
/* ------------------------------------------------------------------------ */

static void record(orc_t* o, const double* r) {
  if (o->nrec == o->caprec) {
    o->caprec = o->caprec ? 2 * o->caprec : 1024;
    o->rec = (double*)realloc(o->rec, sizeof(double) * NREC * o->caprec);
  }
  memcpy(&o->rec[NREC * o->nrec], r, sizeof(double) * NREC);
  o->nrec++;
}

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
  const double tau = o->tau;

  /* 1. moments at t_n (Eqs. rho and v without the force half-shift):
   *    sum f = 1 + delta with delta = sum g; sum e f = sum e g. */
#pragma omp parallel for schedule(static)
  for (long c = 0; c < o->ncell; ++c) {
    if (o->type[c] != T_FLUID) continue;
    double s = 0, jx = 0, jy = 0, jz = 0;
    for (int i = 0; i < NQ; ++i) {
      double g = o->g[c * NQ + i];
      s += g;
      jx += EV[i][0] * g; jy += EV[i][1] * g; jz += EV[i][2] * g;
    }
    o->D[c] = s;
    o->j[3 * c] = jx; o->j[3 * c + 1] = jy; o->j[3 * c + 2] = jz;
  }

  /* 2. flux and mean gauge pressure on the first fluid layer of each plane */
  double Qp[2] = {0, 0}, Pm[2] = {0, 0};
  for (int side = 0; side < 2; ++side) {
    int zl = side == 0 ? 1 : nz - 2, zg = side == 0 ? 0 : nz - 1;
    int gt = side == 0 ? T_INLET : T_OUTLET;
    long cnt = 0;
    double q = 0, ps = 0;
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        if (zl < 0 || zl >= nz) continue;
        long c = cidx(o, x, y, zl);
        if (o->type[c] != T_FLUID || o->type[cidx(o, x, y, zg)] != gt) continue;
        q += o->j[3 * c + 2] / (1.0 + o->D[c]); /* sum e f / sum f, dA = 1 */
        ps += CS2 * o->D[c];                     /* P - c_s^2 */
        cnt++;
      }
    Qp[side] = q;
    Pm[side] = cnt ? ps / cnt : 0.0;
    o->bc[side].area = (double)cnt;
  }

  /* 3. 0D models to t_{n+1} */
  bc_update(&o->bc[0], n, Qp[0], Pm[0]);
  bc_update(&o->bc[1], n, Qp[1], Pm[1]);
  bc_update(&o->bc[2], n, 0.0, 0.0);
  if (o->bc[0].snap) { /* v0(x_f) = v(x_f, T_d) on the inlet layer */
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        long c = cidx(o, x, y, 1);
        for (int a = 0; a < 3; ++a)
          o->v0[3 * ((long)x + (long)nx * y) + a] = (o->type[c] == T_FLUID) ? o->j[3 * c + a] / RHO0 : 0.0;
      }
  }

  /* 4. immersed boundary force b(t_n) */
  memset(o->b, 0, sizeof(double) * 3 * o->ncell);
  if (o->np > 0) {
    double* u = (double*)malloc(sizeof(double) * 3 * o->ncell);
    for (long c = 0; c < 3 * o->ncell; ++c) u[c] = o->j[c] / RHO0;
#pragma omp parallel for schedule(static)
    for (long p = 0; p < o->np; ++p) {
      ib_interp_one(o, &o->X[3 * p], u, &o->Vf[3 * p]);
      for (int a = 0; a < 3; ++a) {
        double Vs = o->X[3 * p + a] - o->Xp[3 * p + a];
        double d = o->Vf[3 * p + a] - Vs;
        o->slip[3 * p + a] += d;
        o->F[3 * p + a] = o->alpha * o->slip[3 * p + a] + o->beta * d; /* on the fluid */
      }
    }
    for (long p = 0; p < o->np; ++p) ib_spread_one(o, &o->X[3 * p], &o->F[3 * p], o->area, o->b);
    free(u);
  }
  if (o->body[0] != 0.0 || o->body[1] != 0.0 || o->body[2] != 0.0) {
    double cf = cos(o->body_omega * (double)n);
    for (long c = 0; c < o->ncell; ++c)
      if (o->type[c] == T_FLUID)
        for (int a = 0; a < 3; ++a) o->b[3 * c + a] += o->body[a] * cf;
  }

  /* 5. collision (Eq. fi, collision part) */
#pragma omp parallel for schedule(static)
  for (long c = 0; c < o->ncell; ++c) {
    if (o->type[c] != T_FLUID) continue;
    double v[3];
    for (int a = 0; a < 3; ++a) v[a] = o->j[3 * c + a] / RHO0 + o->b[3 * c + a] / (2.0 * RHO0);
    for (int a = 0; a < 3; ++a) o->v[3 * c + a] = v[a];
    for (int i = 0; i < NQ; ++i) {
      double gi = o->g[c * NQ + i];
      double ge = geq(i, o->D[c], v);
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
      double out;
      if (t == T_FLUID) {
        out = o->gs[s * NQ + i];
      } else if (t == T_SOLID) {
        out = o->gs[c * NQ + opp(i)];
      } else {
        /* Eq. Non-equilibrium3 with x_f = c: boundary equilibrium at (P*, v*)
         * plus the relaxed non-equilibrium part and forcing of x_f. */
        const orc_bc* bc = &o->bc[t == T_INLET ? 0 : (t == T_OUTLET ? 1 : 2)];
        double Dst, vst[3]; /* P* / c_s^2 - 1 and v* */
        const double* vf = &o->v[3 * c];
        if (bc->vmode == 0) { /* pressure type: (P_0D, v(x_f)) */
          Dst = bc->pstar / CS2;
          for (int a = 0; a < 3; ++a) vst[a] = vf[a];
        } else { /* velocity type: (P(x_f), v_0D) */
          Dst = o->D[c];
          if (bc->kind == K_LV) { /* Eq. vnew: v0(x_f, T_d) S(t_{n+1}) */
            const double* w0 = &o->v0[3 * ((long)x + (long)nx * y)];
            for (int a = 0; a < 3; ++a) vst[a] = w0[a] * bc->S;
          } else if (bc->kind == K_WK3) {
            vst[0] = vf[0]; vst[1] = vf[1]; vst[2] = vf[2] + bc->vconst;
          } else {
            vst[0] = 0.0; vst[1] = 0.0; vst[2] = bc->vconst;
          }
        }
        out = geq(i, Dst, vst) +
              (1.0 - 1.0 / tau) * (o->g[c * NQ + i] - geq(i, o->D[c], vf)) +
              forcing(i, tau, vf, &o->b[3 * c]);
      }
      o->gn[c * NQ + i] = out;
    }
  }
  double* tmp = o->g; o->g = o->gn; o->gn = tmp;

  /* 7. wall position to t_{n+1}: central difference in time */
  if (o->np > 0) {
    double* Fel = (double*)malloc(sizeof(double) * 3 * o->np);
    membrane_force(o, o->X, Fel);
    for (long p = 0; p < o->np; ++p) {
      long k = p / o->nth;
      for (int a = 0; a < 3; ++a) {
        double xn = o->X[3 * p + a];
        double xnew = (k == 0 || k == o->nzl - 1)
                          ? xn
                          : 2.0 * xn - o->Xp[3 * p + a] + (Fel[3 * p + a] - o->F[3 * p + a]) / o->mass;
        o->Xp[3 * p + a] = xn;
        o->X[3 * p + a] = xnew;
      }
    }
    free(Fel);
  }

  double r[NREC];
  r[0] = (double)n;
  r[1] = Qp[0]; r[2] = Pm[0]; r[3] = Qp[1]; r[4] = Pm[1];
  r[5] = o->bc[0].vmode;
  r[6] = o->bc[0].vmode == 0 ? o->bc[0].pstar : (o->bc[0].kind == K_LV ? o->bc[0].S : o->bc[0].vconst);
  r[7] = o->bc[1].vmode;
  r[8] = o->bc[1].vmode == 0 ? o->bc[1].pstar : o->bc[1].vconst;
  r[9] = o->bc[0].kind == K_LV ? o->bc[0].Pv : 0.0;
  r[10] = o->bc[1].kind == K_WK3 ? o->bc[1].Pw : 0.0;
  r[11] = o->bc[0].kind == K_LV ? (double)o->bc[0].open : 0.0;
  record(o, r);
  o->step++;
}

void orc_step(void* ov, long nsteps) {
  orc_t* o = (orc_t*)ov;
  for (long k = 0; k < nsteps; ++k) one_step(o);
}

/* gauge pressure p = c_s^2 sum g and first moment sum e_i g_i of every cell
 * (0 off-fluid) */
void orc_get_fields(void* ov, double* p, double* u) {
  orc_t* o = (orc_t*)ov;
  for (long c = 0; c < o->ncell; ++c) {
    double s = 0, j[3] = {0, 0, 0};
    if (o->type[c] == T_FLUID)
      for (int i = 0; i < NQ; ++i) {
        double g = o->g[c * NQ + i];
        s += g;
        for (int a = 0; a < 3; ++a) j[a] += EV[i][a] * g;
      }
    if (p) p[c] = CS2 * s;
    if (u) for (int a = 0; a < 3; ++a) u[3 * c + a] = j[a];
  }
}

/* last Eulerian force field b (dense [cell][3]) */
void orc_get_force(void* ov, double* b) {
  orc_t* o = (orc_t*)ov;
  memcpy(b, o->b, sizeof(double) * 3 * o->ncell);
}

long orc_get_waveforms(void* ov, double* out, long cap) {
  orc_t* o = (orc_t*)ov;
  long n = o->nrec < cap ? o->nrec : cap;
  if (out && n) memcpy(out, o->rec, sizeof(double) * NREC * n);
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
