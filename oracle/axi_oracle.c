/* Axisymmetric lattice Boltzmann oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain CPU implementation of the paper's 3D-axisymmetric variant (Sec.
 * "Lattice Boltzmann method", Eqs. Afi and AH1): an incompressible D2Q9 BGK
 * model in the pseudo-Cartesian coordinates (x, r) of an axisymmetric flow,
 * with the source H_i of Eq. Afi, coupled at its inlet and outlet to the 0D
 * models of Sec. 2.1.2 through the non-equilibrium extrapolation of Eq.
 * Non-equilibrium3.  Only tests/ and the bench's CPU baseline use it; it
 * shares nothing with the HIP path.  The 0D models are the ones of
 * lbm_oracle.c, reached through their public entry points.
 *
 * Reading of Eq. AH1.  The first-order source h1_i = -w_i rho u_r / r is taken
 * as printed (rho -> rho_0 = 1, the incompressible model): summed over i it
 * is the axisymmetric continuity's extra term -u_r / r.  The second-order
 * term h2 is garbled in the text available (a derivative along y in (x, r)
 * coordinates, an unclear grouping of the velocity products), so the terms
 * it exists for -- the difference between the axisymmetric incompressible
 * Navier-Stokes equations and what the planar D2Q9 model recovers with the
 * mass source -- enter as a body force with Guo's forcing term:
 *   F_x = -u_x u_r / r + (nu / r) (d_r u_x + d_x u_r)
 *   F_r = -u_r^2 / r + (2 nu / r) d_r u_r - 2 nu u_r / r^2
 * (the planar model with the source recovers d_t u + div(u u) = -grad p +
 * nu div(grad u + grad u^T); the axisymmetric equations have u . grad u,
 * nu lap u + (nu / r) d_r u - nu u_r e_r / r^2 instead, and
 * div u = -u_r / r makes up the rest).
 *
 * Pressure.  The explicit source's isotropic second moment (1/3) S, with
 * S = -u_r / r, survives the time discretisation at half strength as a
 * pressure: the lattice's D / 3 is the flow's pressure minus S / 6, a
 * gradient the velocity field does not see.  Every pressure read from the
 * lattice (the column means handed to the 0D models, the field output) is
 * therefore p = D / 3 - j_r / (6 r).  (Entering +grad(S) / 6 as a force
 * instead removes the shift but makes the first row's u_r feed itself at
 * small nu: unstable at tau = 0.51.)  Derivatives: central differences of
 * the unforced velocity; at the axis the mirror values (u_x even, u_r odd);
 * next to a wall the quadratic through the two nearest nodes and the wall's
 * zero (the wall sits half way, as bounce-back places it); next to an
 * inlet / outlet column one-sided second-order differences.
 *
 * Lattice: nodes (i, j), i = 0..nx-1 along x, j = 0..nr-1 along r at
 * r_j = j + 1/2 (the axis r = 0 lies half way below row 0, a mirror); rows
 * j >= nr and SOLID nodes are walls (half-way bounce-back).  Column 0 holds
 * the INLET ghosts and column nx-1 the OUTLET ghosts (or the x direction is
 * periodic).  Populations are stored shifted, g_i = f_i - w_i; D = sum g =
 * 3 p (p gauge), j = sum e g; rho_0 = 1.
 *
 * One step (Algorithm 1's order): moments; flux Q = sum 2 pi r u_x (u_x =
 * j_x / sum f, as in the 3D solver) and ring-area-weighted mean pressure (as
 * below) of
 * the inlet column 1, the outlet column nx-2 and the mid column nx/2; the 0D
 * updates; the axisymmetric force from the unforced velocities; collision
 * with F_i (Guo) and H_i = -w_i u_r / r (u the forced velocity) and pull
 * streaming with bounce-back, the axis mirror and the extrapolation at the
 * ghost columns (x_f the ghost's neighbour along x; the extrapolated value
 * carries x_f's force and source terms).
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

#define AQ 9
#define API (4 * atan((real)1))
#define AREC 14
enum { A_FLUID = 0, A_SOLID = 1, A_INLET = 2, A_OUTLET = 3 };

/* D2Q9 (x, r): rest, 4 axes, 4 diagonals */
static const int AE[AQ][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1}, {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
static const int AOPP[AQ] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const int AMIR[AQ] = {0, 1, 4, 3, 2, 8, 7, 6, 5}; /* e_r -> -e_r */

/* 0D models of lbm_oracle.c */
void* orc_bc_new(int boundary, int kind, const double* par, int npar, const double* st, int nst);
void orc_bc_free(void* c);
void orc_bc_update(void* c, long n, double Qp, double Pbar, double* out);
double orc_bc_vconst(void* c);
void orc_bc_set_area(void* c, double area);

typedef struct {
  int nx, nr, px;
  long n;
  real tau, nu;
  real w[AQ];
  uint8_t* type;         /* [j][i] */
  real *g, *gn;          /* [node][9] */
  real *D, *jx, *jr;     /* moments: D = 3 p, unforced j */
  real *Fx, *Fr;         /* axisymmetric force (+ body force) */

  real *v0;              /* inlet snapshot per row (x, r) at valve closure */
  void* bc[2];
  int kind[2];
  double out[2][8];
  double vc[2];
  real G0, omega;        /* body force G0 cos(omega t) along x */
  long step;
  double* rec;
  long nrec, cap;
} axo_t;

static long NI(const axo_t* o, int i, int j) { return i + (long)o->nx * j; }
static real rj(int j) { return (real)j + (real)0.5; }

static real aeq(const axo_t* o, int k, real D, real ux, real ur) {
  real eu = AE[k][0] * ux + AE[k][1] * ur;
  return o->w[k] * (D + 3 * eu + (real)4.5 * eu * eu - (real)1.5 * (ux * ux + ur * ur));
}
/* Guo's forcing term with the forced velocity (ux, ur) and force (fx, fr) */
static real aforce(const axo_t* o, int k, real ux, real ur, real fx, real fr) {
  real ex = AE[k][0], er = AE[k][1];
  real eu = ex * ux + er * ur;
  return (1 - 1 / (2 * o->tau)) * o->w[k] * (3 * ((ex - ux) * fx + (er - ur) * fr) + 9 * eu * (ex * fx + er * fr));
}

void* axo_create(int nx, int nr, double tau, const uint8_t* flags, int periodic_x) {
  axo_t* o = (axo_t*)calloc(1, sizeof(axo_t));
  o->nx = nx; o->nr = nr; o->px = periodic_x;
  o->n = (long)nx * nr;
  o->tau = tau;
  o->nu = (o->tau - (real)0.5) / 3;
  o->w[0] = (real)4 / 9;
  for (int k = 1; k < 5; ++k) o->w[k] = (real)1 / 9;
  for (int k = 5; k < 9; ++k) o->w[k] = (real)1 / 36;
  o->type = (uint8_t*)malloc(o->n);
  memcpy(o->type, flags, o->n);
  o->g = (real*)calloc(o->n * AQ, sizeof(real));
  o->gn = (real*)calloc(o->n * AQ, sizeof(real));
  o->D = (real*)calloc(o->n, sizeof(real));
  o->jx = (real*)calloc(o->n, sizeof(real));
  o->jr = (real*)calloc(o->n, sizeof(real));
  o->Fx = (real*)calloc(o->n, sizeof(real));
  o->Fr = (real*)calloc(o->n, sizeof(real));
  o->v0 = (real*)calloc(2 * (size_t)nr, sizeof(real));
  double p0 = 0;
  o->bc[0] = orc_bc_new(0, 0, &p0, 1, NULL, 0);
  o->bc[1] = orc_bc_new(1, 0, &p0, 1, NULL, 0);
  return o;
}

void axo_destroy(void* ov) {
  axo_t* o = (axo_t*)ov;
  free(o->type); free(o->g); free(o->gn); free(o->D); free(o->jx); free(o->jr);
  free(o->Fx); free(o->Fr); free(o->v0); free(o->rec);
  orc_bc_free(o->bc[0]);
  orc_bc_free(o->bc[1]);
  free(o);
}

/* 0D model of the inlet (boundary 0) or the outlet (1); kinds and parameters
 * as in lbm_oracle.c.  The ring area of the boundary column (sum 2 pi r_j over
 * its fluid rows) turns the pressure-driven Windkessel's flux deficit into
 * the axial correction. */
void axo_set_bc(void* ov, int boundary, int kind, const double* par, int npar, const double* st, int nst) {
  axo_t* o = (axo_t*)ov;
  orc_bc_free(o->bc[boundary]);
  o->bc[boundary] = orc_bc_new(boundary, kind, par, npar, st, nst);
  o->kind[boundary] = kind;
  int col = boundary == 0 ? 1 : o->nx - 2;
  real area = 0;
  for (int j = 0; j < o->nr; ++j)
    if (o->type[NI(o, col, j)] == A_FLUID) area += 2 * API * rj(j);
  orc_bc_set_area(o->bc[boundary], (double)area);
}

void axo_set_body_force(void* ov, double G0, double omega) {
  axo_t* o = (axo_t*)ov;
  o->G0 = G0;
  o->omega = omega;
}

void axo_set_rest(void* ov, double p) {
  axo_t* o = (axo_t*)ov;
  for (long c = 0; c < o->n; ++c)
    for (int k = 0; k < AQ; ++k) o->g[c * AQ + k] = o->type[c] == A_FLUID ? o->w[k] * 3 * (real)p : 0;
}

void axo_set_pops(void* ov, const double* g) {
  axo_t* o = (axo_t*)ov;
  for (long k = 0; k < o->n * AQ; ++k) o->g[k] = g[k];
}
void axo_get_pops(void* ov, double* g) {
  axo_t* o = (axo_t*)ov;
  for (long k = 0; k < o->n * AQ; ++k) g[k] = (double)o->g[k];
}

/* node type with the walls past the last row; rows below the axis are
 * reported as fluid only through the mirror, never here */
static int atype(const axo_t* o, int i, int j) {
  if (j >= o->nr) return A_SOLID;
  if (o->px) i = (i + o->nx) % o->nx;
  if (i < 0 || i >= o->nx) return A_SOLID;
  return o->type[NI(o, i, j)];
}

/* d/dr of component a (0: x, 1: r) of the unforced velocity at fluid node (i, j) */
static real ddr(const axo_t* o, const real* u, int odd, int i, int j) {
  real uc = u[NI(o, i, j)];
  int up = atype(o, i, j + 1) == A_FLUID;
  int dn = j == 0 ? 1 : atype(o, i, j - 1) == A_FLUID;
  real uu = up ? u[NI(o, i, j + 1)] : 0, ud = 0;
  if (j == 0) ud = odd ? -uc : uc;   /* mirror row below the axis */
  else if (dn) ud = u[NI(o, i, j - 1)];
  if (up && dn) return (uu - ud) / 2;
  /* wall half way above (below): the quadratic through the neighbour on the
   * other side, the node and the wall's zero */
  if (dn) return -ud / 3 - uc;
  if (up) return uu / 3 + uc;
  return 0;
}

static int axfluid(const axo_t* o, int i, int j) {
  if (o->px) i = (i + o->nx) % o->nx;
  return i >= 0 && i < o->nx && o->type[NI(o, i, j)] == A_FLUID;
}
static real uat(const axo_t* o, const real* u, int i, int j) {
  if (o->px) i = (i + o->nx) % o->nx;
  return u[NI(o, i, j)];
}

/* d/dx of a velocity component at fluid node (i, j) */
static real ddx(const axo_t* o, const real* u, int i, int j) {
  int l = axfluid(o, i - 1, j), r = axfluid(o, i + 1, j);
  if (l && r) return (uat(o, u, i + 1, j) - uat(o, u, i - 1, j)) / 2;
  if (r && axfluid(o, i + 2, j))
    return (-3 * u[NI(o, i, j)] + 4 * uat(o, u, i + 1, j) - uat(o, u, i + 2, j)) / 2;
  if (l && axfluid(o, i - 2, j))
    return (3 * u[NI(o, i, j)] - 4 * uat(o, u, i - 1, j) + uat(o, u, i - 2, j)) / 2;
  return 0;
}

static void record(axo_t* o, const double* r) {
  if (o->nrec == o->cap) {
    o->cap = o->cap ? 2 * o->cap : 1024;
    o->rec = (double*)realloc(o->rec, sizeof(double) * AREC * o->cap);
  }
  memcpy(o->rec + AREC * o->nrec, r, sizeof(double) * AREC);
  o->nrec++;
}

/* flux and mean gauge pressure of column col */
static void column(const axo_t* o, int col, real* Q, real* P) {
  real q = 0, pa = 0, a = 0;
  for (int j = 0; j < o->nr; ++j) {
    long c = NI(o, col, j);
    if (o->type[c] != A_FLUID) continue;
    real dA = 2 * API * rj(j);
    q += dA * o->jx[c] / (1 + o->D[c]);
    pa += dA * (o->D[c] / 3 - o->jr[c] / (6 * rj(j)));
    a += dA;
  }
  *Q = q;
  *P = a > 0 ? pa / a : 0;
}

/* axisymmetric force at fluid node (i, j) from the unforced velocities, with
 * the uniform axial body force G */
static void axforce(const axo_t* o, int i, int j, real G, real* Fx, real* Fr) {
  long c = NI(o, i, j);
  real r = rj(j), ux = o->jx[c], ur = o->jr[c], nu = o->nu;
  real dux_dr = ddr(o, o->jx, 0, i, j), dur_dr = ddr(o, o->jr, 1, i, j), dur_dx = ddx(o, o->jr, i, j);
  *Fx = -ux * ur / r + nu / r * (dux_dr + dur_dx) + G;
  *Fr = -ur * ur / r + 2 * nu / r * dur_dr - 2 * nu * ur / (r * r);
}

/* post-collision value of direction k at fluid node c: BGK with Guo's term
 * for the force (Fx, Fr) and the mass source -w_k u_r / r, u the forced velocity */
static real post(const axo_t* o, long c, int k) {
  real fx = o->Fx[c], fr = o->Fr[c];
  real ux = o->jx[c] + fx / 2, ur = o->jr[c] + fr / 2;
  real gk = o->g[c * AQ + k];
  return gk - (gk - aeq(o, k, o->D[c], ux, ur)) / o->tau + aforce(o, k, ux, ur, fx, fr) -
         o->w[k] * ur / rj((int)(c / o->nx));
}

static void one_step(axo_t* o) {
  const int nx = o->nx, nr = o->nr;
  const long n = o->step;
  const real tau = o->tau;
  /* 1. moments */
  for (long c = 0; c < o->n; ++c) {
    real D = 0, jx = 0, jr = 0;
    if (o->type[c] == A_FLUID)
      for (int k = 0; k < AQ; ++k) {
        real gk = o->g[c * AQ + k];
        D += gk;
        jx += AE[k][0] * gk;
        jr += AE[k][1] * gk;
      }
    o->D[c] = D; o->jx[c] = jx; o->jr[c] = jr;
  }
  /* 2.-3. boundary columns and the 0D models */
  real Qi = 0, Pi = 0, Qo = 0, Po = 0, Qm = 0, Pm = 0;
  if (!o->px) {
    column(o, 1, &Qi, &Pi);
    column(o, nx - 2, &Qo, &Po);
    orc_bc_update(o->bc[0], n, (double)Qi, (double)Pi, o->out[0]);
    orc_bc_update(o->bc[1], n, (double)Qo, (double)Po, o->out[1]);
    o->vc[0] = orc_bc_vconst(o->bc[0]);
    o->vc[1] = orc_bc_vconst(o->bc[1]);
    if (o->out[0][6] != 0) /* valve closure: snapshot of the inlet column's velocity */
      for (int j = 0; j < nr; ++j) {
        long c = NI(o, 1, j);
        o->v0[2 * j] = o->jx[c];
        o->v0[2 * j + 1] = o->jr[c];
      }
  }
  column(o, nx / 2, &Qm, &Pm);
  /* 4. axisymmetric force */
  real G = o->G0 * cos(o->omega * (real)n);
  for (int j = 0; j < nr; ++j)
    for (int i = 0; i < nx; ++i) {
      long c = NI(o, i, j);
      if (o->type[c] != A_FLUID) { o->Fx[c] = o->Fr[c] = 0; continue; }
      axforce(o, i, j, G, &o->Fx[c], &o->Fr[c]);
    }
  /* 5. collision and pull streaming */
  for (int j = 0; j < nr; ++j)
    for (int i = 0; i < nx; ++i) {
      long c = NI(o, i, j);
      if (o->type[c] != A_FLUID) continue;
      for (int k = 0; k < AQ; ++k) {
        int si = i - AE[k][0], sj = j - AE[k][1], kk = k;
        if (sj < 0) { sj = 0; kk = AMIR[k]; }   /* across the axis: mirror image */
        if (o->px) si = (si + nx) % nx;
        int st = atype(o, si, sj);
        real v;
        if (st == A_FLUID) {
          v = post(o, NI(o, si, sj), kk);
        } else if (st == A_SOLID) {
          v = post(o, c, AOPP[k]);
        } else {
          /* ghost: extrapolation from its neighbour along x */
          int b = st == A_INLET ? 0 : 1;
          int fi = b == 0 ? si + 1 : si - 1;
          long xf = atype(o, fi, sj) == A_FLUID ? NI(o, fi, sj) : c;
          real fx = o->Fx[xf], fr = o->Fr[xf];
          real ux = o->jx[xf] + fx / 2, ur = o->jr[xf] + fr / 2;
          real Dst, vx, vr;
          if (o->out[b][0] == 0) { /* pressure type: (P*, v(x_f)) */
            Dst = 3 * (real)o->out[b][1];
            vx = ux; vr = ur;
          } else {                 /* velocity type: (P(x_f), v*) */
            Dst = o->D[xf];
            if (o->kind[b] == 3) {   /* LV after closure: the snapshot times S (S = 0 before) */
              real S = (real)o->out[b][2];
              vx = o->v0[2 * sj] * S;
              vr = o->v0[2 * sj + 1] * S;
            } else if (o->kind[b] == 2) {   /* pressure-driven Windkessel: v(x_f) + dv e_x */
              vx = ux + (real)o->vc[b];
              vr = ur;
            } else {                        /* constant velocity */
              vx = (real)o->vc[b];
              vr = 0;
            }
          }
          real gk = o->g[xf * AQ + kk];
          v = aeq(o, kk, Dst, vx, vr) + (1 - 1 / tau) * (gk - aeq(o, kk, o->D[xf], ux, ur)) +
              aforce(o, kk, ux, ur, fx, fr) - o->w[kk] * ur / rj((int)(xf / nx));
        }
        o->gn[c * AQ + k] = v;
      }
    }
  real* t = o->g; o->g = o->gn; o->gn = t;
  double r[AREC] = {(double)n, (double)Qi, (double)Pi, (double)Qo, (double)Po,
                    o->out[0][0], o->out[0][0] == 0 ? o->out[0][1] : (o->out[0][3] != 0 ? o->out[0][2] : o->vc[0]),
                    o->out[1][0], o->out[1][0] == 0 ? o->out[1][1] : o->vc[1],
                    o->out[0][3], o->out[1][4], o->out[0][5], (double)Qm, (double)Pm};
  record(o, r);
  o->step++;
}

void axo_step(void* ov, long nsteps) {
  for (long s = 0; s < nsteps; ++s) one_step((axo_t*)ov);
}

/* gauge pressure and the forced velocity u = j + F/2 of the last step's
 * state (the force from this state's unforced velocities), per node */
void axo_get_fields(void* ov, double* p, double* ux, double* ur) {
  axo_t* o = (axo_t*)ov;
  for (long c = 0; c < o->n; ++c) {
    real D = 0, jx = 0, jr = 0;
    if (o->type[c] == A_FLUID)
      for (int k = 0; k < AQ; ++k) {
        real gk = o->g[c * AQ + k];
        D += gk;
        jx += AE[k][0] * gk;
        jr += AE[k][1] * gk;
      }
    o->D[c] = D; o->jx[c] = jx; o->jr[c] = jr;
  }
  real G = o->G0 * cos(o->omega * (real)o->step);
  for (int j = 0; j < o->nr; ++j)
    for (int i = 0; i < o->nx; ++i) {
      long c = NI(o, i, j);
      p[c] = (double)(o->D[c] / 3 - (o->type[c] == A_FLUID ? o->jr[c] / (6 * rj(j)) : 0));
      if (o->type[c] != A_FLUID) { ux[c] = ur[c] = 0; continue; }
      real fx, fr;
      axforce(o, i, j, G, &fx, &fr);
      ux[c] = (double)(o->jx[c] + fx / 2);
      ur[c] = (double)(o->jr[c] + fr / 2);
    }
}

long axo_get_waveforms(void* ov, double* out, long cap) {
  axo_t* o = (axo_t*)ov;
  long m = o->nrec < cap ? o->nrec : cap;
  if (out && m) memcpy(out, o->rec, sizeof(double) * AREC * m);
  return o->nrec;
}
