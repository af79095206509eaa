/* The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (and the
 * leak checker): one workload read from a file written by the test, run for
 * a few steps through every entry point the tests use, then the standalone
 * 0D, wall and lattice helpers.
 *
 * File layout (native endianness): int32 nx, ny, nz; nx*ny*nz cell-type
 * bytes; double tau; int32 nee_variant; int32 nbc, then per boundary int32
 * boundary, kind, npar, nstate and the doubles par[npar], state[nstate];
 * double p_init; int32 has_wall, and with a wall int32 n_theta, n_z, the
 * doubles X0[3 n_theta n_z], ds_theta, ds_z, area, k, ei, mass, alpha, beta,
 * int32 kernel, shell, double poisson; int32 steps. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void* orc_create(int nx, int ny, int nz, double tau, const uint8_t* flags, int px, int py, int pz);
void orc_destroy(void* o);
void orc_set_nee_variant(void* o, int v);
void orc_set_bc(void* o, int boundary, int kind, const double* par, int npar, const double* st, int nst);
void orc_set_rest(void* o, double p);
int orc_set_membrane(void* o, int nth, int nzl, const double* X0, double ds_th, double ds_z, double area,
                     double ks, double ei, double mass, double alpha, double beta);
void orc_set_wall_options(void* o, int kernel, int external);
void orc_set_shell(void* o, int shell, double poisson);
void orc_set_wall(void* o, const double* X, const double* V);
void orc_step(void* o, long n);
void orc_get_fields(void* o, double* p, double* u);
void orc_get_pops(void* o, double* g);
void orc_set_pops(void* o, const double* g);
void orc_get_force(void* o, double* b);
long orc_get_waveforms(void* o, double* out, long cap);
long orc_get_outlet_waveforms(void* o, double* out, long cap);
void orc_wss(void* o, double dist, double* out);
void orc_membrane_force(void* o, const double* X, double* F);
void orc_get_lagrangian(void* o, double* X, double* Xp, double* slip, double* Vf, double* F);
void orc_get_displacement(void* o, double* Dn, double* Dp);
void orc_ib_interp(void* o, long np, const double* X, const double* u, double* V);
void orc_ib_spread(void* o, long np, const double* X, const double* F, double area, double* b);
void* orc_bc_new(int boundary, int kind, const double* par, int npar, const double* st, int nst);
void orc_bc_free(void* c);
void orc_bc_update(void* c, long n, double Qp, double Pbar, double* out);
void orc_filament_force(int m, const double* X, double ds, double Eh, double EI, double* F);
double orc_smooth_S(double t, double t0, double Ls);
void orc_elastance(const double* p, double t, double* E, double* dE);
void orc_lattice(int* e, double* w);
void orc_feq(double p, const double* v, double* g);
void orc_forcing(double tau, const double* v, const double* b, double* F);

static FILE* in;
static void rd(void* p, size_t sz, size_t n) {
  if (fread(p, sz, n, in) != n) {
    fprintf(stderr, "short input file\n");
    exit(2);
  }
}
static int rdi(void) { int32_t v; rd(&v, 4, 1); return v; }
static double rdd(void) { double v; rd(&v, 8, 1); return v; }

int main(int argc, char** argv) {
  if (argc < 2 || !(in = fopen(argv[1], "rb"))) return 2;
  int nx = rdi(), ny = rdi(), nz = rdi();
  long nc = (long)nx * ny * nz;
  uint8_t* flags = malloc(nc);
  rd(flags, 1, nc);
  double tau = rdd();
  int nee = rdi();
  void* o = orc_create(nx, ny, nz, tau, flags, 0, 0, 0);
  orc_set_nee_variant(o, nee);
  int nbc = rdi();
  for (int b = 0; b < nbc; ++b) {
    int boundary = rdi(), kind = rdi(), npar = rdi(), nst = rdi();
    double par[16], st[4];
    if (npar > 16 || nst > 4) return 2;
    rd(par, 8, npar);
    rd(st, 8, nst);
    orc_set_bc(o, boundary, kind, par, npar, st, nst);
  }
  double p0 = rdd();
  orc_set_rest(o, p0);
  int has_wall = rdi(), np = 0;
  double *X0 = NULL, area = 1;
  if (has_wall) {
    int nth = rdi(), nzl = rdi();
    np = nth * nzl;
    X0 = malloc(sizeof(double) * 3 * np);
    rd(X0, 8, 3 * (size_t)np);
    double ds_th = rdd(), ds_z = rdd();
    area = rdd();
    double k = rdd(), ei = rdd(), mass = rdd(), alpha = rdd(), beta = rdd();
    int kernel = rdi(), shell = rdi();
    double poisson = rdd();
    orc_set_membrane(o, nth, nzl, X0, ds_th, ds_z, area, k, ei, mass, alpha, beta);
    orc_set_wall_options(o, kernel, 0);
    orc_set_shell(o, shell, poisson);
  }
  int steps = rdi();
  fclose(in);

  orc_step(o, steps);
  double* p = malloc(sizeof(double) * nc);
  double* u = malloc(sizeof(double) * 3 * nc);
  double* g = malloc(sizeof(double) * 19 * nc);
  orc_get_fields(o, p, u);
  orc_get_pops(o, g);
  orc_set_pops(o, g);
  orc_get_force(o, u);
  double* w = malloc(sizeof(double) * 14 * (steps + 1));
  double* ow = malloc(sizeof(double) * 24 * (steps + 1));
  long nw = orc_get_waveforms(o, w, steps + 1);
  long now_ = orc_get_outlet_waveforms(o, ow, steps + 1);
  if (nw != steps || now_ != steps) {
    fprintf(stderr, "waveform records: %ld %ld, want %d\n", nw, now_, steps);
    return 1;
  }
  if (has_wall) {
    double* a = malloc(sizeof(double) * 3 * np);
    double* b = malloc(sizeof(double) * 3 * np);
    double* c = malloc(sizeof(double) * 3 * np);
    double* d = malloc(sizeof(double) * 3 * np);
    double* e = malloc(sizeof(double) * 3 * np);
    orc_wss(o, 2.0, a);
    orc_membrane_force(o, X0, a);
    orc_get_lagrangian(o, a, b, c, d, e);
    orc_get_displacement(o, a, b);
    orc_get_fields(o, p, u);
    orc_ib_interp(o, np, X0, u, a);
    orc_ib_spread(o, np, X0, a, area, u);
    /* external solid: the points keep the velocity they are given */
    orc_set_wall_options(o, 1, 1);
    for (long q = 0; q < 3L * np; ++q) b[q] = 1e-3 * (q % 3 == 0);
    orc_set_wall(o, X0, b);
    orc_step(o, 3);
    free(a); free(b); free(c); free(d); free(e);
  }
  orc_destroy(o);

  /* standalone helpers */
  double lv[11] = {2.5e-4, 7.5e-6, 2000, 700, 2e-5, 150, 1.55, 0.7, 1.9, 1.17, 21.9};
  double out[8], E, dE;
  void* bc = orc_bc_new(0, 3, lv, 11, NULL, 0);
  for (long n = 0; n < 4000; ++n) orc_bc_update(bc, n, n < 2000 ? 1e-3 : -1e-4, 1e-5, out);
  orc_bc_free(bc);
  double wk[4] = {0.05, 50, 1, 0};
  for (int mode = 0; mode < 2; ++mode) {
    wk[3] = mode;
    bc = orc_bc_new(1, 2, wk, 4, &p0, 1);
    for (long n = 0; n < 100; ++n) orc_bc_update(bc, n, 1e-3, 1e-4, out);
    orc_bc_free(bc);
  }
  orc_elastance(lv, 100, &E, &dE);
  (void)orc_smooth_S(10, 0, 100);
  int e3[57];
  double wq[19], v[3] = {0.01, -0.02, 0.03}, bb[3] = {1e-5, 0, -1e-5}, gq[19];
  orc_lattice(e3, wq);
  orc_feq(1e-3, v, gq);
  orc_forcing(0.6, v, bb, gq);
  double X[3 * 12], F[3 * 12];
  for (int s = 0; s < 12; ++s) { X[3 * s] = 0.1 * s; X[3 * s + 1] = 0.01 * s * s; X[3 * s + 2] = 0; }
  orc_filament_force(12, X, 0.1, 1.0, 1e-3, F);

  free(flags); free(p); free(u); free(g); free(w); free(ow); free(X0);
  printf("oracle driver: ok\n");
  return 0;
}
