/* Axisymmetric lattice Boltzmann solver on one MI355X (gfx950): the paper's
 * 3D-axisymmetric variant (Sec. "Lattice Boltzmann method", Eqs. Afi and
 * AH1) -- an incompressible D2Q9 BGK model in the pseudo-Cartesian (x, r)
 * coordinates of an axisymmetric flow with the source H_i of Eq. Afi,
 * coupled at its inlet and outlet to the 0D models of Sec. 2.1.2 (LV
 * elastance with valve and smoothing, 3-element Windkessel, constants)
 * through the non-equilibrium extrapolation of Eq. Non-equilibrium3, in the
 * order of Algorithm 1.  Rigid walls (half-way bounce-back).
 *
 * Model.  Populations are stored shifted, g_i = f_i - w_i; D = sum g,
 * j = sum e g, rho_0 = 1; the gauge pressure read from the lattice is
 * p = D / 3 - j_r / (6 r) (the explicit mass source leaves a pressure shift
 * of half its isotropic second moment).  Each step: (1) the flux
 * Q = sum_j 2 pi r_j j_x / (1 + D) and the ring-area-weighted mean gauge
 * pressure of the inlet column 1, the outlet column nx-2 and the mid column
 * nx/2 (FP64); (2) the 0D updates (FP64);
 * (3) per fluid node the body force F = (F_x, F_r),
 *   F_x = -u_x u_r / r + (nu / r)(d_r u_x + d_x u_r) + G,
 *   F_r = -u_r^2 / r + (2 nu / r) d_r u_r - 2 nu u_r / r^2,
 * from the unforced velocities u = j (central differences; mirror values at
 * the axis, the quadratic through the wall's zero next to a wall,
 * second-order one-sided differences next to the inlet / outlet columns;
 * G = G0 cos(omega t) an optional axial body force); (4) BGK collision with
 * the forced velocity u = j + F/2, Guo's forcing term and the mass source
 * H_i = -w_i u_r / r, pull streaming with half-way bounce-back at SOLID
 * nodes and past the last row, the mirror at the axis (r = 0 half way below
 * row 0) and the extrapolation at the ghost columns (x_f the ghost's fluid
 * neighbour along x).  The first-order source is the printed h1; the
 * second-order term of Eq. AH1 is garbled in the available text, and its
 * role -- the difference between the axisymmetric Navier-Stokes equations
 * and what the planar model with the mass source recovers -- is played by F.
 *
 * Geometry.  Node (i, j), i = 0..nx-1 along x, j = 0..nr-1 along r at
 * r_j = j + 1/2; node index i + nx j.  Node types (same codes as the 3D
 * solver): 0 FLUID, 1 SOLID, 2 INLET (column 0 only), 3 OUTLET (column nx-1
 * only).  With periodic_x the x direction wraps and no ghost column exists.
 */
#ifndef LBM_AXI_H
#define LBM_AXI_H

#include <stddef.h>
#include <stdint.h>

#include "lbm0d3d.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_axi lbm_axi;

typedef struct {
  int32_t nx, nr;          /* columns (x) >= 5, rows (r) >= 2 */
  double tau;              /* BGK relaxation time, > 0.5 */
  int32_t precision;       /* LBM_FP64 or LBM_FP32 (populations, moments and
                              force; the 0D models and the column sums run in
                              FP64 either way) */
  const uint8_t* flags;    /* host, nr * nx node types; copied by lbm_axi_init */
  int32_t periodic_x;      /* 1: x wraps (no inlet / outlet columns) */
  int32_t wave_cap;        /* waveform ring capacity in steps, 0 = 4096 */
  double p_ref;            /* reference gauge pressure: the device keeps
                              g - w_i 3 p_ref (exact change of variables, f_eq
                              linear in P); values in and out are still g */
} lbm_axi_config;

/* Device bytes a context over cfg needs.  Errors: LBM_E_INVAL (sizes, tau,
 * precision, node types: INLET off column 0, OUTLET off column nx-1, a
 * FLUID node in a ghost column, ghosts with periodic_x). */
lbm_status lbm_axi_query_size(const lbm_axi_config* cfg, size_t* bytes);

/* Create a context on the caller's device buffer (>= the queried bytes,
 * owned by the caller, kept for the context's life) and HIP stream (NULL =
 * default).  Populations start at rest (g = 0), both boundaries at
 * PRESSURE_CONST 0.  Synchronises.  Errors: LBM_E_INVAL, LBM_E_DEVICE. */
lbm_status lbm_axi_init(const lbm_axi_config* cfg, void* dev_buf, size_t bytes, void* hip_stream, lbm_axi** out);

/* 0D model of the inlet (boundary 0) or the outlet (1): kind and parameters
 * as lbm_couple_0d (lbm_bc_kind; the LV only at the inlet).  The
 * pressure-driven Windkessel spreads its flux deficit over the column's ring
 * area sum 2 pi r_j.  Synchronises.  Errors: LBM_E_INVAL. */
lbm_status lbm_axi_couple_0d(lbm_axi* ctx, int32_t boundary, int32_t kind, const double* params, int32_t nparams,
                             const double* state, int32_t nstate);

/* Axial body force G0 cos(omega t) (t in steps) on every fluid node. */
lbm_status lbm_axi_set_body_force(lbm_axi* ctx, double G0, double omega);

/* Every fluid node at rest at gauge pressure p.  Synchronises. */
lbm_status lbm_axi_set_rest(lbm_axi* ctx, double p);

/* Populations g = f - w as host doubles, [node][9] in the D2Q9 order
 * (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1) of (e_x, e_r).
 * Synchronise.  Errors: LBM_E_INVAL (NULL). */
lbm_status lbm_axi_write_populations(lbm_axi* ctx, const double* g);
lbm_status lbm_axi_read_populations(lbm_axi* ctx, double* g);

/* Advance nsteps steps (asynchronous).  Errors: LBM_E_INVAL (nsteps < 0). */
lbm_status lbm_axi_step(lbm_axi* ctx, int64_t nsteps);

/* Gauge pressure and forced velocity (u_x, u_r) = j + F/2 of every node of
 * the current state, host arrays of nr * nx doubles (zero at non-fluid
 * nodes; any pointer may be NULL).  Synchronises. */
lbm_status lbm_axi_read_fields(lbm_axi* ctx, double* p, double* ux, double* ur);

/* The last min(steps, cap, wave_cap) waveform records in step order, 14
 * doubles each: step, Q_in, P_in, Q_out, P_out, inlet coupling type
 * (0 pressure / 1 velocity), inlet P* or (LV) S or v*, outlet coupling type,
 * outlet P* or v*, ventricle P_v, outlet Windkessel P_w, valve open, Q and P
 * of the mid column.  *n receives the number written.  Synchronises. */
lbm_status lbm_axi_read_waveforms(lbm_axi* ctx, double* out, int64_t cap, int64_t* n);

/* Synchronise; LBM_E_UNSTABLE once a column sum became non-finite. */
lbm_status lbm_axi_sync(lbm_axi* ctx);

/* Message of the last failed call on ctx (or of the last failed
 * query / init when ctx is NULL). */
const char* lbm_axi_last_error(const lbm_axi* ctx);

lbm_status lbm_axi_destroy(lbm_axi* ctx);

#ifdef __cplusplus
}
#endif

#endif
