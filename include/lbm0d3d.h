/*
 * lbm0d3d.h -- C interface of the MI355X (gfx950) 0D-3D coupled lattice
 * Boltzmann library: incompressible D3Q19 BGK with forcing, non-equilibrium
 * extrapolation at 0D-coupled planes, penalty immersed boundary with an
 * elastic membrane wall (Wei, Amlani & Pahlevan, arXiv 2112.05258).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Lattice units: dx = dt = 1, c_s^2 = 1/3, rho_0 = 1.
 * - Cell (x, y, z) of an instance has index x + nx*(y + ny*z).
 * - Populations are handled shifted, g_i = f_i - w_i, in this velocity order
 *   (weights 1/3, 1/18 for the 6 faces, 1/36 for the 12 edges):
 *     0 (0,0,0)  1 (1,0,0)  2 (-1,0,0)  3 (0,1,0)  4 (0,-1,0)  5 (0,0,1)
 *     6 (0,0,-1) 7 (1,1,0)  8 (-1,-1,0) 9 (1,-1,0) 10 (-1,1,0) 11 (1,0,1)
 *     12 (-1,0,-1) 13 (1,0,-1) 14 (-1,0,1) 15 (0,1,1) 16 (0,-1,-1)
 *     17 (0,1,-1) 18 (0,-1,1)
 * - Pressures are gauge, p = P - c_s^2 (so sum f = 1 + 3p).
 * - Cell types (the flags array): FLUID 0, SOLID 1 (halfway bounce-back),
 *   INLET 2 (ghost of boundary 0, only on the plane z = 0), OUTLET 3 (ghost
 *   of an outlet, only on z = nz-1), EXTP 4 (ghost of boundary 2, the
 *   exterior, anywhere on the box faces).  Every cell on the box faces must
 *   be non-FLUID.  Several outlets (Sec. 2.1.2: each outlet has its own 0D
 *   model): an OUTLET ghost carries its outlet index k = 0..7 in bits 5-7 of
 *   its byte (LBM_CELL_OUTLET | k << 5); every other byte is a plain type.
 * - Boundaries (0D records of an instance): 0 inlet, 1 outlet 0, 2 exterior,
 *   2 + k outlet k (k = 1..7).
 *
 * Memory and streams: the caller owns every device buffer (allocate with any
 * allocator, e.g. torch) and the HIP stream.  A context only borrows them;
 * they must outlive it.  Calls that only enqueue work are asynchronous on the
 * stream; calls that return data synchronise the stream first.  lbm_destroy
 * frees host memory only.  One context per host thread.
 *
 * Errors: every call returns an lbm_status; nothing throws across the
 * interface; lbm_last_error() gives a message for the last failure of a
 * context.
 */
#ifndef LBM0D3D_H
#define LBM0D3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
  LBM_OK = 0,
  LBM_E_INVAL = -1,       /* bad argument, size or geometry */
  LBM_E_DEVICE = -2,      /* a HIP call failed */
  LBM_E_UNSTABLE = -3,    /* a boundary flux or pressure became non-finite */
  LBM_E_STATE = -4,       /* call not valid in the current state */
  LBM_E_UNSUPPORTED = -5, /* option not built into this library */
  LBM_E_BAND = -6         /* a wall point left the band of cells set up for it */
} lbm_status;

typedef enum {
  LBM_FP64 = 0,  /* populations stored and collided in FP64 */
  LBM_FP32 = 1,  /* stored and collided in FP32 */
  LBM_FP16S = 2, /* stored as FP16 of s*g (s = power of two), collided in FP32 */
  LBM_BF16S = 3  /* stored as BF16 of g, collided in FP32 */
} lbm_precision;

enum { LBM_CELL_FLUID = 0, LBM_CELL_SOLID = 1, LBM_CELL_INLET = 2, LBM_CELL_OUTLET = 3, LBM_CELL_EXTP = 4 };

/* 0D boundary models (Sec. 2.1.2 and 2.2 of the paper).  Parameters, all in
 * lattice units:
 *  PRESSURE_CONST  [p]                 pressure-type coupling, P* = c_s^2 + p
 *  VELOCITY_CONST  [vz]                velocity-type coupling, v* = (0, 0, vz)
 *  WINDKESSEL3     [Rp, C, Rd, mode]   3-element Windkessel, Eqs. rightbc and
 *                  rightQ marched by forward Euler.  mode 0: the flux Q
 *                  leaving the domain drives the model, P* = Pw + Rp Q
 *                  (explicit coupling: stable for Rp below the acoustic
 *                  impedance c_s / A of the layer and C above A / c_s);
 *                  mode 1: the mean boundary pressure drives it and the
 *                  outflow (P - Pw)/Rp is imposed as v* = v(x_f) + dv e_z with
 *                  dv = (Q_0D - Q_3D)/A (stable for Rp above c_s / A).
 *                  state: [Pw]
 *  LV_ELASTANCE    [Emax, Emin, Tc, Tmax, P_ed, N_S, k, a1, n1, a2, n2]
 *                  hybrid ODE-Dirichlet left ventricle (Eq. LVE) with the
 *                  double-Hill elastance E(t) = (Emax-Emin) k h1 h2 + Emin,
 *                  h1 = (tn/a1)^n1 / (1 + (tn/a1)^n1), h2 = 1/(1 + (tn/a2)^n2),
 *                  tn = (t mod Tc)/Tmax, C_v = 1/E.  The valve opens when
 *                  P_v exceeds the mean inlet pressure (at most once a beat),
 *                  closes on the first step with Q < 0 after inflow (Q > 0)
 *                  has begun since the opening; then
 *                  v* = v0(x_f, T_d) S(t, T_d, N_S) (Eqs. SmoothFunction and
 *                  vnew).  Each beat starts closed with P_v = P_ed.  Inlet only.
 *                  state: [Pv]                                           */
typedef enum {
  LBM_BC_PRESSURE_CONST = 0,
  LBM_BC_VELOCITY_CONST = 1,
  LBM_BC_WINDKESSEL3 = 2,
  LBM_BC_LV_ELASTANCE = 3
} lbm_bc_kind;

typedef struct {
  int32_t nx, ny, nz;    /* box size, each >= 3 */
  double tau;            /* BGK relaxation time (Eq. tau), > 0.5 */
  int32_t precision;     /* lbm_precision */
  double store_scale;    /* FP16S only: s (power of two), 0 = 256 */
  const uint8_t* flags;  /* host, nx*ny*nz cell types; copied by lbm_init */
  int32_t wave_cap;      /* waveform ring capacity in steps, 0 = 4096 */
  double p_ref;          /* reference gauge pressure of the stored populations:
                            the device keeps f_i - w_i (1 + 3 p_ref), an exact
                            change of variables (f_eq is linear in P) that keeps
                            the stored values small where the pressure sits near
                            p_ref; every value handed in or out is still g = f - w */
  int32_t nee_variant;   /* non-equilibrium extrapolation at 0D-coupled ghosts
                            (Eq. Non-equilibrium3): 0 takes x_f as the fluid
                            cell the ghost's population streams into (x_f = x
                            + e_i, the paper's statement); 1 takes x_f as the
                            ghost's neighbour along the inward normal of its box
                            face where that cell is FLUID (Guo, Zheng & Shi
                            2002), else as in 0.  Both agree on the populations
                            along the face normal. */
} lbm_config;

typedef struct {
  void* pop;        /* device, >= pop_bytes from lbm_query_sizes */
  size_t pop_bytes;
  void* work;       /* device, >= work_bytes from lbm_query_sizes */
  size_t work_bytes;
} lbm_buffers;

/* Sizes of the device buffers for n instances (n = 1: one box).  All
 * instances of one context share the precision of cfgs[0].  Limits of one
 * context: fewer than 2^31 cells in all, and one direction's populations
 * under 4 GiB (FP64: 2^29 cells, FP32: 2^30; the kernels address each
 * direction with 32-bit byte offsets).
 * Errors: LBM_E_INVAL for bad sizes, tau, flags, a NULL pointer or a
 * context past those limits. */
lbm_status lbm_query_sizes(const lbm_config* cfgs, int32_t n, size_t* pop_bytes, size_t* work_bytes);

/* Create a context over n independent instances (the batched ensemble when
 * n > 1) on the caller's device buffers and HIP stream (NULL = default
 * stream).  Sets every population to rest (g = 0: u = 0, p = 0, as in the
 * paper's initialisation U_0 = 0, Q_0 = 0), every boundary to
 * PRESSURE_CONST 0, the step counter to 0.  Enqueues host-to-device copies
 * on the stream.  Errors: LBM_E_INVAL (see lbm_query_sizes; buffers too
 * small), LBM_E_DEVICE. */
lbm_status lbm_init(const lbm_config* cfgs, int32_t n, const lbm_buffers* buf, void* hip_stream,
                    lbm_ctx** out);

/* Advance every instance by nsteps full steps (Algorithm 1): boundary
 * reductions and 0D update, IB force (if a wall is registered), fused
 * collide-stream.  Asynchronous, except that with a wall registered it
 * synchronises at every multiple of the band-check interval to test the
 * wall's motion (and rebuilds the band when needed, see lbm_wall_desc).
 * Errors: LBM_E_INVAL (nsteps < 0); LBM_E_BAND or LBM_E_UNSTABLE from a
 * band rebuild. */
lbm_status lbm_step(lbm_ctx* ctx, int64_t nsteps);

/* Steps between wall-motion tests (default 32; 0 never tests, so the band
 * stays where lbm_fsi_exchange built it).  The test is sound while no point
 * moves a whole lattice unit between two tests. */
lbm_status lbm_set_band_check(lbm_ctx* ctx, int32_t every);

/* Set the 0D model of boundary b (0 inlet, 1 outlet 0, 2 exterior, 2 + k
 * outlet k) of instance inst: kind, params (see lbm_bc_kind), optional
 * initial state.  Each outlet's model sees the flux and mean pressure of its
 * own layer (the FLUID cells of z = nz-2 above its ghosts) and sets its own
 * ghosts.  Synchronises the stream.  Errors: LBM_E_INVAL (kind/boundary
 * mismatch: the LV only at the inlet, the exterior constant models only;
 * too few params: PRESSURE/VELOCITY need 1, WINDKESSEL3 3 or 4, LV 11). */
lbm_status lbm_couple_0d(lbm_ctx* ctx, int32_t inst, int32_t boundary, int32_t kind,
                         const double* params, int32_t nparams, const double* state, int32_t nstate);

/* Read the 0D state of one boundary: out[0..7] = [vmode, p*, S, Pv, Pw,
 * valve_open, T_d, dv_or_vz].  Synchronises. */
lbm_status lbm_get_0d(lbm_ctx* ctx, int32_t inst, int32_t boundary, double* out);

/* Elastic wall (Sec. 2.3.2): a structured cylinder membrane of n_theta
 * (periodic) x n_z points (rings 0 and n_z-1 fixed, simply supported), point
 * p = j + n_theta*k.  Forces: penalty IB (Eq. LagForce, force on the fluid
 * F = alpha int(Vf - Vs) + beta (Vf - Vs), alpha, beta < 0; the wall gets -F),
 * Peskin 4-point delta for interpolation (Eq. interpolation) and spreading
 * (Eq. EulForce, b = sum F area delta), membrane stretching and bending by
 * the staggered differences of Eqs. tension and bending along both mesh
 * directions (bending acts on X - X0), central difference in time with
 * areal mass `mass`.  X0_host: 3*n_points doubles (x,y,z per point), rest
 * = initial shape.  band_margin: extra cells kept around the wall
 * (default 2).  The band (the fluid cells the wall exchanges with) follows
 * the wall: every band_check steps (lbm_set_band_check) lbm_step tests how
 * far the points have moved since the band was built and rebuilds it around
 * the current positions once that reaches band_margin - 1 lattice units.
 * A point whose stencil still leaves the band raises LBM_E_BAND at the next
 * lbm_sync; so does a rebuilt band that outgrows the buffer's reserve
 * (twice the initial band plus 4096 cells).  Stencil cells outside the box
 * take no part; a non-finite point stops the rebuild with LBM_E_UNSTABLE. */
typedef struct {
  int32_t n_theta, n_z;
  const double* X0_host;
  double ds_theta, ds_z, area;
  double k_stretch, ei_bend, mass, alpha, beta;
  int32_t band_margin;
  int32_t kernel;   /* delta kernel: 0 Peskin 4-point (default), 1 cosine
                       4-point (1 + cos(pi r / 2)) / 4 on |r| < 2 */
  int32_t mode;     /* 0 built-in membrane (default); 1 external solid: the
                       caller moves the points with lbm_set_wall, no membrane
                       forces act (k_stretch, ei_bend, mass unused), and the
                       library interpolates, forms the penalty force and
                       spreads it; the force on the solid, -F, is read back
                       with lbm_read_wall */
  int32_t shell;    /* 0 (default): Eq. structure along the two mesh
                       directions only (phi, gamma diagonal); 1: the full
                       shell model of Eq. structure, adding the off-diagonal
                       terms -- in-plane shear with phi_12 = 1 / (2 (1 +
                       poisson)) on the strain X_theta . X_z at the mesh-cell
                       centres, and the mixed bending with gamma_12 = 1 (the
                       bending operator becomes the discrete biharmonic) */
  double poisson;   /* Poisson's ratio of the shell model, > -1 (shell = 1) */
} lbm_wall_desc;

/* Device bytes the wall of one instance needs (Lagrangian state + dense
 * velocity / force fields of the instance's cells + band list). */
lbm_status lbm_fsi_query_sizes(lbm_ctx* ctx, int32_t inst, const lbm_wall_desc* wall, size_t* bytes);

/* Register (or replace) the wall of instance inst on the caller's device
 * buffer fsi_buf (>= bytes from lbm_fsi_query_sizes).  From the next step
 * on, every step exchanges velocity and force with the wall.  Synchronises.
 * Errors: LBM_E_INVAL (sizes, a point outside the box or a stencil touching
 * the box faces). */
lbm_status lbm_fsi_exchange(lbm_ctx* ctx, int32_t inst, const lbm_wall_desc* wall, void* fsi_buf,
                            size_t fsi_bytes);

/* External solid (wall mode 1): positions X (host, 3*n_points doubles) of
 * the points at the current step and their velocities V (lattice units per
 * step).  Until the next call the points keep that velocity,
 * X^{n+1} = 2 X^n - X^{n-1}.  Synchronises; rebuilds the band when the
 * points have moved band_margin - 1 units or more since it was built.
 * Errors: LBM_E_INVAL (NULL, no wall or a built-in membrane at inst),
 * LBM_E_UNSTABLE (a non-finite or out-of-box point during a band rebuild),
 * LBM_E_BAND (a rebuilt band larger than the buffer holds). */
lbm_status lbm_set_wall(lbm_ctx* ctx, int32_t inst, const double* X, const double* V);

/* Read the wall state: X, Xprev (positions at t_n, t_{n-1}), slip integral,
 * interpolated fluid velocity Vf and force on the fluid F of the last step;
 * each 3*n_points doubles, any pointer may be NULL.  Synchronises. */
lbm_status lbm_read_wall(lbm_ctx* ctx, int32_t inst, double* X, double* Xprev, double* slip,
                         double* Vf, double* F);

/* Wall shear stress at every point of instance inst's wall (the paper's
 * case study, Sec. 3.2: WSS = mu dv1/dx3, the axial velocity's derivative
 * normal to the wall, from the fluid next to the wall).  At a point X the
 * mesh tangents give the inward unit normal n = -(t_theta x t_z)/|..| and the
 * axial unit vector a = t_z/|t_z| (central differences; one-sided on the end
 * rings); the fluid velocity sum e_i g_i is interpolated trilinearly over
 * the FLUID cells around X + dist n (weights renormalised; NaN where none
 * is FLUID), and WSS = mu ((v - V_wall) . a) / dist with V_wall = X^n -
 * X^{n-1} and mu = (tau - 1/2)/3 (rho_0 = 1).  dist in lattice units,
 * 0 < dist < 64 (2 reaches just past the delta kernel).  wss: host,
 * n_points doubles.  Synchronises.  Errors: LBM_E_INVAL (no wall, NULL,
 * dist out of range). */
lbm_status lbm_wall_shear_stress(lbm_ctx* ctx, int32_t inst, double dist, double* wss);

/* Overwrite the populations of instance inst: g (host, [cell][19] doubles,
 * shifted) for FLUID cells.  Only between an even number of steps.  Converts
 * to the storage precision (round to nearest even).  Synchronises. */
lbm_status lbm_write_populations(lbm_ctx* ctx, int32_t inst, const double* g_host);

/* Uniform rest state at gauge pressure p for every FLUID cell of instance
 * inst (the paper's arbitrary initial P_0).  Asynchronous. */
lbm_status lbm_set_rest(lbm_ctx* ctx, int32_t inst, double p);

/* Read the populations (host [cell][19] doubles, shifted, 0 off-fluid) of
 * instance inst at the current step.  Synchronises. */
lbm_status lbm_read_populations(lbm_ctx* ctx, int32_t inst, double* g_host);

/* The field outputs of Algorithm 1 (pressure and velocity, Eqs. rho and v)
 * at the current step: gauge pressure p = c_s^2 sum g (ncell doubles) and
 * the first moment sum e_i g_i (3*ncell doubles, rho_0 = 1) of instance inst;
 * either may be NULL; 0 off-fluid.  The first moment is the unforced
 * velocity: where the wall's force density b acts, Eq. v's velocity of the
 * next collision is this plus b/2, and b of the next step is only known once
 * that step's exchange has run.  Synchronises. */
lbm_status lbm_read_fields(lbm_ctx* ctx, int32_t inst, double* p_host, double* u_host);

/* The boundary outputs of Algorithm 1 (the flux and pressure waveforms of
 * Sec. 2.1.2 at both 0D-coupled planes and the 0D states driving them).
 * Per-step boundary waveforms of instance inst, 14 doubles per step:
 * [n, Q_in, p_in, Q_out, p_out, in_mode, in_value, out_mode, out_value, Pv,
 *  Pw_out, valve, Q_mid, p_mid] (value = p* in pressure mode, S for the LV
 * and the axial v* or correction otherwise; Q_mid, p_mid: flux and mean
 * gauge pressure, as for the boundary layers, on the mid-length plane
 * z = nz/2 over the columns of the inlet's lumen, i.e. the FLUID cells of
 * that plane above an INLET ghost; recorded only, coupled to nothing).  Writes the last min(cap, steps, wave_cap)
 * records, oldest first, and sets *n to that count.  Synchronises. */
lbm_status lbm_read_waveforms(lbm_ctx* ctx, int32_t inst, double* out, int64_t cap, int64_t* n);

/* Per-outlet waveforms of instance inst (Sec. 2.1.2, each outlet's flux and
 * pressure and its Windkessel state): 24 doubles per step, for outlet
 * k = 0..7 [Q_k, p_k, Pw_k] (flux through its layer in +z, mean gauge
 * pressure of the layer, Windkessel pressure or 0 for another model; 0 for
 * an outlet without cells).  Outlet 0 repeats columns 3, 4 and 10 of
 * lbm_read_waveforms.  Writes the last min(cap, steps, wave_cap) records,
 * oldest first, and sets *n to that count.  Synchronises. */
lbm_status lbm_read_outlet_waveforms(lbm_ctx* ctx, int32_t inst, double* out, int64_t cap, int64_t* n);

/* Wait for the stream and report failures: LBM_E_UNSTABLE if a boundary
 * flux or pressure became non-finite (or a wall point did, at a band
 * rebuild), LBM_E_BAND if a wall point left its band.  Each instance has its
 * own error word, and an instance that fails is frozen from then on: its
 * populations, wall, 0D state and waveform record stay as they were and no
 * kernel touches it again.  A single-instance context reports its failure
 * here; a batch (n > 1) goes on while any instance runs, so lbm_sync fails
 * only once every instance has failed, and lbm_instance_status names the
 * failed ones. */
lbm_status lbm_sync(lbm_ctx* ctx);

/* Status of instance inst: LBM_OK while it runs, LBM_E_UNSTABLE or
 * LBM_E_BAND once it has failed and been frozen.  Synchronises.  Errors:
 * LBM_E_INVAL (index out of range). */
lbm_status lbm_instance_status(lbm_ctx* ctx, int32_t inst);

/* Steps taken so far. */
int64_t lbm_steps(const lbm_ctx* ctx);

/* Kernel timing with HIP events on the context's stream: when on, the
 * launches of each step are bracketed by events, per kind: the collide-stream
 * kernel over the tiles without a 0D ghost of the normal-neighbour
 * extrapolation nearby (id 0), the boundary/0D kernel (1), the band-moment
 * kernel (2), the wall kernels (3: interpolation, force, spreading and the
 * membrane step) and the collide-stream kernel over the tiles next to such
 * ghosts (4; otherwise forked to a second stream beside id 0's launch, timed
 * steps run them in sequence).  lbm_kernel_time synchronises and returns the
 * bracketed intervals and their total milliseconds since timing was switched
 * on. */
lbm_status lbm_set_timing(lbm_ctx* ctx, int32_t on);
lbm_status lbm_kernel_time(lbm_ctx* ctx, int32_t kernel, int64_t* launches, double* total_ms);

/* Replay steps from a captured HIP graph (one even + one odd step) instead
 * of launching kernels one by one (default on; turned off while timing). */
lbm_status lbm_set_graph(lbm_ctx* ctx, int32_t on);

/* With a wall registered, run the wall exchange (band moments,
 * interpolation, force, spreading, membrane) on a second stream of the
 * library's own while the main stream collides the cells outside the wall
 * band; the band cells collide after the spread force is complete.  The
 * cells' slot sets are disjoint, so results are identical either way.
 * Default off: on the elastic-tube workloads the band-only collide pass
 * (band cells in short runs spread over most 256-cell tiles) and the
 * kernels' competition for the CUs cost more than the overlap saves.
 * Timing and autotuning always run the kernels in sequence.
 * Synchronises and drops the captured step graph. */
lbm_status lbm_set_overlap(lbm_ctx* ctx, int32_t on);

/* Deterministic spreading (Eq. EulForce): the wall tiles are launched in
 * six colour classes one after another -- (theta tile index parity) +
 * 2 (z tile index parity), and two more for the last theta column of a ring
 * with an odd tile count -- so that tiles whose stencil boxes meet are never
 * in the same launch.  Each tile's sums are exact (fixed point in LDS), and a
 * cell then receives them in colour order: two runs from the same state give
 * bitwise equal results, where the default single launch sums the tiles in
 * the order the hardware runs them (equal to rounding).  Holds while every
 * tile's box is staged in LDS (the unstaged path for oversized boxes spreads
 * point by point with float atomics) and tiles two apart along theta or z do
 * not reach the same cell (tiles spanning more than the 4-cell stencil, as
 * the defaults do).  Costs the wall exchange its single launch's occupancy.
 * Default off.  Synchronises and drops the captured step graph. */
lbm_status lbm_set_deterministic(lbm_ctx* ctx, int32_t on);

/* Race check of the AA streaming (a debug aid, not part of a step): runs the
 * FP32 collide-stream of the given parity (0 even, 1 odd) over every cell
 * with each population store replaced by an atomic count of the slot it
 * targets, and copies the counts to counts (host, 19 * N uint32, N = the
 * context's total cell count, slot i of global cell c at i * N + c).  The
 * populations are left unchanged.  In a race-free step every count is 0 or
 * 1, and every slot a fluid cell reads in the following step (parity 0:
 * slot opp(i) of c - e_i; parity 1: slot i of c) counts 1.  Synchronises;
 * allocates its counters for the call.  Errors: LBM_E_INVAL (NULL, parity,
 * a context that is not FP32), LBM_E_STATE (a store aimed past the
 * population arrays, which the step's bounded stores would drop),
 * LBM_E_DEVICE. */
lbm_status lbm_debug_slot_writes(lbm_ctx* ctx, int32_t parity, uint32_t* counts);

/* Launch shapes per size class.  The instances of a context are grouped by
 * cell count into size classes (quartiles from 8 instances on, else one
 * class); each class has its own collide-stream launch (workgroup size and
 * cells per lane, over a table of tiles of consecutive cells of one
 * instance) and wall launch (tiles of wall_tile_theta x wall_tile_z mesh
 * points, one 256-lane workgroup each).  Defaults: workgroups of 256 lanes,
 * one cell per lane, 16 x 16 wall tiles -- or, when a wall is attached whose
 * 16 x 16 stencil boxes would fill more than 60 % of the standard LDS
 * staging (coarse meshes), the first of 16 x 8, 8 x 16, 8 x 8 whose boxes
 * do not, unless the class's shapes were set.  Results do not depend on the shapes, except for
 * the rounding order of the wall force's float additions. */
typedef struct {
  int32_t block;            /* collide workgroup: 128, 256 or 512 lanes */
  int32_t cells_per_lane;   /* 1 or 2 */
  int32_t wall_tile_theta;  /* 8, 16 or 32 mesh points along theta */
  int32_t wall_tile_z;      /* mesh points along z: 0 = 256 / wall_tile_theta
                               (tiles of 256 points: 8 x 32, 16 x 16, 32 x 8),
                               or the smaller tiles 8 x 16, 16 x 8, 8 x 8, whose
                               stencil boxes fit the staging memory on coarse
                               meshes (one lane per point, the other lanes idle
                               while the points are processed) */
} lbm_launch;

int32_t lbm_num_classes(lbm_ctx* ctx);
/* Instances, cells and wall points of class cls (any pointer may be NULL). */
lbm_status lbm_class_info(lbm_ctx* ctx, int32_t cls, int32_t* instances, int64_t* cells, int64_t* wall_points);
lbm_status lbm_get_launch(lbm_ctx* ctx, int32_t cls, lbm_launch* out);
/* Set a class's shapes (LBM_E_INVAL outside the values above); synchronises
 * and drops the captured step graph. */
lbm_status lbm_set_launch(lbm_ctx* ctx, int32_t cls, const lbm_launch* launch);

/* Autotuner: times the current shapes and every collide shape (6), then
 * the current and every wall tile (6, if walls are registered), over
 * trial_steps steps each (rounded up to even, after 2 untimed steps), per
 * class with HIP events; a class changes shape only for a candidate at
 * least 2 % faster than its current one.  The trial steps are ordinary steps of the method: the state
 * advances by *advanced steps (may be NULL).  Call after the 0D couplings
 * and walls are set. */
lbm_status lbm_autotune(lbm_ctx* ctx, int32_t trial_steps, int64_t* advanced);

/* Checkpoint / resume.  lbm_save waits for the stream and writes to the
 * file at path everything that determines later steps: populations, cell
 * flags (band bits), the 0D boundary records, step counters, waveform rings,
 * inlet snapshots, the error and motion words, and per wall its two
 * displacement levels, slip integral, last interpolated velocity and force,
 * displacement at the last band build and its band.  lbm_load restores such
 * a file into a context built the same way (lbm_init with the same
 * configurations, the same walls attached; 0D couplings are restored from
 * the file), after which stepping continues bit for bit as the saved run
 * would have.  lbm_load reads and checks the whole file on the host before
 * it uploads anything: the cell types must equal the context's own (only the
 * band bits may differ), each band list must hold ascending FLUID cells of
 * its instance that are exactly the cells with the band bit, the 0D records
 * must name valid kinds for their boundaries, and nothing may follow the
 * band lists.  Errors: LBM_E_INVAL (NULL, unopenable or unwritable path),
 * LBM_E_STATE (not a checkpoint, truncated, malformed, or a context of another
 * shape, precision, storage scale or waveform capacity; a saved band larger
 * than the wall buffer holds), LBM_E_DEVICE.  A load refused with
 * LBM_E_STATE leaves the context as it was. */
lbm_status lbm_save(lbm_ctx* ctx, const char* path);
lbm_status lbm_load(lbm_ctx* ctx, const char* path);

const char* lbm_last_error(const lbm_ctx* ctx);
void lbm_destroy(lbm_ctx* ctx);

/* Number of cells / population bytes per cell of instance inst. */
int64_t lbm_num_cells(const lbm_ctx* ctx, int32_t inst);
int32_t lbm_bytes_per_population(const lbm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* LBM0D3D_H */
