// lbm_kernels.hip -- gfx950 kernels of the 0D-3D coupled lattice Boltzmann
// step (Wei, Amlani & Pahlevan, arXiv 2112.05258, Algorithm 1).
//
// Per step, on one stream:
//   k_reduce    boundary layers: flux Q = sum j_z / sum f and mean gauge
//               pressure (Sec. 2.1.2) in FP64, fixed-order tree reductions;
//               the last workgroup of an instance advances its 0D models one
//               forward-Euler step (Eqs. LVE, rightbc, rightQ, SmoothFunction)
//               and writes the waveform record
//   k_band      unforced velocity of the wall's band cells, clears the force
//   k_wall      per wall point: interpolation (Eq. interpolation), penalty
//               force (Eq. LagForce), spreading (Eq. EulForce), membrane
//               forces (Eqs. tension, bending) and the time step of the wall
//   k_collide   fused BGK collide-stream (Eqs. fi, feq, f, rho, v) in the AA
//               in-place pattern with halfway bounce-back and the
//               non-equilibrium extrapolation of Eq. Non-equilibrium3 at
//               0D-coupled ghost nodes
// The lattice work is HBM-bound (no contraction): one cell per lane,
// 19 coalesced loads and 19 coalesced stores per cell.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "lbm_internal.h"
#include "zerod.h"

namespace lbm {

// D3Q19 in the interface order.
__device__ constexpr int EX[NQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
__device__ constexpr int EY[NQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__device__ constexpr int EZ[NQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
__device__ constexpr int OPP[NQ] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};

// face direction along axis a (0 x, 1 y, 2 z) with sign sg, and the two face
// directions an edge direction (i >= 7) is the sum of
__device__ constexpr int face_dir(int a, int sg) { return 1 + 2 * a + (sg < 0 ? 1 : 0); }
__device__ constexpr int edge_a(int i) { return EX[i] != 0 ? face_dir(0, EX[i]) : face_dir(1, EY[i]); }
__device__ constexpr int edge_b(int i) { return EZ[i] != 0 ? face_dir(2, EZ[i]) : face_dir(1, EY[i]); }

// Workgroups are handed to the 8 XCDs in turn (workgroup b to XCD b mod 8),
// and each XCD has its own L2.  This maps workgroup b of nb to a tile index
// such that the workgroups of one XCD take consecutive tiles, so that
// neighbouring tiles, which share halo lines, share an L2.  A bijection of
// [0, nb).  Used by the band moments (cfg1 FP32 136 -> 123 us, FP16 80 ->
// 64 us: neighbouring band chunks share the lines of their rows' runs) and
// the membrane step (32.5 -> 27.7 us: halo rows); the collide (one stream
// through memory) and k_wall measured slower with it.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}

template <class R>
__device__ __forceinline__ R wgt(int i) {
  return i == 0 ? R(1) / R(3) : (i < 7 ? R(1) / R(18) : R(1) / R(36));
}

// ---------------------------------------------------------------------------
// storage types: value stored = scale * g (scale used by the 16-bit modes)
// ---------------------------------------------------------------------------
template <class S> struct Store;
template <> struct Store<double> {
  using R = double;
  __device__ static R ld(const double* p, float) { return *p; }
  __device__ static void st(double* p, R v, float) { *p = v; }
};
template <> struct Store<float> {
  using R = float;
  __device__ static R ld(const float* p, float) { return *p; }
  __device__ static void st(float* p, R v, float) { *p = v; }
};
template <> struct Store<__half> {
  using R = float;
  __device__ static R ld(const __half* p, float inv) { return __half2float(*p) * inv; }
  __device__ static void st(__half* p, R v, float s) { *p = __float2half_rn(v * s); }
};
template <> struct Store<__hip_bfloat16> {
  using R = float;
  __device__ static R ld(const __hip_bfloat16* p, float inv) { return __bfloat162float(*p) * inv; }
  __device__ static void st(__hip_bfloat16* p, R v, float s) { *p = __float2bfloat16(v * s); }
};

// Buffer addressing of one direction's array: a uniform descriptor (base,
// size in bytes; accesses at or past the size read 0 and write nothing) and a
// 32-bit byte offset per lane, instead of a 64-bit address per lane and
// direction.  Needs NT * sizeof(S) < 2^32 (checked at init).
typedef __amdgpu_buffer_rsrc_t Rsrc;
__device__ __forceinline__ Rsrc dir_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
template <class S> struct BufIO;
template <> struct BufIO<double> {
  __device__ static double ld(Rsrc r, uint32_t o, float) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, o, 0, 0));
  }
  __device__ static void st(Rsrc r, uint32_t o, double v, float) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r, o, 0, 0);
  }
};
template <> struct BufIO<float> {
  __device__ static float ld(Rsrc r, uint32_t o, float) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, o, 0, 0));
  }
  __device__ static void st(Rsrc r, uint32_t o, float v, float) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, o, 0, 0);
  }
};
template <> struct BufIO<__half> {
  __device__ static float ld(Rsrc r, uint32_t o, float inv) {
    return __half2float(__builtin_bit_cast(__half, __builtin_amdgcn_raw_buffer_load_b16(r, o, 0, 0))) * inv;
  }
  __device__ static void st(Rsrc r, uint32_t o, float v, float s) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, __float2half_rn(v * s)), r, o, 0, 0);
  }
};
template <> struct BufIO<__hip_bfloat16> {
  __device__ static float ld(Rsrc r, uint32_t o, float inv) {
    return __bfloat162float(__builtin_bit_cast(__hip_bfloat16, __builtin_amdgcn_raw_buffer_load_b16(r, o, 0, 0))) *
           inv;
  }
  __device__ static void st(Rsrc r, uint32_t o, float v, float s) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, __float2bfloat16(v * s)), r, o, 0, 0);
  }
};

template <class R> struct V4;
template <> struct V4<float> { using T = float4; };
template <> struct V4<double> { using T = double4; };

__device__ __forceinline__ void dir_offsets(int64_t sy, int64_t sz, int64_t off[NQ]) {
#pragma unroll
  for (int i = 0; i < NQ; ++i) off[i] = EX[i] + EY[i] * sy + EZ[i] * sz;
}

// Populations of cell c at the current step (parity = step & 1), AA layout:
// even: g_i = A[i][c]; odd: g_i = A[opp i][c - e_i].  Halfway bounce-back
// needs no case here: a population streamed toward a SOLID cell is stored
// where the next step's plain load finds it (see collide_body).
template <class S, bool ODD>
__device__ __forceinline__ void load_cell(const S* __restrict__ A, int64_t NT, int64_t c, const int64_t off[NQ],
                                          float inv, typename Store<S>::R g[NQ]) {
#pragma unroll
  for (int i = 0; i < NQ; ++i)
    g[i] = ODD ? Store<S>::ld(A + OPP[i] * NT + c - off[i], inv) : Store<S>::ld(A + i * NT + c, inv);
}

// ---------------------------------------------------------------------------
// k_reduce: layer flux / pressure, then (last block) the 0D update
// ---------------------------------------------------------------------------
template <class S, bool ODD>
__device__ __forceinline__ void reduce_block(const Dev& d, const int blk) {
  using R = typename Store<S>::R;
  __shared__ double sq[RBLOCK], sp[RBLOCK];
  __shared__ int last;
  const RedTab t = d.red[blk];
  // an instance that failed in an earlier step is frozen from this step on:
  // no further reductions, 0D updates or records, and the later kernels of
  // the step skip it (uniform over the block)
  if (d.err[t.inst] != 0u) {
    if (threadIdx.x == 0) atomicOr(d.err + t.inst, ERR_FROZEN);
    return;
  }
  const InstDesc& I = d.inst[t.inst];
  const int64_t sy = I.nx, sz = (int64_t)I.nx * I.ny;
  int64_t off[NQ];
  dir_offsets(sy, sz, off);
  const S* A = (const S*)d.pop;
  double q = 0.0, ps = 0.0;
  for (int k = threadIdx.x; k < t.count; k += RBLOCK) {
    const int64_t c = I.cell0 + d.lay[I.lay_off[t.plane] + t.start + k];
    R g[NQ];
    load_cell<S, ODD>(A, d.NT, c, off, d.inv_scale, g);
    double s = I.dref, jz = 0.0;
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      s += (double)g[i];
      jz += EZ[i] * (double)g[i];
    }
    q += jz / (1.0 + s);
    ps += s / 3.0;
  }
  sq[threadIdx.x] = q;
  sp[threadIdx.x] = ps;
  __syncthreads();
  for (int w = RBLOCK / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      sq[threadIdx.x] += sq[threadIdx.x + w];
      sp[threadIdx.x] += sp[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    d.red_part[2 * blk] = sq[0];
    d.red_part[2 * blk + 1] = sp[0];
    InstState* st = d.st + t.inst;
    const uint32_t done =
        __hip_atomic_fetch_add(&st->counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    last = (done == (uint32_t)(I.nred - 1));
  }
  __syncthreads();
  if (!last) return;

  // ---- last block of this instance: finish the sums in a fixed order (a
  // strided pass per lane, then one tree per plane that has cells), all
  // lanes loading partials at once
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  InstState* st = d.st + t.inst;
  double qa[NPL], pa[NPL];
#pragma unroll
  for (int pl = 0; pl < NPL; ++pl) qa[pl] = pa[pl] = 0.0;
  for (int b = I.red0 + (int)threadIdx.x; b < I.red0 + I.nred; b += RBLOCK) {
    const double vq = __hip_atomic_load(&d.red_part[2 * b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const double vp = __hip_atomic_load(&d.red_part[2 * b + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int pl = d.red[b].plane;
#pragma unroll
    for (int q = 0; q < NPL; ++q)
      if (pl == q) { qa[q] += vq; pa[q] += vp; }
  }
  double Q[NPL], P[NPL];
#pragma unroll
  for (int pl = 0; pl < NPL; ++pl) {
    Q[pl] = P[pl] = 0.0;
    if (I.lay_n[pl] == 0) continue;   // uniform over the block
    sq[threadIdx.x] = qa[pl];
    sp[threadIdx.x] = pa[pl];
    __syncthreads();
    for (int w = RBLOCK / 2; w > 0; w >>= 1) {
      if (threadIdx.x < w) {
        sq[threadIdx.x] += sq[threadIdx.x + w];
        sp[threadIdx.x] += sp[threadIdx.x + w];
      }
      __syncthreads();
    }
    Q[pl] = sq[0];
    P[pl] = sp[0] / (double)I.lay_n[pl];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  // planes: inlet, outlets (coupled to the 0D models), mid-length (recorded)
  bool finite = isfinite(Q[0]) && isfinite(P[0]);
#pragma unroll
  for (int k = 0; k < NOUT; ++k) finite = finite && isfinite(Q[outlet_slot(k)]) && isfinite(P[outlet_slot(k)]);
  if (!finite) atomicOr(d.err + t.inst, ERR_NONFINITE);
  const int64_t n = st->step;
  BcDev* bc = d.bc + NBC * t.inst;
  bc[0].area = (double)I.lay_n[0];
  zerod_update(bc[0], n, Q[0], P[0]);
  double* ro = d.owave + ((int64_t)t.inst * d.wave_cap + (n % d.wave_cap)) * NOREC;
#pragma unroll 1
  for (int k = 0; k < NOUT; ++k) {
    const int s = outlet_slot(k);
    bc[s].area = (double)I.lay_n[s];
    zerod_update(bc[s], n, Q[s], P[s]);
    ro[3 * k] = Q[s];
    ro[3 * k + 1] = P[s];
    ro[3 * k + 2] = bc[s].kind == BC_WK3 ? bc[s].Pw : 0.0;
  }
  zerod_update(bc[2], n, 0.0, 0.0);
  double* r = d.wave + ((int64_t)t.inst * d.wave_cap + (n % d.wave_cap)) * NREC;
  r[0] = (double)n;
  r[1] = Q[0]; r[2] = P[0]; r[3] = Q[1]; r[4] = P[1];
  r[5] = bc[0].vmode;
  r[6] = bc[0].vmode == 0 ? bc[0].pstar : (bc[0].kind == BC_LV ? bc[0].S : bc[0].vz);
  r[7] = bc[1].vmode;
  r[8] = bc[1].vmode == 0 ? bc[1].pstar : bc[1].vz;
  r[9] = bc[0].kind == BC_LV ? bc[0].Pv : 0.0;
  r[10] = bc[1].kind == BC_WK3 ? bc[1].Pw : 0.0;
  r[11] = bc[0].kind == BC_LV ? (double)bc[0].open : 0.0;
  r[12] = Q[2]; r[13] = P[2];
  st->step = n + 1;
  __hip_atomic_store(&st->counter, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

template <class S, bool ODD>
__global__ __launch_bounds__(RBLOCK) void k_reduce(Dev d) {
  reduce_block<S, ODD>(d, blockIdx.x);
}

// ---------------------------------------------------------------------------
// k_collide: fused collide-stream
// ---------------------------------------------------------------------------

// g_eq(delta, v*) - g_eq(delta, v) for the velocity-type coupling.
template <class R>
__device__ __forceinline__ R deq_velocity(int i, R vx, R vy, R vz, R sx, R sy, R sz) {
  const R eu = EX[i] * vx + EY[i] * vy + EZ[i] * vz;
  const R es = EX[i] * sx + EY[i] * sy + EZ[i] * sz;
  const R uu = vx * vx + vy * vy + vz * vz;
  const R ss = sx * sx + sy * sy + sz * sz;
  return wgt<R>(i) * (R(3) * (es - eu) + R(4.5) * (es * es - eu * eu) - R(1.5) * (ss - uu));
}

// s += e x for a lattice component e in {-1, 0, 1}, known at compile time
// once the direction loops are unrolled.  The first nonzero term initialises
// s, so neither a product with 0 nor a 0 + x is left in the code (IEEE rules
// keep the compiler from dropping them itself).
template <class R>
__device__ __forceinline__ void eacc(R& s, bool& first, int e, R x) {
  if (e == 0) return;
  const R t = e > 0 ? x : -x;
  s = first ? t : s + t;
  first = false;
}

// e_i . (x, y, z) over the nonzero components of e_i (0 for the rest vector)
template <class R>
__device__ __forceinline__ R edot(int i, R x, R y, R z) {
  R s = R(0);
  bool first = true;
  eacc(s, first, EX[i], x);
  eacc(s, first, EY[i], y);
  eacc(s, first, EZ[i], z);
  return s;
}

// Moments of one cell (Eqs. rho, v): dl = sum g - dref (= delta - 3 p_ref),
// j = sum e g, the velocity v = j + b / 2 of the forced scheme, and the
// parts of the equilibrium shared by all directions.
template <class R> struct Mom {
  R dl, jx, jy, jz, vx, vy, vz, bx, by, bz, t0, vb;
};
template <class R, bool BAND>
__device__ __forceinline__ Mom<R> moments(const R g[NQ], R bx, R by, R bz) {
  Mom<R> m;
  m.dl = g[0];
  m.jx = m.jy = m.jz = R(0);
  bool fx = true, fy = true, fz = true;
#pragma unroll
  for (int i = 1; i < NQ; ++i) {
    m.dl += g[i];
    eacc(m.jx, fx, EX[i], g[i]);
    eacc(m.jy, fy, EY[i], g[i]);
    eacc(m.jz, fz, EZ[i], g[i]);
  }
  m.bx = bx; m.by = by; m.bz = bz;
  m.vx = BAND ? m.jx + R(0.5) * bx : m.jx;
  m.vy = BAND ? m.jy + R(0.5) * by : m.jy;
  m.vz = BAND ? m.jz + R(0.5) * bz : m.jz;
  m.t0 = m.dl - R(1.5) * (m.vx * m.vx + m.vy * m.vy + m.vz * m.vz);
  m.vb = m.vx * bx + m.vy * by + m.vz * bz;
  return m;
}

// Post-collision value of direction i (Eqs. fi, feq, f):
// g* = (1 - 1/tau) g + (1/tau) g_eq, g_eq = w (dl + 3 eu + 4.5 eu^2 - 1.5 uu),
// plus the forcing term w (1 - 1/(2 tau)) (3 (e - v).b + 9 (e.v)(e.b)) on
// band cells (zero where b = 0).
template <class R, bool BAND>
__device__ __forceinline__ R relax(int i, const Mom<R>& m, R g, R om) {
  const R eu = edot<R>(i, m.vx, m.vy, m.vz);
  const R r = i == 0 ? m.t0 : eu * (R(3) + R(4.5) * eu) + m.t0;
  R v = (R(1) - om) * g + (om * wgt<R>(i)) * r;
  if (BAND) {
    const R eb = edot<R>(i, m.bx, m.by, m.bz);
    v += ((R(1) - R(0.5) * om) * wgt<R>(i)) * (R(3) * (eb - m.vb) + R(9) * eu * eb);
  }
  return v;
}

// One lattice cell (global index c, local index local of instance inst) of
// the collide-stream step.  NEAR: the wave holds a cell next to a 0D-coupled
// ghost, or (odd step) next to a solid (per-direction source and target
// types are looked up);
// BAND: the wave holds a cell of the wall's band (the IB force enters, zero
// at the wave's other cells).  The plain body has neither.
template <class S, bool ODD, bool NEAR, bool BAND, bool NEE, bool COUNT = false>
__device__ __forceinline__ void collide_body(const Dev& d, const int inst, const InstDesc& I, const int64_t local,
                                             const uint32_t c, const uint8_t fl) {
  using R = typename Store<S>::R;
  using R4 = typename V4<R>::T;
  const int32_t sy = I.nx, sz = I.nx * I.ny;
  int32_t off[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) off[i] = EX[i] + EY[i] * sy + EZ[i] * sz;
  S* __restrict__ A = (S*)d.pop;
  const int64_t NT = d.NT;

  // source cell types (only cells next to walls or ghosts look), 3 bits per
  // direction in one 64-bit word.  16-bit storage: the precomputed word, one
  // load instead of 18 (its wave-level instruction count is what the 16-bit
  // collide pays for); FP32 / FP64: from the flags, whose lines the wave
  // reads anyway (the word's extra lines cost the bandwidth-bound step more)
  uint64_t ntb = 0;
  if (NEAR && (fl & F_NEAR)) {
    if constexpr (sizeof(S) == 2) {
      ntb = d.nbr[c];
    } else {
#pragma unroll
      for (int i = 1; i < NQ; ++i) ntb |= (uint64_t)(d.flags[c - off[i]] & TYPE_MASK) << (3 * i);
    }
  }
  auto nt = [&](int i) -> uint32_t { return (uint32_t)(ntb >> (3 * i)) & 7u; };

  constexpr uint32_t ES = sizeof(S);
  const uint32_t dir_bytes = (uint32_t)(NT * ES);
  auto rs = [&](int i) { return dir_rsrc(A + i * NT, dir_bytes); };
  // a store of direction dir at byte offset o; the counting build (the
  // slot-writer check) counts it in d.slotcnt instead of storing -- an
  // offset past the direction's array (which the buffer store would drop)
  // in the extra counter after the 19 * NT slots
  auto put = [&](int dir, uint32_t o, typename Store<S>::R v) {
    if constexpr (COUNT) {
      const uint64_t k = o / ES;
      atomicAdd(d.slotcnt + (k < (uint64_t)NT ? (uint64_t)dir * (uint64_t)NT + k : (uint64_t)NQ * (uint64_t)NT), 1u);
    } else {
      BufIO<S>::st(rs(dir), o, v, d.scale);
    }
  };
  R g[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    if (!ODD) g[i] = BufIO<S>::ld(rs(i), c * ES, d.inv_scale);
    else g[i] = BufIO<S>::ld(rs(OPP[i]), (uint32_t)(c - off[i]) * ES, d.inv_scale);
  }
  R bx = 0, by = 0, bz = 0;
  if (BAND && (fl & F_BAND)) {
    const R4 b = ((const R4*)I.b4)[local];
    bx = b.x; by = b.y; bz = b.z;
  }
  const Mom<R> m = moments<R, BAND>(g, bx, by, bz);
  const R om = R(I.omega);

  // collision and streaming, direction by direction.  A 0D-coupled ghost
  // x = c - e_i hands the fluid cell x + e_i the value
  // g*_i(x_f) + g_eq(P*, v*) - g_eq(P(x_f), v(x_f)) (Eq. Non-equilibrium3).
  // Literal reading: x_f = x + e_i, this cell.  Normal-neighbour reading
  // (I.nee): x_f is the ghost's neighbour along the inward normal of its
  // face.  Ghosts sit on the box faces and fluid cells inside, so the normal
  // neighbour of the ghost c - e_i is c itself for a face direction, and for
  // an edge direction e_i = e_a + e_b it is c - e_b or c - e_a, whichever is
  // FLUID (at most one is: the other lies on the ghost's face); none being
  // FLUID falls back to x_f = c.  That cell forms the value from its own
  // moments and stores it into the receiver's slot (written by no one else
  // in the step: the ghost neither reads nor writes), and the receiver skips
  // it.  Each value is formed right after g*_i, so that the post-collision
  // values need not stay live.
  R4 v0 = {0, 0, 0, 0};
  bool have_v0 = false;
  // 0D record of the ghost cell gc of type tg: an OUTLET ghost names its
  // outlet in the high bits of its flag byte (loaded only for outlets)
  auto ghost_value = [&](int i, uint32_t tg, uint32_t gc, R v) -> R {
    const int slot = tg == T_INLET ? 0 : (tg == T_EXTP ? 2 : outlet_slot(d.flags[gc] >> OUT_SHIFT));
    const BcDev& B = d.bc[NBC * inst + slot];
    if (B.vmode == 0) return v + wgt<R>(i) * (R(B.dstar - I.dref) - m.dl);
    R sx, s_y, s_z;
    if (B.vkind == VK_SNAPSHOT) {
      if (!have_v0) {
        R4* vp = (R4*)d.v0 + I.v0_off + (local % sz);
        if (B.snap) {
          v0 = R4{m.jx, m.jy, m.jz, R(0)};
          *vp = v0;
        } else {
          v0 = *vp;
        }
        have_v0 = true;
      }
      const R Sf = R(B.S);
      sx = v0.x * Sf; s_y = v0.y * Sf; s_z = v0.z * Sf;
    } else if (B.vkind == VK_CORRECT) {
      sx = m.vx; s_y = m.vy; s_z = m.vz + R(B.vz);
    } else {
      sx = 0; s_y = 0; s_z = R(B.vz);
    }
    return v + deq_velocity<R>(i, m.vx, m.vy, m.vz, sx, s_y, s_z);
  };
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const R v = relax<R, BAND>(i, m, g[i], om);
    if (!ODD) put(OPP[i], c * ES, v);
    else put(i, (uint32_t)(c + off[i]) * ES, v);
    // halfway bounce-back: g*_i toward a SOLID cell x = c + e_i returns to c
    // as direction opp i.  It goes to the slot the next step's plain load of
    // that direction reads: x's A[i][x] after an even step, the own A[opp i][c]
    // after an odd one (slots no other cell touches).  The plain store above
    // then lands in a slot nobody reads (the solid's, or the own slot whose
    // reader would be the solid).
    if (NEAR && i > 0 && nt(OPP[i]) == T_SOLID) {
      if (!ODD) put(i, (uint32_t)(c + off[i]) * ES, v);
      else put(OPP[i], c * ES, v);
    }
    if (!NEAR || i == 0) continue;
    const bool edge = i >= 7;
    if (nt(i) >= T_INLET &&
        !(NEE && edge && I.nee && (nt(edge_a(i)) == T_FLUID || nt(edge_b(i)) == T_FLUID))) {
      const R out = ghost_value(i, nt(i), (uint32_t)(c - off[i]), v);
      if (!ODD) put(OPP[i], (uint32_t)(c - off[i]) * ES, out);
      else put(i, c * ES, out);
    }
    if (NEE && edge && I.nee) {
      // this cell as the normal neighbour of the ghost c - e_k, handing
      // direction i to the receiver c + e_t (e_i = e_k + e_t)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = h == 0 ? edge_a(i) : edge_b(i);
        const int t = h == 0 ? edge_b(i) : edge_a(i);
        if (nt(k) >= T_INLET && nt(OPP[t]) == T_FLUID) {
          const R out = ghost_value(i, nt(k), (uint32_t)(c - off[k]), v);
          if (!ODD) put(OPP[i], (uint32_t)(c - off[k]) * ES, out);
          else put(i, (uint32_t)(c + off[t]) * ES, out);
        }
      }
    }
  }
}

// one lattice cell (local index of instance inst) of the collide-stream step
// mode: COLLIDE_ALL, COLLIDE_BULK (cells outside the wall band) or
// COLLIDE_BAND (band cells only).  A cell writes the slots it reads, and
// next to a wall or ghost also slots that no fluid cell reads in the step
// (a solid's or ghost's slot, or an own slot whose reader is a solid), so
// the two partial passes touch disjoint memory and the bulk pass may run
// while the wall exchange still reads the band cells' populations.  The body is chosen per wave (a vote over its
// active lanes), so the choice never splits a wave.
template <class S, bool ODD, bool NEE, bool COUNT = false>
__device__ __forceinline__ void collide_cell(const Dev& d, const int inst, const int64_t local, const int mode) {
  const InstDesc& I = d.inst[inst];
  if (local >= I.ncell) return;
  // global cell index fits 32 bits (NT < 2^31); per-direction arrays are
  // addressed as uniform base + 32-bit lane offset
  const uint32_t c = (uint32_t)(I.cell0 + local);
  // the instance's error word is loaded beside the cell's flags, so that
  // the two latencies overlap; a frozen instance is left alone
  const uint8_t fl = d.flags[c];
  const uint32_t ew = d.err[inst];
  if ((fl & TYPE_MASK) != T_FLUID || (ew & ERR_FROZEN)) return;
  if (mode != COLLIDE_ALL && ((fl & F_BAND) != 0) != (mode == COLLIDE_BAND)) return;
  if (__any(fl & F_NEAR))
    collide_body<S, ODD, true, true, NEE, COUNT>(d, inst, I, local, c, fl);
  else if (__any(fl & F_BAND))
    collide_body<S, ODD, false, true, NEE, COUNT>(d, inst, I, local, c, fl);
  else
    collide_body<S, ODD, false, false, NEE, COUNT>(d, inst, I, local, c, fl);
}

// One workgroup of BS lanes per tile of BS * CPT consecutive cells of one
// instance (the tile table of a size class); lane t takes cells start + t,
// start + t + BS, ... so every load and store stays coalesced.  BS and CPT
// are chosen per size class by the autotuner.  NEE: built with the
// normal-neighbour extrapolation (a separate kernel, launched only over the
// tiles that hold a cell next to a 0D ghost, so that every other tile keeps
// the smaller register budget).
template <class S, bool ODD, int BS, int CPT, bool NEE>
__global__ __launch_bounds__(BS) void k_collide(Dev d, const CTile* __restrict__ tab, int mode) {
  const CTile t = tab[blockIdx.x];
#pragma unroll
  for (int q = 0; q < CPT; ++q) collide_cell<S, ODD, NEE>(d, t.inst, (int64_t)t.start + q * BS + (int)threadIdx.x, mode);
}

// The slot-writer check of the AA pattern: the FP32 collide with every
// population store replaced by an atomic count of its slot in d.slotcnt
// (19 * NT counters), over tiles of 256 cells; the populations are left as
// they are.  A race-free step writes each slot at most once, and every slot
// a fluid cell reads in the next step exactly once.
template <bool ODD, bool NEE>
__global__ __launch_bounds__(256) void k_collide_count(Dev d, const CTile* __restrict__ tab) {
  const CTile t = tab[blockIdx.x];
  collide_cell<float, ODD, NEE, true>(d, t.inst, (int64_t)t.start + (int)threadIdx.x, COLLIDE_ALL);
}

// ---------------------------------------------------------------------------
// k_band: unforced velocity of band cells, force cleared
// ---------------------------------------------------------------------------
// The 18 moving directions only (e_0 = 0); all loads are independent of each
// other, so a wave keeps all of them in flight (band cells form short runs
// along x, and the kernel is bound by the partly used cache lines).
template <class S, bool ODD>
__device__ __forceinline__ void band_block(const Dev& d, const int wall, const int bx) {
  using R = typename Store<S>::R;
  using R4 = typename V4<R>::T;
  const int inst = d.walls[wall];
  if (d.err[inst] & ERR_FROZEN) return;
  const InstDesc& I = d.inst[inst];
  // chunk bx of this wall's band, in XCD-aware order over the wall's own
  // chunks (its workgroups are consecutive, so they go to the XCDs in turn)
  const int nb = (I.nband + WBLOCK - 1) / WBLOCK;
  if (bx >= nb) return;
  const int k = xcd_tile(bx, nb) * WBLOCK + threadIdx.x;
  if (k >= I.nband) return;
  const int64_t lc = I.band[k];
  const int64_t c = I.cell0 + lc;
  const int64_t NT = d.NT;
  const S* __restrict__ A = (const S*)d.pop;
  const float inv = d.inv_scale;
  R g[NQ];
  if (!ODD) {
#pragma unroll
    for (int i = 1; i < NQ; ++i) g[i] = Store<S>::ld(A + i * NT + c, inv);
  } else {
    // odd step: g_i = A[opp i][c - e_i] (bounce-back values included)
    int64_t off[NQ];
    dir_offsets(I.nx, (int64_t)I.nx * I.ny, off);
#pragma unroll
    for (int i = 1; i < NQ; ++i) g[i] = Store<S>::ld(A + OPP[i] * NT + c - off[i], inv);
  }
  R jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int i = 1; i < NQ; ++i) {
    jx += EX[i] * g[i];
    jy += EY[i] * g[i];
    jz += EZ[i] * g[i];
  }
  ((R4*)I.u4)[lc] = R4{jx, jy, jz, R(0)};
  ((R4*)I.b4)[lc] = R4{0, 0, 0, 0};
}

template <class S, bool ODD>
__global__ __launch_bounds__(WBLOCK) void k_band(Dev d) {
  band_block<S, ODD>(d, blockIdx.y, blockIdx.x);
}

// The boundary reductions and the band moments in one launch: the first
// nred workgroups reduce (few, latency-bound), the others take nbx band
// workgroups per wall.  The two read populations only and write disjoint
// state, so the reductions run in the shadow of the band's memory traffic.
template <class S, bool ODD>
__global__ __launch_bounds__(WBLOCK) void k_reduce_band(Dev d, int nred, int nbx) {
  static_assert(RBLOCK == WBLOCK, "one workgroup size for both parts");
  const int b = (int)blockIdx.x;
  if (b < nred) {
    reduce_block<S, ODD>(d, b);
  } else {
    band_block<S, ODD>(d, (b - nred) / nbx, (b - nred) % nbx);
  }
}

// ---------------------------------------------------------------------------
// k_wall: one lane per wall point
// ---------------------------------------------------------------------------
template <class R>
__device__ __forceinline__ R phi4(R r) {
  // both branches evaluated (their square roots clamped where unused) and
  // the result selected, so the 12 weights of a point take no branch
  r = fabs(r);
  const R a = (R(3) - R(2) * r + sqrt(fmax(R(1) + R(4) * r - R(4) * r * r, R(0)))) * R(0.125);
  const R b = (R(5) - R(2) * r - sqrt(fmax(R(-7) + R(12) * r - R(4) * r * r, R(0)))) * R(0.125);
  return r <= R(1) ? a : (r < R(2) ? b : R(0));
}

// the 4-point cosine delta (1 + cos(pi r / 2)) / 4 on |r| < 2 (variant kernel)
template <class R>
__device__ __forceinline__ R phicos(R r) {
  r = fabs(r);
  const R v = R(0.25) * (R(1) + cos(R(1.5707963267948966) * r));
  return r < R(2) ? v : R(0);
}

// Add to device memory with a global (not flat) atomic and no returned
// value: a flat atomic also counts as an LDS operation, so the wait of the
// next LDS read (or of any later load) would wait for it to complete; this
// one nothing waits for.
__device__ __forceinline__ void gadd(float* p, float v) {
  (void)__builtin_amdgcn_global_atomic_fadd_f32((__attribute__((address_space(1))) float*)p, v);
}
__device__ __forceinline__ void gadd(double* p, double v) {
  (void)__builtin_amdgcn_global_atomic_fadd_f64((__attribute__((address_space(1))) double*)p, v);
}

__device__ __forceinline__ double3 ld3(const double* p, int64_t k) {
  const double4 v = ((const double4*)p)[k];
  return make_double3(v.x, v.y, v.z);
}

// tension vector T D0 X on a half edge with edge vector e (Eq. tension)
__device__ __forceinline__ double3 tension(double3 e, double ds, double ks) {
  const double dx = e.x / ds, dy = e.y / ds, dz = e.z / ds;
  const double T = ks * (sqrt(dx * dx + dy * dy + dz * dz) - 1.0);
  return make_double3(T * dx, T * dy, T * dz);
}

// fixed-point accumulator type for the LDS spreading: same width as R
template <class R> struct FixOf;
template <> struct FixOf<float> {
  using T = int;
  static constexpr int M = 23;
  __device__ static void add(int* p, float v) { atomicAdd(p, __float2int_rn(v)); }
};
template <> struct FixOf<double> {
  using T = long long;
  static constexpr int M = 52;
  __device__ static void add(long long* p, double v) {
    atomicAdd((unsigned long long*)p, (unsigned long long)__double2ll_rn(v));
  }
};

// Wall points are processed in tiles of TJ x TK mesh points (theta x z), one
// tile per 256-lane workgroup.  The tile's stencils span a small box of
// lattice cells; when it fits in LDS the band velocity of the box is staged
// there for the interpolation, and the same LDS then accumulates the spread
// force with LDS atomics before one flush of the box's non-zero cells with
// global atomics (instead of 64 x 3 global atomics per point).
// The tile shape TJ x TK is chosen per size class by the autotuner: 256
// points wide in theta (32 x 8), square (16 x 16) or long in z (8 x 32), or
// the smaller 8 x 16, 16 x 8 and 8 x 8 tiles, whose stencil boxes still fit
// the staging memory on coarse meshes (there the 256 lanes stage and flush
// the box, and a lane per point takes the stencils while the others idle).
// In the staged path the 4 x 4 x 4 stencil loops are unrolled and free of
// branches: each staged cell holds (u, m) with u = 0 outside the band and
// m = 1 at a fluid cell outside the band, so one 16-byte LDS read per
// stencil cell serves both the interpolation and the band check; tile-wide
// extents and maxima are reduced within each wave first, so only one lane
// per wave touches the shared LDS word.
// colour >= 0 (the deterministic spreading mode): only the tiles of that
// colour, (theta tile parity) + 2 (z tile parity), or 4 + (z tile parity) for
// the last theta column of an odd ring (theta is periodic); the host launches
// the colours one after another, so a cell receives the tiles' sums in colour
// order wherever tiles of one colour do not share a cell.
template <class R, int TJ, int TK, bool BIG>
__global__ __launch_bounds__(WBLOCK) void k_wall(Dev d, const int32_t* __restrict__ walls, int parity, int colour) {
  static_assert(TJ * TK <= WBLOCK && TJ % 2 == 0 && TK % 2 == 0, "one lane per point of the tile");
  using R4 = typename V4<R>::T;
  using Fix = typename FixOf<R>::T;
  // box cells: at 0.5 lu spacing a 16 x 16 or 8 x 32 tile spans <= ~1100,
  // a 32 x 8 tile <= ~1700; at ~0.9 lu a 16 x 16 tile up to ~3500 (BIG,
  // which trades occupancy for staging), an 8 x 16 tile ~1500 and an 8 x 8
  // tile ~900; a larger box takes the unstaged path
  constexpr int BOXCAP = BIG ? wall_boxcap_big(sizeof(R)) : wall_boxcap(sizeof(R), TJ);
  static_assert(3 * sizeof(Fix) <= sizeof(R4), "the spread accumulators reuse the staging box");
  __shared__ R4 sbox[BOXCAP];
  __shared__ uint8_t sfl[BOXCAP];
  __shared__ int sext[6];   // min x, y, z; max x, y, z of the stencil bases
  __shared__ int semax;
  const int inst = walls[blockIdx.y];
  if (d.err[inst] & ERR_FROZEN) return;   // whole block leaves
  const InstDesc& I = d.inst[inst];
  const int nth = I.nth, nzl = I.nzl;
  const int ntj = (nth + TJ - 1) / TJ;
  const int bx = (int)blockIdx.x;
  if (bx >= ntj * ((nzl + TK - 1) / TK)) return;  // whole block leaves
  if (colour >= 0) {
    const int jt = bx % ntj, kt = bx / ntj;
    const int col = ((ntj & 1) && jt == ntj - 1) ? 4 + (kt & 1) : (jt & 1) + 2 * (kt & 1);
    if (col != colour) return;   // whole block leaves
  }
  // wave w takes the parity sub-lattice (w & 1, w >> 1) of the TJ x TK patch:
  // its (TJ/2) x (TK/2) points are >= 1 lu apart, so for a given stencil
  // offset the 64 lanes mostly hit distinct cells and the LDS atomics do not
  // serialise.
  const int wv = (int)threadIdx.x >> 6, ln = (int)threadIdx.x & 63;
  const int j = (bx % ntj) * TJ + 2 * (ln % (TJ / 2)) + (wv & 1);
  const int k = (bx / ntj) * TK + 2 * (ln / (TJ / 2)) + (wv >> 1);
  const bool point = ln < (TJ / 2) * (TK / 2) && j < nth && k < nzl;
  const int64_t p = point ? j + (int64_t)nth * k : 0;
  // the wall is carried as displacement D = X - X0 (ping-pong D^n / D^{n-1})
  const double* Dc = I.Xab[parity];
  double* Dn = I.Xab[parity ^ 1];
  const double3 X0 = ld3(I.X0, p), D = ld3(Dc, p), Dm = ld3(Dn, p);
  double4* SL = (double4*)I.slip;
  // the instance fields used after this kernel's first global stores, read
  // now: read through I after a store that might alias it, each would be a
  // vector load waited for together with the stores before it
  const double ialpha = I.alpha, ibeta = I.beta, iarea = I.area;
  R4* const IVf = (R4*)I.Vf;
  double4* const IFp = (double4*)I.Fp;
  R* const B = (R*)I.b4;
  const int64_t snx = I.nx, snxy = (int64_t)I.nx * I.ny;
  double4 sl = SL[p];   // the slip integral, loaded with the rest of the point's state
  // A point that is not finite or has left the lattice box (a run that has
  // blown up) cannot be in its band: it is flagged and takes no part, so
  // that no stencil index is ever formed from it (the comparisons are false
  // for NaN).
  const double px = X0.x + D.x, py = X0.y + D.y, pz = X0.z + D.z;
  const bool inside = px >= -1.0 && py >= -1.0 && pz >= -1.0 && px <= (double)I.nx &&
                      py <= (double)I.ny && pz <= (double)I.nz;
  if (point && !inside) atomicOr(d.err + inst, ERR_BAND);
  const bool valid = point && inside;

  if (threadIdx.x < 6) sext[threadIdx.x] = threadIdx.x < 3 ? 0x7fffffff : -0x7fffffff;
  if (threadIdx.x == 0) semax = -100000;
  __syncthreads();
  const int bx0 = valid ? (int)floor(px) - 1 : 0, by0 = valid ? (int)floor(py) - 1 : 0,
            bz0 = valid ? (int)floor(pz) - 1 : 0;
  {   // wave reductions over the active (here: all) lanes, one atomic per wave
    const int lo[3] = {__ockl_wfred_min_i32(valid ? bx0 : 0x7fffffff), __ockl_wfred_min_i32(valid ? by0 : 0x7fffffff),
                       __ockl_wfred_min_i32(valid ? bz0 : 0x7fffffff)};
    const int hi[3] = {__ockl_wfred_max_i32(valid ? bx0 : -0x7fffffff), __ockl_wfred_max_i32(valid ? by0 : -0x7fffffff),
                       __ockl_wfred_max_i32(valid ? bz0 : -0x7fffffff)};
    if (ln == 0) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        atomicMin(&sext[a], lo[a]);
        atomicMax(&sext[3 + a], hi[a]);
      }
    }
  }
  R wx[4], wy[4], wz[4];
  const bool cosk = I.kernel == 1;   // uniform over the launch's instance
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const R rx = (R)(((double)(bx0 + a) - X0.x) - D.x), ry = (R)(((double)(by0 + a) - X0.y) - D.y),
            rz = (R)(((double)(bz0 + a) - X0.z) - D.z);
    wx[a] = cosk ? phicos<R>(rx) : phi4<R>(rx);
    wy[a] = cosk ? phicos<R>(ry) : phi4<R>(ry);
    wz[a] = cosk ? phicos<R>(rz) : phi4<R>(rz);
  }
  __syncthreads();
  // every valid point has its stencil base in [-2, n], so the extents are
  // small and positive; a tile without a valid point has min > max
  const int ox = sext[0], oy = sext[1], oz = sext[2];
  const bool any = sext[0] <= sext[3];
  const int ex = any ? sext[3] - ox + 4 : 0, ey = any ? sext[4] - oy + 4 : 0, ez = any ? sext[5] - oz + 4 : 0;
  const int64_t vol = (int64_t)ex * ey * ez;
  const bool staged = any && vol <= BOXCAP;   // uniform over the block
  const int exy = ex * ey;
  // box index q -> cell by float division: exact, as (q + 0.5) / n sits at
  // least 0.5 / n from an integer and q < 2^21 keeps the rounding far below
  const float rex = 1.0f / (float)max(ex, 1), rexy = 1.0f / (float)max(exy, 1);
  const R4* U = (const R4*)I.u4;
  auto box_cell = [&](int q, int& x, int& y, int& z) {
    const int zq = (int)(((float)q + 0.5f) * rexy);
    const int r = q - zq * exy;
    const int yq = (int)(((float)r + 0.5f) * rex);
    x = ox + (r - yq * ex);
    y = oy + yq;
    z = oz + zq;
  };
  const int inx = I.nx, iny = I.ny, inz = I.nz;
  const int64_t icell0 = I.cell0;
  auto in_box = [&](int x, int y, int z) { return x >= 0 && y >= 0 && z >= 0 && x < inx && y < iny && z < inz; };
  // first box index of a point's stencil
  const int q0 = valid && staged ? (bx0 - ox) + ex * ((by0 - oy) + ey * (bz0 - oz)) : 0;

  // ---- interpolation of the unforced velocity over the 4x4x4 stencil ----
  if (staged) {
    // the flag byte and the band velocity of a box cell are loaded together
    // (the velocity array spans the instance's cells; only band cells hold a
    // current value, the others are masked by the flag afterwards), so a
    // lane's loads do not wait on each other
    for (int q = threadIdx.x; q < (int)vol; q += WBLOCK) {
      int x, y, z;
      box_cell(q, x, y, z);
      uint8_t f = T_SOLID;
      R4 u = {0, 0, 0, 0};
      if (in_box(x, y, z)) {
        const int64_t lc = x + (int64_t)I.nx * (y + (int64_t)I.ny * z);
        f = d.flags[I.cell0 + lc];
        const R4 v = U[lc];
        const bool fluid = (f & TYPE_MASK) == T_FLUID, band = (f & F_BAND) != 0;
        u = R4{fluid && band ? v.x : R(0), fluid && band ? v.y : R(0), fluid && band ? v.z : R(0),
               fluid && !band ? R(1) : R(0)};
      }
      sfl[q] = f;
      sbox[q] = u;
    }
    __syncthreads();
  }
  R Vx = 0, Vy = 0, Vz = 0;
  bool outside = false;
  if (valid && staged) {
    R o = 0;   // > 0 iff a stencil weight != 0 falls on fluid outside the band
#pragma unroll
    for (int cz = 0; cz < 4; ++cz)
#pragma unroll
      for (int cy = 0; cy < 4; ++cy) {
        const R wyz = wy[cy] * wz[cz];
        const R4* row = sbox + q0 + ex * cy + exy * cz;
#pragma unroll
        for (int cx = 0; cx < 4; ++cx) {
          const R4 u = row[cx];
          const R w = wx[cx] * wyz;
          Vx += u.x * w;
          Vy += u.y * w;
          Vz += u.z * w;
          o = fmax(o, u.w * fabs(w));
        }
      }
    outside = o > R(0);
  } else if (valid) {
    for (int cz = 0; cz < 4; ++cz)
      for (int cy = 0; cy < 4; ++cy) {
        const R wyz = wy[cy] * wz[cz];
        for (int cx = 0; cx < 4; ++cx) {
          const int x = bx0 + cx, y = by0 + cy, z = bz0 + cz;
          if (!in_box(x, y, z)) continue;
          const int64_t lc = x + (int64_t)I.nx * (y + (int64_t)I.ny * z);
          const uint8_t f = d.flags[I.cell0 + lc];
          if ((f & TYPE_MASK) != T_FLUID) continue;
          const R w = wx[cx] * wyz;
          if (!(f & F_BAND)) {
            if (w != R(0)) outside = true;
            continue;
          }
          const R4 u = U[lc];
          Vx += u.x * w; Vy += u.y * w; Vz += u.z * w;
        }
      }
  }
  if (outside) atomicOr(d.err + inst, ERR_BAND);

  // ---- penalty force on the fluid (Eq. LagForce) ----
  double Fx = 0, Fy = 0, Fz = 0;
  if (valid) {
    const double dxv = (double)Vx - (D.x - Dm.x);
    const double dyv = (double)Vy - (D.y - Dm.y);
    const double dzv = (double)Vz - (D.z - Dm.z);
    sl.x += dxv; sl.y += dyv; sl.z += dzv;
    SL[p] = sl;
    Fx = ialpha * sl.x + ibeta * dxv;
    Fy = ialpha * sl.y + ibeta * dyv;
    Fz = ialpha * sl.z + ibeta * dzv;
    IVf[p] = R4{Vx, Vy, Vz, R(0)};
    IFp[p] = double4{Fx, Fy, Fz, 0.0};
  }

  // ---- spreading (Eq. EulForce): b(node) += F area delta ----
  // (B, snx, snxy: read up front, as above; read through I after an atomic
  // on B they would be reloaded, and waited for, in every flush iteration)
  const R fx = (R)(Fx * iarea), fy = (R)(Fy * iarea), fz = (R)(Fz * iarea);
  // Spreading into the LDS box in fixed point: integer LDS atomics run at
  // full rate where float ones do not, and an integer sum is exact, so the
  // result does not depend on the order of the tile's contributions.  The
  // scale is a power of two per tile, 2^(M - e) with e the exponent of the
  // tile's largest |F area| and M the significand width of R (headroom of
  // 2^7 resp. 2^10 for the sums).
  if (staged) {
    __syncthreads();  // everyone is done reading the staged velocity
    Fix* acc = (Fix*)sbox;
    for (int q = threadIdx.x; q < (int)vol; q += WBLOCK) sbox[q] = R4{0, 0, 0, 0};
    int em = -100000;
    if (valid) {
      const R m = fmax(fabs(fx), fmax(fabs(fy), fabs(fz)));
      if (m > R(0)) em = (int)ilogb(m);
    }
    em = __ockl_wfred_max_i32(em);
    if (ln == 0 && em > -100000) atomicMax(&semax, em);
    __syncthreads();
    const int e = semax < -1000 ? 0 : semax;
    const R S = ldexp(R(1), FixOf<R>::M - e), invS = ldexp(R(1), e - FixOf<R>::M);
    if (valid) {
      const R sx = fx * S, sy = fy * S, sz = fz * S;
#pragma unroll
      for (int cz = 0; cz < 4; ++cz)
#pragma unroll
        for (int cy = 0; cy < 4; ++cy) {
          const R wyz = wy[cy] * wz[cz];
          Fix* row = acc + 3 * (q0 + ex * cy + exy * cz);
#pragma unroll
          for (int cx = 0; cx < 4; ++cx) {
            const R w = wx[cx] * wyz;
            FixOf<R>::add(row + 3 * cx, sx * w);
            FixOf<R>::add(row + 3 * cx + 1, sy * w);
            FixOf<R>::add(row + 3 * cx + 2, sz * w);
          }
        }
    }
    __syncthreads();
    // the flush: lane t takes component t % 4 (the fourth idles) of box cell
    // t / 4, so one atomic instruction of a wave covers 16 consecutive cells'
    // components, two 128-byte lines of the force array in FP32, where one
    // component of 64 cells touched eight (the L2 takes float atomics per
    // line: 161 -> 133 us of wall + membrane on the 0.5 lu tube in motion)
    for (int q4 = threadIdx.x; q4 < 4 * (int)vol; q4 += WBLOCK) {
      const int q = q4 >> 2, c3 = q4 & 3;
      const uint8_t f = sfl[q];
      if (c3 == 3 || (f & TYPE_MASK) != T_FLUID || !(f & F_BAND)) continue;
      const Fix a = acc[3 * q + c3];
      if (a == 0) continue;
      int x, y, z;
      box_cell(q, x, y, z);
      gadd(B + 4 * (x + snx * y + snxy * z) + c3, (R)a * invS);
    }
  } else if (valid) {
    for (int cz = 0; cz < 4; ++cz)
      for (int cy = 0; cy < 4; ++cy) {
        const R wyz = wy[cy] * wz[cz];
        for (int cx = 0; cx < 4; ++cx) {
          const int x = bx0 + cx, y = by0 + cy, z = bz0 + cz;
          if (!in_box(x, y, z)) continue;
          const int64_t lc = x + snx * y + snxy * z;
          const uint8_t f = d.flags[icell0 + lc];
          if ((f & TYPE_MASK) != T_FLUID || !(f & F_BAND)) continue;
          const R w = wx[cx] * wyz;
          if (w == R(0)) continue;
          gadd(B + 4 * lc + 0, fx * w);
          gadd(B + 4 * lc + 1, fy * w);
          gadd(B + 4 * lc + 2, fz * w);
        }
      }
  }
}

// k_motion: largest displacement of a wall point since its band was built
// (max norm; positive floats order as their bit patterns) into the moved
// word, launched right before the host's wall-motion test rather than in
// every step.  D is the current displacement (Xab of the step parity).
// Each workgroup strides over the points (MOTION_BLOCKS workgroups per wall)
// and reduces in LDS, so that one atomic per workgroup reaches the moved
// word: one per wave made the atomics on that single word the kernel's cost.
constexpr int MOTION_BLOCKS = 256;
__global__ __launch_bounds__(WBLOCK) void k_motion(Dev d, int parity) {
  __shared__ uint32_t red[WBLOCK / 64];
  const int inst = d.walls[blockIdx.y];
  if (d.err[inst] != 0u) return;   // failed instances take no part in the test (whole block)
  const InstDesc& I = d.inst[inst];
  uint32_t mv = 0u;
  for (int64_t p = (int64_t)blockIdx.x * WBLOCK + threadIdx.x; p < I.np; p += (int64_t)gridDim.x * WBLOCK) {
    const double3 D = ld3(I.Xab[parity], p), Dr = ld3(I.Dref, p);
    mv = max(mv, __float_as_uint((float)fmax(fabs(D.x - Dr.x), fmax(fabs(D.y - Dr.y), fabs(D.z - Dr.z)))));
  }
  mv = __ockl_wfred_max_u32(mv);   // all lanes of the wave are active here
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mv;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t m = red[0];
    for (int w = 1; w < WBLOCK / 64; ++w) m = max(m, red[w]);
    if (m != 0u) atomicMax(d.moved, m);
  }
}

// ---------------------------------------------------------------------------
// k_wss: wall shear stress at every point of one wall (diagnostic, not on the
// step's path).  The mesh tangents give the inward normal n and the axial
// direction a; the fluid velocity sum e g of the FLUID cells around
// Y = X + dist n is interpolated trilinearly (weights renormalised over the
// FLUID cells; NaN if none), and WSS = mu ((v(Y) - V_wall) . a) / dist.
// ---------------------------------------------------------------------------
template <class S, bool ODD>
__global__ __launch_bounds__(WBLOCK) void k_wss(Dev d, int inst, double dist, double mu, double* __restrict__ out) {
  using R = typename Store<S>::R;
  const InstDesc& I = d.inst[inst];
  const int64_t p = (int64_t)blockIdx.x * WBLOCK + threadIdx.x;
  if (p >= I.np) return;
  const int nth = I.nth, nzl = I.nzl;
  const int j = (int)(p % nth), k = (int)(p / nth);
  const double* Dc = I.Xab[ODD ? 1 : 0];
  const double* Dm = I.Xab[ODD ? 0 : 1];
  auto pos = [&](int64_t q) {
    const double3 a = ld3(I.X0, q), b = ld3(Dc, q);
    return make_double3(a.x + b.x, a.y + b.y, a.z + b.z);
  };
  const double3 X = pos(p);
  const double3 e = pos((j + 1) % nth + (int64_t)nth * k), w = pos((j + nth - 1) % nth + (int64_t)nth * k);
  const double3 up = pos(k < nzl - 1 ? p + nth : p), dn = pos(k > 0 ? p - nth : p);
  const double3 tt = make_double3(e.x - w.x, e.y - w.y, e.z - w.z);
  const double3 tz = make_double3(up.x - dn.x, up.y - dn.y, up.z - dn.z);
  double3 n = make_double3(-(tt.y * tz.z - tt.z * tz.y), -(tt.z * tz.x - tt.x * tz.z), -(tt.x * tz.y - tt.y * tz.x));
  const double nn = sqrt(n.x * n.x + n.y * n.y + n.z * n.z), na = sqrt(tz.x * tz.x + tz.y * tz.y + tz.z * tz.z);
  n.x /= nn; n.y /= nn; n.z /= nn;
  const double3 a = make_double3(tz.x / na, tz.y / na, tz.z / na);
  const double3 Dn = ld3(Dc, p), Dp = ld3(Dm, p);
  const double Y[3] = {X.x + dist * n.x, X.y + dist * n.y, X.z + dist * n.z};
  const int b[3] = {(int)floor(Y[0]), (int)floor(Y[1]), (int)floor(Y[2])};
  int64_t off[NQ];
  dir_offsets(I.nx, (int64_t)I.nx * I.ny, off);
  const S* A = (const S*)d.pop;
  double vx = 0, vy = 0, vz = 0, ws = 0;
  for (int cz = 0; cz < 2; ++cz)
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx) {
        const int x = b[0] + cx, y = b[1] + cy, z = b[2] + cz;
        if (x < 0 || y < 0 || z < 0 || x >= I.nx || y >= I.ny || z >= I.nz) continue;
        const int64_t c = I.cell0 + x + (int64_t)I.nx * (y + (int64_t)I.ny * z);
        if ((d.flags[c] & TYPE_MASK) != T_FLUID) continue;
        const double wt = (cx ? Y[0] - b[0] : 1.0 - (Y[0] - b[0])) * (cy ? Y[1] - b[1] : 1.0 - (Y[1] - b[1])) *
                          (cz ? Y[2] - b[2] : 1.0 - (Y[2] - b[2]));
        R g[NQ];
        load_cell<S, ODD>(A, d.NT, c, off, d.inv_scale, g);
        double jx = 0, jy = 0, jz = 0;
#pragma unroll
        for (int i = 1; i < NQ; ++i) {
          jx += EX[i] * (double)g[i];
          jy += EY[i] * (double)g[i];
          jz += EZ[i] * (double)g[i];
        }
        vx += wt * jx; vy += wt * jy; vz += wt * jz;
        ws += wt;
      }
  if (!(ws > 0.0)) {
    out[p] = __builtin_nan("");
    return;
  }
  const double s = (vx / ws - (Dn.x - Dp.x)) * a.x + (vy / ws - (Dn.y - Dp.y)) * a.y + (vz / ws - (Dn.z - Dp.z)) * a.z;
  out[p] = mu * s / dist;
}

// ---------------------------------------------------------------------------
// Band rebuild on the device (launched at each band check, gated on the
// motion word).  The band of a wall is the FLUID cells within the margin m of
// the 4x4x4 stencils of its points: the stencil bases b = floor(X) - 1
// (clamped into the box) are marked, the marks are dilated to
// [b - m, b + 3 + m] along x, y and z in turn (one running window per
// line), the band bits of the flags are set from the result and the band
// list is compacted in ascending cell order.  Every kernel leaves at once
// when the gate is shut.  Invariant: bmark is zero between rebuilds.
// ---------------------------------------------------------------------------
__global__ void k_band_gate(Dev d, float thresh) {
  if (threadIdx.x != 0) return;
  const float moved = __uint_as_float(*d.moved);
  const uint32_t open = moved < thresh ? 0u : 1u;   // a NaN motion opens it as well
  *d.gate = open;
  if (open) *d.moved = 0u;
}

__global__ __launch_bounds__(WBLOCK) void k_band_seed(Dev d, int parity) {
  if (*d.gate == 0u) return;
  const int inst = d.walls[blockIdx.y];
  if (d.err[inst] != 0u) return;   // failed instances get an empty band
  const InstDesc& I = d.inst[inst];
  const int64_t p = (int64_t)blockIdx.x * WBLOCK + threadIdx.x;
  if (p >= I.np) return;
  const double3 X0 = ld3(I.X0, p), D = ld3(I.Xab[parity], p);
  ((double4*)I.Dref)[p] = double4{D.x, D.y, D.z, 0.0};
  const double x = X0.x + D.x, y = X0.y + D.y, z = X0.z + D.z;
  // a non-finite point (or one far outside the box) fails its instance; the
  // comparisons are false for NaN
  if (!(fabs(x) <= 1e9 && fabs(y) <= 1e9 && fabs(z) <= 1e9)) {
    atomicOr(d.err + inst, ERR_NONFINITE | ERR_FROZEN);
    return;
  }
  const int bx = min(max((int)floor(x) - 1, 0), I.nx - 1);
  const int by = min(max((int)floor(y) - 1, 0), I.ny - 1);
  const int bz = min(max((int)floor(z) - 1, 0), I.nz - 1);
  d.bmark[I.cell0 + bx + (int64_t)I.nx * (by + (int64_t)I.ny * bz)] = 1;
}

// one lane per line along axis of one walled instance: out[i] = 1 when in
// holds a mark in [i - 3 - m, i + m] on the line
__global__ __launch_bounds__(WBLOCK) void k_band_dilate(Dev d, int axis, const uint8_t* __restrict__ in,
                                                        uint8_t* __restrict__ out) {
  if (*d.gate == 0u) return;
  const InstDesc& I = d.inst[d.walls[blockIdx.y]];
  const int64_t q = (int64_t)blockIdx.x * WBLOCK + threadIdx.x;
  const int64_t sxy = (int64_t)I.nx * I.ny;
  int n;
  int64_t c0, st;
  if (axis == 0) {          // lines (y, z)
    if (q >= (int64_t)I.ny * I.nz) return;
    n = I.nx; c0 = q * I.nx; st = 1;
  } else if (axis == 1) {   // lines (x, z)
    if (q >= (int64_t)I.nx * I.nz) return;
    n = I.ny; c0 = q % I.nx + sxy * (q / I.nx); st = I.nx;
  } else {                  // lines (x, y)
    if (q >= sxy) return;
    n = I.nz; c0 = q; st = sxy;
  }
  const int m = I.band_margin;
  const int64_t base = I.cell0 + c0;
  int cnt = 0;
  for (int i = -3 - m; i < n; ++i) {
    const int add = i + m, drop = i - 4 - m;
    if (add >= 0 && add < n) cnt += in[base + add * st];
    if (drop >= 0 && drop < n) cnt -= in[base + drop * st];
    if (i >= 0) out[base + i * st] = cnt > 0 ? 1 : 0;
  }
}

// sum over a 256-lane workgroup (every lane active)
__device__ __forceinline__ int block_sum(int v, int* sh) {
  v = __ockl_wfred_add_i32(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  const int t = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return t;
}

// exclusive prefix over a 256-lane workgroup (every lane active)
__device__ __forceinline__ int block_prefix(int v, int* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < WBLOCK; off <<= 1) {
    const int a = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += a;
    __syncthreads();
  }
  const int r = sh[threadIdx.x] - v;
  __syncthreads();
  return r;
}

// band bits from the dilated marks (FLUID cells only), marks cleared, band
// cells counted per block of BCELLS cells (4 consecutive cells per lane)
__global__ __launch_bounds__(WBLOCK) void k_band_flags(Dev d) {
  __shared__ int sh[4];
  if (*d.gate == 0u) return;
  const InstDesc& I = d.inst[d.walls[blockIdx.y]];
  const int64_t b0 = (int64_t)blockIdx.x * BCELLS;
  if (b0 >= I.ncell) return;   // whole block
  uint8_t* fl = (uint8_t*)d.flags;
  int cnt = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t lc = b0 + 4 * threadIdx.x + q;
    if (lc >= I.ncell) break;
    const int64_t c = I.cell0 + lc;
    const uint8_t f = fl[c];
    const bool band = d.btmp[c] != 0 && (f & TYPE_MASK) == T_FLUID;
    const uint8_t nf = band ? (uint8_t)(f | F_BAND) : (uint8_t)(f & ~F_BAND);
    if (nf != f) fl[c] = nf;
    d.bmark[c] = 0;
    cnt += band ? 1 : 0;
  }
  cnt = block_sum(cnt, sh);
  if (threadIdx.x == 0) d.bcnt[I.cblk0 + blockIdx.x] = cnt;
}

// exclusive scan of each wall's block counts (one workgroup per wall); the
// total is the new band size, and a band past the list's capacity fails
// the instance
__global__ __launch_bounds__(WBLOCK) void k_band_scan(Dev d) {
  __shared__ int sh[WBLOCK];
  if (*d.gate == 0u) return;
  const int inst = d.walls[blockIdx.x];
  InstDesc& I = ((InstDesc*)d.inst)[inst];
  const int nblk = (int)((I.ncell + BCELLS - 1) / BCELLS);
  int32_t* cnt = d.bcnt + I.cblk0;
  const int per = (nblk + WBLOCK - 1) / WBLOCK;
  const int lo = min(nblk, (int)threadIdx.x * per), hi = min(nblk, lo + per);
  int s = 0;
  for (int b = lo; b < hi; ++b) s += cnt[b];
  int run = block_prefix(s, sh);
  for (int b = lo; b < hi; ++b) {
    const int v = cnt[b];
    cnt[b] = run;
    run += v;
  }
  if (threadIdx.x == WBLOCK - 1) {
    if (run > I.band_cap) atomicOr(d.err + inst, ERR_BAND | ERR_FROZEN);
    else I.nband = run;
  }
}

// the band list: cell ids in ascending order at the scanned block offsets
__global__ __launch_bounds__(WBLOCK) void k_band_write(Dev d) {
  __shared__ int sh[WBLOCK];
  if (*d.gate == 0u) return;
  const InstDesc& I = d.inst[d.walls[blockIdx.y]];
  const int64_t b0 = (int64_t)blockIdx.x * BCELLS;
  if (b0 >= I.ncell) return;   // whole block
  bool in[4];
  int cnt = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t lc = b0 + 4 * threadIdx.x + q;
    in[q] = lc < I.ncell && (d.flags[I.cell0 + lc] & F_BAND) != 0;
    cnt += in[q] ? 1 : 0;
  }
  int off = d.bcnt[I.cblk0 + blockIdx.x] + block_prefix(cnt, sh);
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (in[q]) {
      if (off < I.band_cap) I.band[off] = (int32_t)(b0 + 4 * threadIdx.x + q);
      ++off;
    }
}

// k_membrane: membrane forces (Eqs. tension and bending along theta and z,
// and with the shell model the off-diagonal terms of Eq. structure)
// and the wall's central-difference step, one lane per point, after k_wall
// has produced this step's penalty force.  A workgroup takes a tile of
// MJ x MK points (theta x z) and stages X0 and D of the tile and its 2-point
// halo (periodic in theta) in LDS once, instead of each lane reading its ~30
// neighbour values from L2.
constexpr int MJ = MEM_TJ, MK = MEM_TK, MH = 2;
constexpr int MLJ = MJ + 2 * MH, MLK = MK + 2 * MH;
// SHELL: the build with the shell model's terms, taken when some wall asks
// for them (they cost the plain membrane registers even when skipped).
template <bool SHELL>
__global__ __launch_bounds__(WBLOCK) void k_membrane(Dev d, int parity) {
  const int inst = d.walls[blockIdx.y];
  if (d.err[inst] & ERR_FROZEN) return;
  const InstDesc& I = d.inst[inst];
  const int nth = I.nth, nzl = I.nzl;
  const int ntj = (nth + MJ - 1) / MJ;
  // this wall's tiles in XCD-aware order over its own tile count
  const int ntile = ntj * ((nzl + MK - 1) / MK);
  if ((int)blockIdx.x >= ntile) return;  // whole block leaves
  const int bx = xcd_tile(blockIdx.x, ntile);
  const int j0 = (bx % ntj) * MJ, k0 = (bx / ntj) * MK;
  __shared__ double3 sx0[MLK][MLJ], sd[MLK][MLJ];
  const double* Dc = I.Xab[parity];
  double* Dn = I.Xab[parity ^ 1];
  for (int q = (int)threadIdx.x; q < MLJ * MLK; q += WBLOCK) {
    const int hj = q % MLJ, hk = q / MLJ;
    const int kk = k0 - MH + hk;
    if (kk < 0 || kk >= nzl) continue;   // rows past the ends are never read
    const int jj = ((j0 - MH + hj) % nth + nth) % nth;
    const int64_t pp = jj + (int64_t)nth * kk;
    sx0[hk][hj] = ld3(I.X0, pp);
    sd[hk][hj] = ld3(Dc, pp);
  }
  __syncthreads();
  const int tj = (int)threadIdx.x % MJ, tk = (int)threadIdx.x / MJ;
  const int j = j0 + tj, k = k0 + tk;
  if (j >= nth || k >= nzl) return;
  const int64_t p = j + (int64_t)nth * k;
  // staged values at theta offset dj, z offset dk from this point
  auto DD = [&](int dj, int dk) -> double3 { return sd[tk + MH + dk][tj + MH + dj]; };
  auto XX = [&](int dj, int dk) -> double3 { return sx0[tk + MH + dk][tj + MH + dj]; };
  const double3 D = DD(0, 0), Dm = ld3(Dn, p);
  const double4 Fw = ((const double4*)I.Fp)[p];
  const double Fx = Fw.x, Fy = Fw.y, Fz = Fw.z;
  // edge vector X_b - X_a = (X0_b - X0_a) + (D_b - D_a), a and b as offsets
  auto edge = [&](int ja, int ka, int jb, int kb) -> double3 {
    const double3 xa = XX(ja, ka), xb = XX(jb, kb), da = DD(ja, ka), db = DD(jb, kb);
    return make_double3((xb.x - xa.x) + (db.x - da.x), (xb.y - xa.y) + (db.y - da.y),
                        (xb.z - xa.z) + (db.z - da.z));
  };
  const double dt2 = I.ds_th * I.ds_th, dz2 = I.ds_z * I.ds_z;
  double3 f = make_double3(0.0, 0.0, 0.0);
  {
    const double3 tp = tension(edge(0, 0, 1, 0), I.ds_th, I.ks);
    const double3 tm = tension(edge(-1, 0, 0, 0), I.ds_th, I.ks);
    f.x += (tp.x - tm.x) / I.ds_th; f.y += (tp.y - tm.y) / I.ds_th; f.z += (tp.z - tm.z) / I.ds_th;
    const double3 y2m = DD(-2, 0), y1m = DD(-1, 0), y0 = D, y1p = DD(1, 0), y2p = DD(2, 0);
    // curvature at j-1, j, j+1, then its second difference
    const double kmx = (y0.x - 2.0 * y1m.x + y2m.x) / dt2, kcx = (y1p.x - 2.0 * y0.x + y1m.x) / dt2,
                 kpx = (y2p.x - 2.0 * y1p.x + y0.x) / dt2;
    const double kmy = (y0.y - 2.0 * y1m.y + y2m.y) / dt2, kcy = (y1p.y - 2.0 * y0.y + y1m.y) / dt2,
                 kpy = (y2p.y - 2.0 * y1p.y + y0.y) / dt2;
    const double kmz = (y0.z - 2.0 * y1m.z + y2m.z) / dt2, kcz = (y1p.z - 2.0 * y0.z + y1m.z) / dt2,
                 kpz = (y2p.z - 2.0 * y1p.z + y0.z) / dt2;
    f.x -= I.ei * (kpx - 2.0 * kcx + kmx) / dt2;
    f.y -= I.ei * (kpy - 2.0 * kcy + kmy) / dt2;
    f.z -= I.ei * (kpz - 2.0 * kcz + kmz) / dt2;
  }
  const bool interior = k > 0 && k < nzl - 1;
  if (interior) {
    const double3 tp = tension(edge(0, 0, 0, 1), I.ds_z, I.ks);
    const double3 tm = tension(edge(0, -1, 0, 0), I.ds_z, I.ks);
    f.x += (tp.x - tm.x) / I.ds_z; f.y += (tp.y - tm.y) / I.ds_z; f.z += (tp.z - tm.z) / I.ds_z;
    // curvature along z, zero on the end rings (simply supported)
    auto kap = [&](int kk) -> double3 {
      if (kk <= 0 || kk >= nzl - 1) return make_double3(0.0, 0.0, 0.0);
      const double3 a = DD(0, kk - 1 - k), b = DD(0, kk - k), c = DD(0, kk + 1 - k);
      return make_double3((c.x - 2.0 * b.x + a.x) / dz2, (c.y - 2.0 * b.y + a.y) / dz2,
                          (c.z - 2.0 * b.z + a.z) / dz2);
    };
    const double3 km = kap(k - 1), kc = kap(k), kp = kap(k + 1);
    f.x -= I.ei * (kp.x - 2.0 * kc.x + km.x) / dz2;
    f.y -= I.ei * (kp.y - 2.0 * kc.y + km.y) / dz2;
    f.z -= I.ei * (kp.z - 2.0 * kc.z + km.z) / dz2;
    if (SHELL && I.shell) {
      // The off-diagonal terms of Eq. structure.  In-plane shear: on each of
      // the four mesh cells around the point, the tangents X_theta and X_z
      // at the cell centre (means of the cell's two edges along each
      // direction), the strain S = X_theta . X_z and the fluxes
      // A = Eh phi12 S X_z (differentiated along theta) and
      // B = Eh phi12 S X_theta (along z); their divergence at the point
      // differences the centre pairs on either side.
      const double c = I.ks * I.phi12;
      auto flux = [&](int dj, int dk, double3& A, double3& B) {
        const double3 e0 = edge(dj, dk, dj + 1, dk), e1 = edge(dj, dk + 1, dj + 1, dk + 1);
        const double3 e2 = edge(dj, dk, dj, dk + 1), e3 = edge(dj + 1, dk, dj + 1, dk + 1);
        const double3 xt = make_double3((e0.x + e1.x) / (2.0 * I.ds_th), (e0.y + e1.y) / (2.0 * I.ds_th),
                                        (e0.z + e1.z) / (2.0 * I.ds_th));
        const double3 xz = make_double3((e2.x + e3.x) / (2.0 * I.ds_z), (e2.y + e3.y) / (2.0 * I.ds_z),
                                        (e2.z + e3.z) / (2.0 * I.ds_z));
        const double cs = c * (xt.x * xz.x + xt.y * xz.y + xt.z * xz.z);
        A = make_double3(cs * xz.x, cs * xz.y, cs * xz.z);
        B = make_double3(cs * xt.x, cs * xt.y, cs * xt.z);
      };
      double3 Ane, Bne, Ase, Bse, Anw, Bnw, Asw, Bsw;
      flux(0, 0, Ane, Bne);
      flux(0, -1, Ase, Bse);
      flux(-1, 0, Anw, Bnw);
      flux(-1, -1, Asw, Bsw);
      const double ht = 2.0 * I.ds_th, hz = 2.0 * I.ds_z;
      f.x += ((Ane.x + Ase.x) - (Anw.x + Asw.x)) / ht + ((Bne.x + Bnw.x) - (Bse.x + Bsw.x)) / hz;
      f.y += ((Ane.y + Ase.y) - (Anw.y + Asw.y)) / ht + ((Bne.y + Bnw.y) - (Bse.y + Bsw.y)) / hz;
      f.z += ((Ane.z + Ase.z) - (Anw.z + Asw.z)) / ht + ((Bne.z + Bnw.z) - (Bse.z + Bsw.z)) / hz;
      // mixed bending (gamma_12 = gamma_21 = 1): -2 EI times the second z
      // difference of the theta curvature, zero on the end rings
      auto kth = [&](int dk) -> double3 {
        if (k + dk <= 0 || k + dk >= nzl - 1) return make_double3(0.0, 0.0, 0.0);
        const double3 a = DD(-1, dk), b = DD(0, dk), e = DD(1, dk);
        return make_double3((e.x - 2.0 * b.x + a.x) / dt2, (e.y - 2.0 * b.y + a.y) / dt2,
                            (e.z - 2.0 * b.z + a.z) / dt2);
      };
      const double3 qm = kth(-1), qc = kth(0), qp = kth(1);
      f.x -= 2.0 * I.ei * (qp.x - 2.0 * qc.x + qm.x) / dz2;
      f.y -= 2.0 * I.ei * (qp.y - 2.0 * qc.y + qm.y) / dz2;
      f.z -= 2.0 * I.ei * (qp.z - 2.0 * qc.z + qm.z) / dz2;
    }
  }

  // central difference in time; the wall receives -F.  An external solid
  // (moved by the caller) keeps its velocity between the caller's updates.
  double4 out;
  if (I.ext) {
    out.x = 2.0 * D.x - Dm.x;
    out.y = 2.0 * D.y - Dm.y;
    out.z = 2.0 * D.z - Dm.z;
  } else if (interior) {
    out.x = 2.0 * D.x - Dm.x + (f.x - Fx) / I.mass;
    out.y = 2.0 * D.y - Dm.y + (f.y - Fy) / I.mass;
    out.z = 2.0 * D.z - Dm.z + (f.z - Fz) / I.mass;
  } else {
    out.x = D.x; out.y = D.y; out.z = D.z;
  }
  out.w = 0.0;
  ((double4*)Dn)[p] = out;
}

// ---------------------------------------------------------------------------
// rest state fill: stored g = w_i dshift (dshift = 3 p - dref)
// ---------------------------------------------------------------------------
template <class S>
__global__ void k_fill_rest(Dev d, int64_t cell0, int64_t ncell, double dshift) {
  using R = typename Store<S>::R;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ncell) return;
  const int64_t c = cell0 + k;
  const bool fl = (d.flags[c] & TYPE_MASK) == T_FLUID;
  S* A = (S*)d.pop;
#pragma unroll
  for (int i = 0; i < NQ; ++i) Store<S>::st(A + i * d.NT + c, fl ? (R)(wgt<double>(i) * dshift) : R(0), d.scale);
}

// ---------------------------------------------------------------------------
// launchers: hipLaunchKernel returns the launch status itself, so a stale
// error left in the thread by an unrelated runtime call is never reported.
// ---------------------------------------------------------------------------
namespace {
template <class... P>
hipError_t launch(void (*k)(P...), dim3 g, dim3 b, hipStream_t s, P... a) {
  void* args[] = {(void*)&a...};
  return hipLaunchKernel((const void*)k, g, b, args, 0, s);
}
}  // namespace

#define LBM_DISPATCH(prec, F)                     \
  switch (prec) {                                 \
    case 0: F(double); break;                     \
    case 1: F(float); break;                      \
    case 2: F(__half); break;                     \
    case 3: F(__hip_bfloat16); break;             \
    default: return hipErrorInvalidValue;         \
  }

hipError_t launch_reduce(const Dev& d, int prec, int parity, int nred, hipStream_t s) {
  if (nred <= 0) return hipSuccess;
#define F(T)                                                                              \
  return parity ? launch(k_reduce<T, true>, dim3(nred), dim3(RBLOCK), s, Dev(d))          \
                : launch(k_reduce<T, false>, dim3(nred), dim3(RBLOCK), s, Dev(d));
  LBM_DISPATCH(prec, F)
#undef F
  return hipErrorInvalidValue;
}

namespace {
template <class T, int BS, int CPT>
hipError_t collide_bs(const Dev& d, int parity, bool nee, const CTile* tab, int ntile, int mode, hipStream_t s) {
  const dim3 g(ntile), b(BS);
  if (nee)
    return parity ? launch(k_collide<T, true, BS, CPT, true>, g, b, s, Dev(d), tab, int(mode))
                  : launch(k_collide<T, false, BS, CPT, true>, g, b, s, Dev(d), tab, int(mode));
  return parity ? launch(k_collide<T, true, BS, CPT, false>, g, b, s, Dev(d), tab, int(mode))
                : launch(k_collide<T, false, BS, CPT, false>, g, b, s, Dev(d), tab, int(mode));
}
template <class T>
hipError_t collide_t(const Dev& d, int parity, int bs, int cpt, bool nee, const CTile* tab, int ntile, int mode,
                     hipStream_t s) {
  switch (bs * 4 + cpt) {
    case 128 * 4 + 1: return collide_bs<T, 128, 1>(d, parity, nee, tab, ntile, mode, s);
    case 128 * 4 + 2: return collide_bs<T, 128, 2>(d, parity, nee, tab, ntile, mode, s);
    case 256 * 4 + 1: return collide_bs<T, 256, 1>(d, parity, nee, tab, ntile, mode, s);
    case 256 * 4 + 2: return collide_bs<T, 256, 2>(d, parity, nee, tab, ntile, mode, s);
    case 512 * 4 + 1: return collide_bs<T, 512, 1>(d, parity, nee, tab, ntile, mode, s);
    case 512 * 4 + 2: return collide_bs<T, 512, 2>(d, parity, nee, tab, ntile, mode, s);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace

hipError_t launch_collide(const Dev& d, int prec, int parity, int bs, int cpt, bool nee, const CTile* tab,
                          int ntile, int mode, hipStream_t s) {
  if (ntile <= 0) return hipSuccess;
#define F(T) return collide_t<T>(d, parity, bs, cpt, nee, tab, ntile, mode, s);
  LBM_DISPATCH(prec, F)
#undef F
  return hipErrorInvalidValue;
}

hipError_t launch_collide_count(const Dev& d, int parity, bool nee, const CTile* tab, int ntile, hipStream_t s) {
  if (ntile <= 0) return hipSuccess;
  const dim3 g((unsigned)ntile), b(256);
  if (nee)
    return parity ? launch(k_collide_count<true, true>, g, b, s, Dev(d), tab)
                  : launch(k_collide_count<false, true>, g, b, s, Dev(d), tab);
  return parity ? launch(k_collide_count<true, false>, g, b, s, Dev(d), tab)
                : launch(k_collide_count<false, false>, g, b, s, Dev(d), tab);
}

hipError_t launch_reduce_band(const Dev& d, int prec, int parity, int nred, hipStream_t s) {
  const int nbx = d.nwall > 0 ? (d.max_band + WBLOCK - 1) / WBLOCK : 0;
  const int64_t nb = (int64_t)nred + (int64_t)nbx * d.nwall;
  if (nb <= 0) return hipSuccess;
  if (nb > 0x7fffffff) return hipErrorInvalidValue;
#define F(T)                                                                                          \
  return parity ? launch(k_reduce_band<T, true>, dim3((unsigned)nb), dim3(WBLOCK), s, Dev(d), nred, nbx) \
                : launch(k_reduce_band<T, false>, dim3((unsigned)nb), dim3(WBLOCK), s, Dev(d), nred, nbx);
  LBM_DISPATCH(prec, F)
#undef F
  return hipErrorInvalidValue;
}

hipError_t launch_band(const Dev& d, int prec, int parity, hipStream_t s) {
  if (d.nwall <= 0 || d.max_band <= 0) return hipSuccess;
  const dim3 grid((d.max_band + WBLOCK - 1) / WBLOCK, d.nwall);
#define F(T)                                                                              \
  return parity ? launch(k_band<T, true>, grid, dim3(WBLOCK), s, Dev(d))                  \
                : launch(k_band<T, false>, grid, dim3(WBLOCK), s, Dev(d));
  LBM_DISPATCH(prec, F)
#undef F
  return hipErrorInvalidValue;
}

namespace {
template <class R>
hipError_t wall_t(const Dev& d, int parity, int tj, int tk, bool big, const int32_t* walls, dim3 grid, int colour,
                  hipStream_t s) {
  const dim3 b(WBLOCK);
#define W(J, K)                                                                                      \
  if (tj == J && tk == K)                                                                           \
    return big ? launch(k_wall<R, J, K, true>, grid, b, s, Dev(d), walls, int(parity), int(colour)) \
               : launch(k_wall<R, J, K, false>, grid, b, s, Dev(d), walls, int(parity), int(colour));
  W(8, 32) W(16, 16) W(32, 8) W(8, 16) W(16, 8) W(8, 8)
#undef W
  return hipErrorInvalidValue;
}
}  // namespace

hipError_t launch_wall(const Dev& d, int prec, int parity, int tj, int tk, bool big, const int32_t* walls, int nwall,
                       int tiles, int colour, hipStream_t s) {
  if (nwall <= 0 || tiles <= 0) return hipSuccess;
  const dim3 grid((unsigned)tiles, (unsigned)nwall);
  return prec == 0 ? wall_t<double>(d, parity, tj, tk, big, walls, grid, colour, s)
                   : wall_t<float>(d, parity, tj, tk, big, walls, grid, colour, s);
}

hipError_t launch_motion(const Dev& d, int parity, hipStream_t s) {
  if (d.nwall <= 0 || d.max_np <= 0) return hipSuccess;
  const dim3 g((unsigned)std::min<int64_t>(MOTION_BLOCKS, (d.max_np + WBLOCK - 1) / WBLOCK), d.nwall);
  return launch(k_motion, g, dim3(WBLOCK), s, Dev(d), int(parity));
}
hipError_t launch_wss(const Dev& d, int prec, int parity, int inst, int64_t np, double dist, double mu, double* out,
                      hipStream_t s) {
  if (np <= 0) return hipSuccess;
  const dim3 g((unsigned)((np + WBLOCK - 1) / WBLOCK));
#define F(T)                                                                                            \
  return parity ? launch(k_wss<T, true>, g, dim3(WBLOCK), s, Dev(d), int(inst), dist, mu, out)          \
                : launch(k_wss<T, false>, g, dim3(WBLOCK), s, Dev(d), int(inst), dist, mu, out);
  LBM_DISPATCH(prec, F)
#undef F
  return hipErrorInvalidValue;
}
hipError_t launch_band_rebuild(const Dev& d, int parity, float thresh, const int maxlines[3], int maxblk,
                               hipStream_t s) {
  if (d.nwall <= 0) return hipSuccess;
  hipError_t e;
  if ((e = launch(k_band_gate, dim3(1), dim3(64), s, Dev(d), thresh)) != hipSuccess) return e;
  const dim3 gp((unsigned)((d.max_np + WBLOCK - 1) / WBLOCK), d.nwall);
  if ((e = launch(k_band_seed, gp, dim3(WBLOCK), s, Dev(d), int(parity))) != hipSuccess) return e;
  const uint8_t* src[3] = {d.bmark, d.btmp, d.bmark};
  uint8_t* dst[3] = {d.btmp, d.bmark, d.btmp};   // x: marks -> tmp, y: tmp -> marks, z: marks -> tmp
  for (int a = 0; a < 3; ++a) {
    const dim3 gl((unsigned)((maxlines[a] + WBLOCK - 1) / WBLOCK), d.nwall);
    if ((e = launch(k_band_dilate, gl, dim3(WBLOCK), s, Dev(d), int(a), src[a], dst[a])) != hipSuccess) return e;
  }
  const dim3 gb((unsigned)maxblk, d.nwall);
  if ((e = launch(k_band_flags, gb, dim3(WBLOCK), s, Dev(d))) != hipSuccess) return e;
  if ((e = launch(k_band_scan, dim3(d.nwall), dim3(WBLOCK), s, Dev(d))) != hipSuccess) return e;
  return launch(k_band_write, gb, dim3(WBLOCK), s, Dev(d));
}

hipError_t launch_membrane(const Dev& d, int parity, hipStream_t s) {
  if (d.nwall <= 0 || d.max_np <= 0 || d.max_mtile <= 0) return hipSuccess;
  const dim3 g2((unsigned)d.max_mtile, d.nwall);
  return d.any_shell ? launch(k_membrane<true>, g2, dim3(WBLOCK), s, Dev(d), int(parity))
                     : launch(k_membrane<false>, g2, dim3(WBLOCK), s, Dev(d), int(parity));
}

hipError_t launch_fill_rest(const Dev& d, int prec, int64_t cell0, int64_t ncell, double dshift, hipStream_t s) {
  if (ncell <= 0) return hipSuccess;
  const unsigned nb = (unsigned)((ncell + 255) / 256);
#define F(T) return launch(k_fill_rest<T>, dim3(nb), dim3(256), s, Dev(d), int64_t(cell0), int64_t(ncell), double(dshift));
  LBM_DISPATCH(prec, F)
#undef F
  return hipErrorInvalidValue;
}

}  // namespace lbm
