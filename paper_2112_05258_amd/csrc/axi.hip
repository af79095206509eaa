// Axisymmetric D2Q9 lattice Boltzmann solver (Eqs. Afi, AH1) with the 0D
// couplings of the 3D solver, for gfx950.  Model and interface:
// include/lbm_axi.h.
//
// Data: populations g[9][n] (SoA, node c = i + nx j), stored shifted by
// w_i 3 p_ref (an exact change of variables that keeps FP32 values small
// near the reference pressure, as in the 3D solver), in two buffers
// (pull streaming, ping-pong); the moments D, j_x, j_r in two buffers as
// well (the collide kernel writes the moments of the state it produces,
// while other lanes still read the previous ones); the force F; the inlet
// snapshot; the two 0D records; the waveform ring.  One step is three
// launches: the column sums and 0D update (one workgroup), the force (one
// lane per node), collide-and-stream (one lane per node).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "lbm_axi.h"
#include "lbm_internal.h"
#include "zerod.h"

namespace {

using lbm::BcDev;

constexpr int AQ = 9;
constexpr int AREC = 14;
constexpr int ABLOCK = 256;
enum : uint8_t { A_FLUID = 0, A_SOLID = 1, A_INLET = 2, A_OUTLET = 3 };

__constant__ int AEX[AQ] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__constant__ int AER[AQ] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__constant__ int AOPP[AQ] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
__constant__ int AMIR[AQ] = {0, 1, 4, 3, 2, 8, 7, 6, 5};

struct AxiDev {
  int32_t nx, nr, px, cap;
  int64_t n;
  double tau, nu;
  double dref;       // 3 p_ref: the stored populations are g - w dref
  const uint8_t* type;
  void* g[2];
  void* D[2];
  void* jx[2];
  void* jr[2];
  void* Fx;
  void* Fr;
  void* v0;          // 2 per row
  BcDev* bc;         // inlet, outlet
  double* wave;      // [cap][AREC]
  uint32_t* err;
  double G0, om;
  double* fields;    // 3 n doubles for read-back
};

template <class T>
__device__ __forceinline__ T wgt(int k) {
  return k == 0 ? T(4) / T(9) : (k < 5 ? T(1) / T(9) : T(1) / T(36));
}

template <class T>
__device__ __forceinline__ T aeq(int k, T D, T ux, T ur) {
  const T eu = T(AEX[k]) * ux + T(AER[k]) * ur;
  return wgt<T>(k) * (D + T(3) * eu + T(4.5) * eu * eu - T(1.5) * (ux * ux + ur * ur));
}

template <class T>
__device__ __forceinline__ T aforce(int k, T tau, T ux, T ur, T fx, T fr) {
  const T ex = T(AEX[k]), er = T(AER[k]);
  const T eu = ex * ux + er * ur;
  return (T(1) - T(1) / (T(2) * tau)) * wgt<T>(k) *
         (T(3) * ((ex - ux) * fx + (er - ur) * fr) + T(9) * eu * (ex * fx + er * fr));
}

__device__ __forceinline__ int atype(const AxiDev& d, int i, int j) {
  if (j >= d.nr) return A_SOLID;
  if (d.px) i = (i + d.nx) % d.nx;
  if (i < 0 || i >= d.nx) return A_SOLID;
  return d.type[i + (int64_t)d.nx * j];
}
__device__ __forceinline__ bool afluid(const AxiDev& d, int i, int j) {
  if (d.px) i = (i + d.nx) % d.nx;
  return i >= 0 && i < d.nx && d.type[i + (int64_t)d.nx * j] == A_FLUID;
}
__device__ __forceinline__ int64_t anode(const AxiDev& d, int i, int j) {
  if (d.px) i = (i + d.nx) % d.nx;
  return i + (int64_t)d.nx * j;
}

// d/dr of a velocity component (odd: changes sign across the axis)
template <class T>
__device__ T ddr(const AxiDev& d, const T* u, bool odd, int i, int j) {
  const T uc = u[anode(d, i, j)];
  const bool up = atype(d, i, j + 1) == A_FLUID;
  const bool dn = j == 0 ? true : atype(d, i, j - 1) == A_FLUID;
  const T uu = up ? u[anode(d, i, j + 1)] : T(0);
  T ud = T(0);
  if (j == 0) ud = odd ? -uc : uc;
  else if (dn) ud = u[anode(d, i, j - 1)];
  if (up && dn) return (uu - ud) / T(2);
  if (dn) return -ud / T(3) - uc;   // wall half way above: quadratic through its zero
  if (up) return uu / T(3) + uc;    // wall half way below
  return T(0);
}

template <class T>
__device__ T ddx(const AxiDev& d, const T* u, int i, int j) {
  const bool l = afluid(d, i - 1, j), r = afluid(d, i + 1, j);
  if (l && r) return (u[anode(d, i + 1, j)] - u[anode(d, i - 1, j)]) / T(2);
  if (r && afluid(d, i + 2, j))
    return (T(-3) * u[anode(d, i, j)] + T(4) * u[anode(d, i + 1, j)] - u[anode(d, i + 2, j)]) / T(2);
  if (l && afluid(d, i - 2, j))
    return (T(3) * u[anode(d, i, j)] - T(4) * u[anode(d, i - 1, j)] + u[anode(d, i - 2, j)]) / T(2);
  return T(0);
}

template <class T>
__device__ void axforce(const AxiDev& d, const T* jx, const T* jr, int i, int j, T G, T& fx, T& fr) {
  const int64_t c = i + (int64_t)d.nx * j;
  const T r = T(j) + T(0.5), ux = jx[c], ur = jr[c], nu = T(d.nu);
  const T dux_dr = ddr<T>(d, jx, false, i, j), dur_dr = ddr<T>(d, jr, true, i, j), dur_dx = ddx<T>(d, jr, i, j);
  fx = -ux * ur / r + nu / r * (dux_dr + dur_dx) + G;
  fr = -ur * ur / r + T(2) * nu / r * dur_dr - T(2) * nu * ur / (r * r);
}

// moments of buffer b (set-up and after population writes)
template <class T>
__global__ void k_axi_moments(AxiDev d, int b) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= d.n) return;
  const T* g = (const T*)d.g[b];
  T D = T(0), jx = T(0), jr = T(0);
  if (d.type[c] == A_FLUID)
    for (int k = 0; k < AQ; ++k) {
      const T gk = g[k * d.n + c];
      D += gk;
      jx += T(AEX[k]) * gk;
      jr += T(AER[k]) * gk;
    }
  ((T*)d.D[b])[c] = D;
  ((T*)d.jx[b])[c] = jx;
  ((T*)d.jr[b])[c] = jr;
}

// column sums (FP64) and the 0D updates; one workgroup
__device__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = ABLOCK / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

template <class T>
__global__ __launch_bounds__(ABLOCK) void k_axi_bc(AxiDev d, int b, int64_t n) {
  __shared__ double sh[ABLOCK];
  __shared__ int snap;
  const T* D = (const T*)d.D[b];
  const T* jx = (const T*)d.jx[b];
  const T* jr = (const T*)d.jr[b];
  const double twopi = 6.283185307179586476925286766559;
  double Q[3] = {0, 0, 0}, P[3] = {0, 0, 0};
  const int cols[3] = {1, d.nx - 2, d.nx / 2};
  for (int s = d.px ? 2 : 0; s < 3; ++s) {
    double q = 0, pa = 0, a = 0;
    for (int j = threadIdx.x; j < d.nr; j += ABLOCK) {
      const int64_t c = cols[s] + (int64_t)d.nx * j;
      if (d.type[c] != A_FLUID) continue;
      const double dA = twopi * ((double)j + 0.5);
      const double Dt = (double)D[c] + d.dref;
      q += dA * (double)jx[c] / (1.0 + Dt);
      pa += dA * (Dt / 3.0 - (double)jr[c] / (6.0 * ((double)j + 0.5)));
      a += dA;
    }
    q = block_sum(q, sh);
    pa = block_sum(pa, sh);
    a = block_sum(a, sh);
    Q[s] = q;
    P[s] = a > 0 ? pa / a : 0.0;
  }
  if (threadIdx.x == 0) {
    snap = 0;
    if (!d.px) {
      lbm::zerod_update(d.bc[0], n, Q[0], P[0]);
      lbm::zerod_update(d.bc[1], n, Q[1], P[1]);
      snap = d.bc[0].snap;
    }
    bool bad = false;
    for (int s = 0; s < 3; ++s) bad = bad || !isfinite(Q[s]) || !isfinite(P[s]);
    if (bad) atomicOr(d.err, 1u);
    const BcDev &b0 = d.bc[0], &b1 = d.bc[1];
    double* r = d.wave + (n % d.cap) * AREC;
    r[0] = (double)n;
    r[1] = Q[0]; r[2] = P[0]; r[3] = Q[1]; r[4] = P[1];
    r[5] = d.px ? 0.0 : b0.vmode;
    r[6] = d.px ? 0.0 : (b0.vmode == 0 ? b0.pstar : (b0.kind == lbm::BC_LV ? b0.S : b0.vz));
    r[7] = d.px ? 0.0 : b1.vmode;
    r[8] = d.px ? 0.0 : (b1.vmode == 0 ? b1.pstar : b1.vz);
    r[9] = b0.kind == lbm::BC_LV ? b0.Pv : 0.0;
    r[10] = b1.kind == lbm::BC_WK3 ? b1.Pw : 0.0;
    r[11] = b0.kind == lbm::BC_LV ? (double)b0.open : 0.0;
    r[12] = Q[2]; r[13] = P[2];
  }
  __syncthreads();
  if (snap)   // valve closure: the inlet column's unforced velocity
    for (int j = threadIdx.x; j < d.nr; j += ABLOCK) {
      const int64_t c = 1 + (int64_t)d.nx * j;
      ((T*)d.v0)[2 * j] = jx[c];
      ((T*)d.v0)[2 * j + 1] = jr[c];
    }
}

template <class T>
__global__ void k_axi_force(AxiDev d, int b, int64_t n) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= d.n) return;
  T fx = T(0), fr = T(0);
  if (d.type[c] == A_FLUID) {
    const T G = T(d.G0 * cos(d.om * (double)n));
    axforce<T>(d, (const T*)d.jx[b], (const T*)d.jr[b], (int)(c % d.nx), (int)(c / d.nx), G, fx, fr);
  }
  ((T*)d.Fx)[c] = fx;
  ((T*)d.Fr)[c] = fr;
}

// post-collision value of direction k at fluid node c of buffer b
template <class T>
__device__ __forceinline__ T post(const AxiDev& d, int b, int64_t c, int k) {
  const T fx = ((const T*)d.Fx)[c], fr = ((const T*)d.Fr)[c];
  const T ux = ((const T*)d.jx[b])[c] + fx / T(2), ur = ((const T*)d.jr[b])[c] + fr / T(2);
  const T gk = ((const T*)d.g[b])[k * d.n + c];
  const T tau = T(d.tau);
  return gk - (gk - aeq<T>(k, ((const T*)d.D[b])[c], ux, ur)) / tau + aforce<T>(k, tau, ux, ur, fx, fr) -
         wgt<T>(k) * ur / (T(c / d.nx) + T(0.5));
}

template <class T>
__global__ void k_axi_collide(AxiDev d, int b) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= d.n) return;
  const int nb = b ^ 1;
  T* gn = (T*)d.g[nb];
  if (d.type[c] != A_FLUID) {
    ((T*)d.D[nb])[c] = T(0);
    ((T*)d.jx[nb])[c] = T(0);
    ((T*)d.jr[nb])[c] = T(0);
    return;
  }
  const int i = (int)(c % d.nx), j = (int)(c / d.nx);
  const T tau = T(d.tau);
  T D = T(0), jx = T(0), jr = T(0);
  for (int k = 0; k < AQ; ++k) {
    int si = i - AEX[k], sj = j - AER[k], kk = k;
    if (sj < 0) { sj = 0; kk = AMIR[k]; }   // across the axis: mirror image
    const int st = atype(d, si, sj);
    T v;
    if (st == A_FLUID) {
      v = post<T>(d, b, anode(d, si, sj), kk);
    } else if (st == A_SOLID) {
      v = post<T>(d, b, c, AOPP[k]);
    } else {
      // ghost: extrapolation from its neighbour along x
      const int w = st == A_INLET ? 0 : 1;
      const int fi = w == 0 ? si + 1 : si - 1;
      const int64_t xf = atype(d, fi, sj) == A_FLUID ? anode(d, fi, sj) : c;
      const T fx = ((const T*)d.Fx)[xf], fr = ((const T*)d.Fr)[xf];
      const T ux = ((const T*)d.jx[b])[xf] + fx / T(2), ur = ((const T*)d.jr[b])[xf] + fr / T(2);
      const T Df = ((const T*)d.D[b])[xf];
      const BcDev& B = d.bc[w];
      T Dst, vx, vr;
      if (B.vmode == 0) {
        Dst = T(3.0 * B.pstar - d.dref);
        vx = ux;
        vr = ur;
      } else {
        Dst = Df;
        if (B.kind == lbm::BC_LV) {
          const T S = T(B.S);
          vx = ((const T*)d.v0)[2 * sj] * S;
          vr = ((const T*)d.v0)[2 * sj + 1] * S;
        } else if (B.kind == lbm::BC_WK3) {
          vx = ux + T(B.vz);
          vr = ur;
        } else {
          vx = T(B.vz);
          vr = T(0);
        }
      }
      const T gk = ((const T*)d.g[b])[kk * d.n + xf];
      v = aeq<T>(kk, Dst, vx, vr) + (T(1) - T(1) / tau) * (gk - aeq<T>(kk, Df, ux, ur)) +
          aforce<T>(kk, tau, ux, ur, fx, fr) - wgt<T>(kk) * ur / (T(xf / d.nx) + T(0.5));
    }
    gn[k * d.n + c] = v;
    D += v;
    jx += T(AEX[k]) * v;
    jr += T(AER[k]) * v;
  }
  ((T*)d.D[nb])[c] = D;
  ((T*)d.jx[nb])[c] = jx;
  ((T*)d.jr[nb])[c] = jr;
}

// gauge pressure and forced velocity of buffer b into d.fields
template <class T>
__global__ void k_axi_fields(AxiDev d, int b) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= d.n) return;
  const bool fl = d.type[c] == A_FLUID;
  d.fields[c] = fl ? ((double)((const T*)d.D[b])[c] + d.dref) / 3.0 -
                         (double)((const T*)d.jr[b])[c] / (6.0 * ((double)(c / d.nx) + 0.5))
                   : 0.0;
  d.fields[d.n + c] = fl ? (double)(((const T*)d.jx[b])[c] + ((const T*)d.Fx)[c] / T(2)) : 0.0;
  d.fields[2 * d.n + c] = fl ? (double)(((const T*)d.jr[b])[c] + ((const T*)d.Fr)[c] / T(2)) : 0.0;
}

template <class T>
__global__ void k_axi_fill(AxiDev d, int b, double D0) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= d.n) return;
  const bool fl = d.type[c] == A_FLUID;
  for (int k = 0; k < AQ; ++k) ((T*)d.g[b])[k * d.n + c] = fl ? wgt<T>(k) * T(D0) : T(0);
}

template <class T>
__global__ void k_axi_put(AxiDev d, int b, const double* src, int to_device) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= d.n) return;
  T* g = (T*)d.g[b];
  for (int k = 0; k < AQ; ++k) {
    const double shift = d.type[c] == A_FLUID ? wgt<double>(k) * d.dref : 0.0;
    if (to_device) g[k * d.n + c] = (T)(src[c * AQ + k] - shift);
    else ((double*)src)[c * AQ + k] = (double)g[k * d.n + c] + shift;
  }
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  size_t type, g[2], D[2], jx[2], jr[2], Fx, Fr, v0, bc, wave, err, fields, xfer, total;
};

Layout plan(const lbm_axi_config& c) {
  Layout L{};
  const size_t n = (size_t)c.nx * c.nr, es = c.precision == LBM_FP64 ? 8 : 4;
  const size_t cap = c.wave_cap > 0 ? (size_t)c.wave_cap : 4096;
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t at = o; o = align256(o + bytes); return at; };
  L.type = take(n);
  for (int b = 0; b < 2; ++b) L.g[b] = take(AQ * n * es);
  for (int b = 0; b < 2; ++b) { L.D[b] = take(n * es); L.jx[b] = take(n * es); L.jr[b] = take(n * es); }
  L.Fx = take(n * es);
  L.Fr = take(n * es);
  L.v0 = take(2 * (size_t)c.nr * es);
  L.bc = take(2 * sizeof(BcDev));
  L.wave = take(cap * AREC * 8);
  L.err = take(4);
  L.fields = take(3 * n * 8);
  L.xfer = take(n * AQ * 8);
  L.total = o;
  return L;
}

std::string g_err;

bool valid(const lbm_axi_config* c, std::string& err) {
  if (!c || !c->flags) { err = "config or flags NULL"; return false; }
  if (c->nx < 5 || c->nr < 2) { err = "need nx >= 5 and nr >= 2"; return false; }
  if ((int64_t)c->nx * c->nr >= ((int64_t)1 << 31)) { err = "grid too large"; return false; }
  if (!(c->tau > 0.5)) { err = "tau must be > 0.5"; return false; }
  if (c->precision != LBM_FP64 && c->precision != LBM_FP32) { err = "precision must be FP64 or FP32"; return false; }
  if (c->periodic_x != 0 && c->periodic_x != 1) { err = "periodic_x must be 0 or 1"; return false; }
  if (!std::isfinite(c->p_ref)) { err = "p_ref must be finite"; return false; }
  for (int j = 0; j < c->nr; ++j)
    for (int i = 0; i < c->nx; ++i) {
      const uint8_t t = c->flags[i + (size_t)c->nx * j];
      if (t > A_OUTLET) { err = "node type out of range"; return false; }
      if (t == A_INLET && (i != 0 || c->periodic_x)) { err = "INLET node off column 0 (or periodic)"; return false; }
      if (t == A_OUTLET && (i != c->nx - 1 || c->periodic_x)) {
        err = "OUTLET node off column nx-1 (or periodic)";
        return false;
      }
      if (!c->periodic_x && (i == 0 || i == c->nx - 1) && t == A_FLUID) {
        err = "FLUID node in a ghost column";
        return false;
      }
    }
  return true;
}

}  // namespace

struct lbm_axi {
  lbm_axi_config cfg;
  AxiDev d;
  Layout L;
  char* buf;
  hipStream_t stream;
  int cur;           // buffer holding the current state
  int64_t step;
  std::vector<uint8_t> flags;
  std::string err;
};

namespace {

lbm_status fail(lbm_axi* c, lbm_status s, const std::string& m) {
  (c ? c->err : g_err) = m;
  return s;
}

#define AXCHK(ctx, call)                                                                          \
  do {                                                                                            \
    hipError_t e_ = (call);                                                                       \
    if (e_ != hipSuccess) return fail(ctx, LBM_E_DEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

dim3 grid(int64_t n) { return dim3((unsigned)((n + ABLOCK - 1) / ABLOCK)); }

template <class T>
hipError_t launch_step(lbm_axi* c) {
  const AxiDev& d = c->d;
  k_axi_bc<T><<<1, ABLOCK, 0, c->stream>>>(d, c->cur, c->step);
  k_axi_force<T><<<grid(d.n), ABLOCK, 0, c->stream>>>(d, c->cur, c->step);
  k_axi_collide<T><<<grid(d.n), ABLOCK, 0, c->stream>>>(d, c->cur);
  return hipGetLastError();
}

template <class T>
hipError_t launch_moments(lbm_axi* c) {
  k_axi_moments<T><<<grid(c->d.n), ABLOCK, 0, c->stream>>>(c->d, c->cur);
  return hipGetLastError();
}

hipError_t moments(lbm_axi* c) {
  return c->cfg.precision == LBM_FP64 ? launch_moments<double>(c) : launch_moments<float>(c);
}

}  // namespace

extern "C" {

lbm_status lbm_axi_query_size(const lbm_axi_config* cfg, size_t* bytes) {
  if (!bytes) return fail(nullptr, LBM_E_INVAL, "bytes NULL");
  if (!valid(cfg, g_err)) return LBM_E_INVAL;
  *bytes = plan(*cfg).total;
  return LBM_OK;
}

lbm_status lbm_axi_init(const lbm_axi_config* cfg, void* buf, size_t bytes, void* stream, lbm_axi** out) {
  if (!out) return fail(nullptr, LBM_E_INVAL, "out NULL");
  *out = nullptr;
  if (!valid(cfg, g_err)) return LBM_E_INVAL;
  const Layout L = plan(*cfg);
  if (!buf || bytes < L.total) return fail(nullptr, LBM_E_INVAL, "device buffer missing or too small");
  lbm_axi* c = new lbm_axi();
  c->cfg = *cfg;
  c->cfg.wave_cap = cfg->wave_cap > 0 ? cfg->wave_cap : 4096;
  c->flags.assign(cfg->flags, cfg->flags + (size_t)cfg->nx * cfg->nr);
  c->cfg.flags = nullptr;
  c->L = L;
  c->buf = (char*)buf;
  c->stream = (hipStream_t)stream;
  c->cur = 0;
  c->step = 0;
  AxiDev& d = c->d;
  d.nx = cfg->nx; d.nr = cfg->nr; d.px = cfg->periodic_x; d.cap = c->cfg.wave_cap;
  d.n = (int64_t)cfg->nx * cfg->nr;
  d.tau = cfg->tau;
  d.nu = (cfg->tau - 0.5) / 3.0;
  d.dref = 3.0 * cfg->p_ref;
  d.type = (const uint8_t*)(c->buf + L.type);
  for (int b = 0; b < 2; ++b) {
    d.g[b] = c->buf + L.g[b];
    d.D[b] = c->buf + L.D[b];
    d.jx[b] = c->buf + L.jx[b];
    d.jr[b] = c->buf + L.jr[b];
  }
  d.Fx = c->buf + L.Fx;
  d.Fr = c->buf + L.Fr;
  d.v0 = c->buf + L.v0;
  d.bc = (BcDev*)(c->buf + L.bc);
  d.wave = (double*)(c->buf + L.wave);
  d.err = (uint32_t*)(c->buf + L.err);
  d.G0 = 0.0;
  d.om = 0.0;
  d.fields = (double*)(c->buf + L.fields);
  auto bad = [&](hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    delete c;
    return LBM_E_DEVICE;
  };
  hipError_t e = hipMemsetAsync(buf, 0, L.total, c->stream);
  if (e != hipSuccess) return bad(e, "clear");
  e = hipMemcpyAsync(c->buf + L.type, c->flags.data(), c->flags.size(), hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) return bad(e, "node types");
  BcDev B[2];
  std::memset(B, 0, sizeof B);
  for (int b = 0; b < 2; ++b) {
    B[b].kind = lbm::BC_PRESSURE;
    B[b].boundary = b;
    B[b].Td = -1;
  }
  e = hipMemcpyAsync(d.bc, B, sizeof B, hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) return bad(e, "0D records");
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return bad(e, "synchronise");
  *out = c;
  return LBM_OK;
}

lbm_status lbm_axi_couple_0d(lbm_axi* c, int32_t b, int32_t kind, const double* params, int32_t np,
                             const double* state, int32_t nst) {
  if (!c) return LBM_E_INVAL;
  if (b < 0 || b > 1) return fail(c, LBM_E_INVAL, "boundary must be 0 (inlet) or 1 (outlet)");
  if (c->cfg.periodic_x) return fail(c, LBM_E_INVAL, "a periodic grid has no inlet or outlet");
  if (!params && np > 0) return fail(c, LBM_E_INVAL, "params NULL");
  const int need = kind == lbm::BC_PRESSURE || kind == lbm::BC_VELOCITY ? 1
                   : (kind == lbm::BC_WK3 ? 3 : (kind == lbm::BC_LV ? 11 : -1));
  if (need < 0) return fail(c, LBM_E_INVAL, "unknown 0D kind");
  if (np < need || np > 16) return fail(c, LBM_E_INVAL, "wrong number of 0D parameters");
  if (kind == lbm::BC_LV && b != 0) return fail(c, LBM_E_INVAL, "the LV model couples to the inlet only");
  if (kind == lbm::BC_WK3 && !(params[0] > 0 && params[1] > 0 && params[2] > 0))
    return fail(c, LBM_E_INVAL, "Windkessel Rp, C, Rd must be positive");
  if (kind == lbm::BC_LV && !(params[1] > 0 && params[2] > 0 && params[3] > 0 && params[5] > 0))
    return fail(c, LBM_E_INVAL, "LV Emin, Tc, Tmax, N_S must be positive");
  BcDev B;
  std::memset(&B, 0, sizeof B);
  B.kind = kind;
  B.boundary = b;
  for (int k = 0; k < np; ++k) B.par[k] = params[k];
  B.Td = -1;
  if (kind == lbm::BC_WK3) B.Pw = (state && nst > 0) ? state[0] : 0.0;
  if (kind == lbm::BC_LV) B.Pv = (state && nst > 0) ? state[0] : params[4];
  const int col = b == 0 ? 1 : c->cfg.nx - 2;
  double area = 0.0;
  for (int j = 0; j < c->cfg.nr; ++j)
    if (c->flags[col + (size_t)c->cfg.nx * j] == A_FLUID) area += 6.283185307179586476925286766559 * (j + 0.5);
  B.area = area;
  AXCHK(c, hipStreamSynchronize(c->stream));
  AXCHK(c, hipMemcpy(c->d.bc + b, &B, sizeof B, hipMemcpyHostToDevice));
  return LBM_OK;
}

lbm_status lbm_axi_set_body_force(lbm_axi* c, double G0, double omega) {
  if (!c) return LBM_E_INVAL;
  c->d.G0 = G0;
  c->d.om = omega;
  return LBM_OK;
}

lbm_status lbm_axi_set_rest(lbm_axi* c, double p) {
  if (!c) return LBM_E_INVAL;
  const double D0 = 3.0 * p - c->d.dref;
  if (c->cfg.precision == LBM_FP64) k_axi_fill<double><<<grid(c->d.n), ABLOCK, 0, c->stream>>>(c->d, c->cur, D0);
  else k_axi_fill<float><<<grid(c->d.n), ABLOCK, 0, c->stream>>>(c->d, c->cur, D0);
  AXCHK(c, hipGetLastError());
  AXCHK(c, moments(c));
  AXCHK(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

lbm_status lbm_axi_write_populations(lbm_axi* c, const double* g) {
  if (!c || !g) return LBM_E_INVAL;
  double* x = (double*)(c->buf + c->L.xfer);
  AXCHK(c, hipMemcpyAsync(x, g, (size_t)c->d.n * AQ * 8, hipMemcpyHostToDevice, c->stream));
  if (c->cfg.precision == LBM_FP64) k_axi_put<double><<<grid(c->d.n), ABLOCK, 0, c->stream>>>(c->d, c->cur, x, 1);
  else k_axi_put<float><<<grid(c->d.n), ABLOCK, 0, c->stream>>>(c->d, c->cur, x, 1);
  AXCHK(c, hipGetLastError());
  AXCHK(c, moments(c));
  AXCHK(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

lbm_status lbm_axi_read_populations(lbm_axi* c, double* g) {
  if (!c || !g) return LBM_E_INVAL;
  double* x = (double*)(c->buf + c->L.xfer);
  if (c->cfg.precision == LBM_FP64) k_axi_put<double><<<grid(c->d.n), ABLOCK, 0, c->stream>>>(c->d, c->cur, x, 0);
  else k_axi_put<float><<<grid(c->d.n), ABLOCK, 0, c->stream>>>(c->d, c->cur, x, 0);
  AXCHK(c, hipGetLastError());
  AXCHK(c, hipMemcpyAsync(g, x, (size_t)c->d.n * AQ * 8, hipMemcpyDeviceToHost, c->stream));
  AXCHK(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

lbm_status lbm_axi_step(lbm_axi* c, int64_t nsteps) {
  if (!c) return LBM_E_INVAL;
  if (nsteps < 0) return fail(c, LBM_E_INVAL, "nsteps < 0");
  for (int64_t s = 0; s < nsteps; ++s) {
    AXCHK(c, c->cfg.precision == LBM_FP64 ? launch_step<double>(c) : launch_step<float>(c));
    c->cur ^= 1;
    c->step++;
  }
  return LBM_OK;
}

lbm_status lbm_axi_read_fields(lbm_axi* c, double* p, double* ux, double* ur) {
  if (!c) return LBM_E_INVAL;
  const AxiDev& d = c->d;
  if (c->cfg.precision == LBM_FP64) {
    k_axi_force<double><<<grid(d.n), ABLOCK, 0, c->stream>>>(d, c->cur, c->step);
    k_axi_fields<double><<<grid(d.n), ABLOCK, 0, c->stream>>>(d, c->cur);
  } else {
    k_axi_force<float><<<grid(d.n), ABLOCK, 0, c->stream>>>(d, c->cur, c->step);
    k_axi_fields<float><<<grid(d.n), ABLOCK, 0, c->stream>>>(d, c->cur);
  }
  AXCHK(c, hipGetLastError());
  double* outs[3] = {p, ux, ur};
  for (int k = 0; k < 3; ++k)
    if (outs[k]) AXCHK(c, hipMemcpyAsync(outs[k], d.fields + k * d.n, (size_t)d.n * 8, hipMemcpyDeviceToHost, c->stream));
  AXCHK(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

lbm_status lbm_axi_read_waveforms(lbm_axi* c, double* out, int64_t cap, int64_t* n) {
  if (!c || !n || (cap > 0 && !out)) return LBM_E_INVAL;
  AXCHK(c, hipStreamSynchronize(c->stream));
  const int64_t have = std::min<int64_t>(c->step, c->d.cap);
  const int64_t m = std::min<int64_t>(have, cap);
  std::vector<double> ring((size_t)c->d.cap * AREC);
  if (m > 0) AXCHK(c, hipMemcpy(ring.data(), c->d.wave, ring.size() * 8, hipMemcpyDeviceToHost));
  for (int64_t k = 0; k < m; ++k) {
    const int64_t s = c->step - m + k;
    std::memcpy(out + k * AREC, ring.data() + (s % c->d.cap) * AREC, AREC * 8);
  }
  *n = m;
  return LBM_OK;
}

lbm_status lbm_axi_sync(lbm_axi* c) {
  if (!c) return LBM_E_INVAL;
  AXCHK(c, hipStreamSynchronize(c->stream));
  uint32_t e = 0;
  AXCHK(c, hipMemcpy(&e, c->d.err, 4, hipMemcpyDeviceToHost));
  if (e) return fail(c, LBM_E_UNSTABLE, "a column flux or pressure became non-finite");
  return LBM_OK;
}

const char* lbm_axi_last_error(const lbm_axi* c) { return c ? c->err.c_str() : g_err.c_str(); }

lbm_status lbm_axi_destroy(lbm_axi* c) {
  if (!c) return LBM_E_INVAL;
  (void)hipStreamSynchronize(c->stream);
  delete c;
  return LBM_OK;
}

}  // extern "C"
