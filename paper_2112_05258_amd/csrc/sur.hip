// Learned surrogate: MLP forward, backward and Adam on the gfx950 matrix
// cores.  BF16 operands, FP32 accumulation (v_mfma_f32_32x32x16_bf16), FP32
// master weights, gradients and Adam moments.
//
// Kernels
//   k_gemm<AKC, BKC, EPI>  C = A B with a fused epilogue; A is m x k and B is
//                          k x n, each stored either k-contiguous (KC) or
//                          m- resp. n-contiguous.  The three forms are the
//                          forward product (h W^T), the backward data
//                          product (dz W) and the weight gradient (dz^T h).
//   k_prep_x / k_prep_t    input normalisation (optionally gathering a
//                          shuffled mini-batch) and target standardisation
//   k_loss                 squared error, its gradient in BF16, loss sum
//   k_colsum               bias gradients
//   k_adam / k_cast        Adam step; BF16 (K-padded) copy of the weights
//   k_frag / k_mlp_fwd     inference of the whole network in one kernel for
//                          width 512 and 512 outputs: weights in MFMA fragment
//                          order, activations kept in LDS between layers
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "lbm_surrogate.h"

namespace sur {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// block tile BM x BN, k-step BK; 4 waves, each 64 x 64 = 2 x 2 MFMA tiles.
// The training products are small (a few hundred rows) and their k-loops
// wait on memory once per k-step, so the k-step is deep: 64.
constexpr int BM = 128, BN = 128, BK = 64;
constexpr int LDK = BK + 8;  // LDS row pitch in bf16 (144 B: 16-B aligned, rows 36 banks apart)
constexpr int TQ = BK / 16;  // 16-byte chunks per lane of a 128 x BK tile
static_assert(BK % 32 == 0, "transposed tiles are stored as pairs of k");
constexpr int KPAD = 32;     // input width of the first layer is padded to this

enum { EPI_FWD_GELU = 0, EPI_FWD_OUT = 1, EPI_BWD_GELU = 2, EPI_WGRAD = 3 };

// FP32 -> BF16, round to nearest even (NaN kept quiet); both results are
// formed and one selected, so an epilogue of many conversions stays
// straight-line code
__device__ __forceinline__ uint16_t f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  const uint32_t rne = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
  const uint32_t qnan = (u >> 16) | 0x40u;
  return (uint16_t)((u & 0x7fffffffu) > 0x7f800000u ? qnan : rne);
}

// Phi(z) = (1 + erf(z / sqrt 2)) / 2, the standard normal CDF, with erf from
// Abramowitz & Stegun 7.1.26 (|error| <= 1.5e-7): for x >= 0,
// 1 - erf(x) = t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) exp(-x^2),
// t = 1 / (1 + p x).  The z < 0 side takes that tail directly (no
// cancellation).  About a dozen instructions, against erff's several dozen:
// the GELU epilogues of the forward products are VALU work next to MFMA.
__device__ __forceinline__ float phi_cdf(float z) {
  const float x = fabsf(z) * 0.70710678118654752f;
  const float t = __builtin_amdgcn_rcpf(1.0f + 0.3275911f * x);
  const float poly =
      t * (0.254829592f + t * (-0.284496736f + t * (1.421413741f + t * (-1.453152027f + t * 1.061405429f))));
  const float q = poly * __expf(-x * x);   // 1 - erf(x)
  return z >= 0.0f ? 1.0f - 0.5f * q : 0.5f * q;
}

__device__ __forceinline__ float gelu(float z) { return z * phi_cdf(z); }

// d/dz [z Phi(z)] = Phi(z) + z phi(z)
__device__ __forceinline__ float gelu_grad(float z) {
  return phi_cdf(z) + z * 0.39894228040143268f * __expf(-0.5f * z * z);
}

struct GemmArgs {
  const uint16_t* A;
  int64_t lda;
  int a_ext;            // rows of A along m that exist in memory (loads beyond read zero)
  const uint16_t* B;
  int64_t ldb;
  int b_ext;            // the same along n
  int M, N, K;          // output m x n (stores are bounded by M, N), depth K (multiple of 8)
  const float* bias;    // n
  const float* zin;     // EPI_BWD_GELU: pre-activation of the layer below (ldo)
  float* outf;          // FP32 output (EPI_FWD_OUT, EPI_WGRAD)
  uint16_t* outh;       // BF16 output (EPI_FWD_GELU, EPI_BWD_GELU)
  float* zout;          // EPI_FWD_GELU: pre-activation (may be null)
  int64_t ldo;
  const float* mu;      // EPI_FWD_OUT: output de-standardisation (may be null)
  const float* sigma;
  int ksplit;           // EPI_WGRAD: depth split over ksplit workgroups (1: none)
  float* part;          // their partial products, ksplit x M x N
};

// the backward data product of a depth split: the slices added in order,
// then the GELU derivative, BF16 out (as the product's own epilogue does)
__global__ void k_sum_parts_bwd(const float* __restrict__ part, int ksplit, int M, int N,
                                const float* __restrict__ zin, uint16_t* __restrict__ outh, int64_t ldo) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)M * N) return;
  float s = 0.0f;
#pragma unroll 4
  for (int z = 0; z < ksplit; ++z) s += part[(int64_t)z * M * N + e];
  const int64_t o = (e / N) * ldo + e % N;
  outh[o] = f2bf(s * gelu_grad(zin[o]));
}

// out[m ldo + n] = sum over z of part[z][m][n], in z order
__global__ void k_sum_parts(const float* __restrict__ part, int ksplit, int M, int N, float* __restrict__ out,
                            int64_t ldo) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)M * N) return;
  float s = 0.0f;
#pragma unroll 16
  for (int z = 0; z < ksplit; ++z) s += part[(int64_t)z * M * N + e];
  out[(e / N) * ldo + e % N] = s;
}

// A 128 x BK tile (rows r0.., depth k0..) in two steps: its 16 BK 16-byte
// chunks into registers (TQ per lane), then into LDS as S[r][k].  KC:
// G[r * ld + k], a chunk is 8 k of one row; otherwise G[k * ld + r], a chunk
// is 8 rows of one k, transposed on the way into LDS: a lane takes the chunks
// of two adjacent k (2p, 2p + 1) over the same 8 rows and writes each row's
// pair as one 4-byte word, the 32 pairs of a wave's half side by side (rows
// 8 apart fall 32 banks apart: no bank conflicts).  Every chunk is loaded
// from an index clamped into the matrix (ext >= 1 rows, resp. a multiple of
// 8; K a positive multiple of 8) and the ones outside it are zeroed only
// when stored, so no load sits in a branch and nothing waits for the loads
// before the store.
template <bool KC>
__device__ __forceinline__ void tile_gload(uint4 (&v)[TQ], bool (&ok)[TQ], const uint16_t* G, int64_t ld, int ext,
                                           int r0, int k0, int K, int tid) {
#pragma unroll
  for (int q = 0; q < TQ; ++q) {
    const int c = tid + 256 * q;
    if (KC) {
      const int r = r0 + c / (BK / 8), k = k0 + (c % (BK / 8)) * 8;
      ok[q] = r < ext && k + 8 <= K;
      v[q] = *(const uint4*)(G + (int64_t)min(r, ext - 1) * ld + min(k, K - 8));
    } else {
      const int u = tid + 256 * (q >> 1);          // pair unit: k pair u % (BK / 2), 8 rows u / (BK / 2)
      const int k = k0 + 2 * (u % (BK / 2)) + (q & 1), r = r0 + (u / (BK / 2)) * 8;
      ok[q] = k < K && r + 8 <= ext;
      v[q] = *(const uint4*)(G + (int64_t)min(k, K - 1) * ld + min(r, ext - 8));
    }
  }
}
template <bool KC>
__device__ __forceinline__ void tile_sstore(uint16_t* S, const uint4 (&v)[TQ], const bool (&ok)[TQ], int tid) {
  if (KC) {
#pragma unroll
    for (int q = 0; q < TQ; ++q) {
      const int c = tid + 256 * q;
      *(uint4*)(S + (c / (BK / 8)) * LDK + (c % (BK / 8)) * 8) = ok[q] ? v[q] : make_uint4(0, 0, 0, 0);
    }
  } else {
#pragma unroll
    for (int q = 0; q < TQ; q += 2) {
      const int u = tid + 256 * (q >> 1);
      const int p = u % (BK / 2), rc = (u / (BK / 2)) * 8;
      const uint4 w0 = ok[q] ? v[q] : make_uint4(0, 0, 0, 0), w1 = ok[q + 1] ? v[q + 1] : make_uint4(0, 0, 0, 0);
      const uint16_t* e0 = (const uint16_t*)&w0;
      const uint16_t* e1 = (const uint16_t*)&w1;
#pragma unroll
      for (int j = 0; j < 8; ++j)
        *(uint32_t*)(S + (rc + j) * LDK + 2 * p) = (uint32_t)e0[j] | ((uint32_t)e1[j] << 16);
    }
  }
}

template <bool AKC, bool BKC, int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) uint16_t As[2][BM * LDK];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][BN * LDK];
  const int tid = (int)threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m0 = (int)blockIdx.y * BM, n0 = (int)blockIdx.x * BN;
  // split over the depth (weight gradients of a large batch, backward data
  // products of few rows): workgroup z takes depth kb .. ke and writes its
  // partial product to slice z of g.part, which k_sum_parts (resp.
  // k_sum_parts_bwd, with the GELU derivative) adds up in slice order
  const int kz = (int)blockIdx.z;
  const int kc = g.ksplit > 1 ? ((g.K + g.ksplit - 1) / g.ksplit + BK - 1) / BK * BK : g.K;
  const int kb = kz * kc, ke = min(g.K, kb + kc);
  const int wm = (wv >> 1) * 64, wn = (wv & 1) * 64;
  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

  // operand fragments: lane l supplies row (l % 32) and the 8 k of half (l / 32).
  // The next k-step's tiles are fetched into registers while the current one
  // is multiplied out of LDS, then stored into the other LDS buffer.
  const int fr = lane & 31, fk = (lane >> 5) * 8;
  uint4 ra[TQ], rb[TQ];
  bool oa[TQ], ob[TQ];
  if (kb < ke) {
    tile_gload<AKC>(ra, oa, g.A, g.lda, g.a_ext, m0, kb, ke, tid);
    tile_gload<BKC>(rb, ob, g.B, g.ldb, g.b_ext, n0, kb, ke, tid);
    tile_sstore<AKC>(As[0], ra, oa, tid);
    tile_sstore<BKC>(Bs[0], rb, ob, tid);
  }
  __syncthreads();
  const int nk = kb < ke ? (ke - kb + BK - 1) / BK : 0;
  for (int st = 0; st < nk; ++st) {
    const int cur = st & 1;
    const bool more = st + 1 < nk;
    if (more) {
      tile_gload<AKC>(ra, oa, g.A, g.lda, g.a_ext, m0, kb + (st + 1) * BK, ke, tid);
      tile_gload<BKC>(rb, ob, g.B, g.ldb, g.b_ext, n0, kb + (st + 1) * BK, ke, tid);
    }
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      bf16x8 a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = *(const bf16x8*)(As[cur] + (wm + t * 32 + fr) * LDK + kk + fk);
        b[t] = *(const bf16x8*)(Bs[cur] + (wn + t * 32 + fr) * LDK + kk + fk);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) {
      tile_sstore<AKC>(As[cur ^ 1], ra, oa, tid);
      tile_sstore<BKC>(Bs[cur ^ 1], rb, ob, tid);
    }
    __syncthreads();
  }

  // accumulator v of lane l holds row 8 (v / 4) + 4 (l / 32) + v % 4 and
  // column l % 32 of its 32 x 32 tile.  The epilogue's operand loads (bias,
  // pre-activations) are all issued before the first is used, at indices
  // clamped into the matrix, so they do not wait on each other one by one
  // behind the per-element bounds test.
  auto row_of = [&](int i, int v) { return m0 + wm + i * 32 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3); };
  auto col_of = [&](int j) { return n0 + wn + j * 32 + (lane & 31); };
  float zb[2][2][16];
  if (EPI == EPI_BWD_GELU && g.ksplit <= 1) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v)
          zb[i][j][v] = g.zin[(int64_t)min(row_of(i, v), g.M - 1) * g.ldo + min(col_of(j), g.N - 1)];
  }
  float bj[2] = {0.0f, 0.0f}, mj[2] = {0.0f, 0.0f}, sj[2] = {1.0f, 1.0f};
  if (EPI == EPI_FWD_GELU || EPI == EPI_FWD_OUT) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = min(col_of(j), g.N - 1);
      bj[j] = g.bias[n];
      if (EPI == EPI_FWD_OUT && g.mu) {
        mj[j] = g.mu[n];
        sj[j] = g.sigma[n];
      }
    }
  }
  // a tile inside the matrix stores without per-element tests (straight-line
  // code: no waits for earlier stores between the elements)
  // the optional output (pre-activations, de-standardisation, the split's
  // partial slice) is chosen once, outside the element loop
  const bool full = m0 + BM <= g.M && n0 + BN <= g.N;
  const bool opt = EPI == EPI_FWD_GELU ? g.zout != nullptr : EPI == EPI_FWD_OUT ? g.mu != nullptr : g.ksplit > 1;
  auto epi = [&](auto checked, auto with) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int m = row_of(i, v);
        const int n = col_of(j);
        if (decltype(checked)::value && (m >= g.M || n >= g.N)) continue;
        const float s = acc[i][j][v];
        const int64_t o = (int64_t)m * g.ldo + n;
        if (EPI == EPI_FWD_GELU) {
          const float z = s + bj[j];
          if (decltype(with)::value) g.zout[o] = z;
          g.outh[o] = f2bf(gelu(z));
        } else if (EPI == EPI_FWD_OUT) {
          const float y = s + bj[j];
          g.outf[o] = decltype(with)::value ? mj[j] + sj[j] * y : y;
        } else if (EPI == EPI_BWD_GELU) {
          if (decltype(with)::value)
            g.part[((int64_t)kz * g.M + m) * g.N + n] = s;
          else
            g.outh[o] = f2bf(s * gelu_grad(zb[i][j][v]));
        } else if (decltype(with)::value) {
          g.part[((int64_t)kz * g.M + m) * g.N + n] = s;
        } else {
          g.outf[o] = s;
        }
      }
  };
  if (full && opt)
    epi(std::false_type{}, std::true_type{});
  else if (full)
    epi(std::false_type{}, std::false_type{});
  else if (opt)
    epi(std::true_type{}, std::true_type{});
  else
    epi(std::true_type{}, std::false_type{});
}

// Forward product C = A B^T with both operands k-contiguous (activations h and
// weights W): training's forward pass, and inference for other shapes.  Block tile 128 x 256, each of the 4
// waves 64 x 128 (2 x 4 MFMA tiles: 6 fragment reads from LDS per 8 MFMAs),
// k-step BK.  The next k-step's tiles are fetched into registers while the
// current one is multiplied out of LDS, and stored into the other half of a
// double-buffered LDS after it: one barrier per k-step.
constexpr int FBM = 128, FBN = 256;
constexpr int FWD_SMALL_M = 8192;   // at most this many rows: the 128 x 128 kernel

template <int EPI>
__global__ __launch_bounds__(256) void k_gemm_fwd(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) uint16_t As[2][FBM * LDK];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][FBN * LDK];
  const int tid = (int)threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m0 = (int)blockIdx.y * FBM, n0 = (int)blockIdx.x * FBN;
  const int wm = (wv >> 1) * 64, wn = (wv & 1) * 128;
  f32x16 acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;
  // 16-byte chunks of 8 k: A tile 128 x BK = 16 BK chunks (TQ per lane), B
  // tile 256 x BK (2 TQ per lane); out-of-range chunks are zero
  // (loads from indices clamped into the matrices, zeroed when stored: no
  // load in a branch, no wait before the store)
  constexpr int CR = BK / 8;   // chunks per row
  uint4 ra[TQ], rb[2 * TQ];
  bool oa[TQ], ob[2 * TQ];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < TQ; ++q) {
      const int c = tid + 256 * q, r = m0 + c / CR, k = k0 + (c % CR) * 8;
      oa[q] = r < g.a_ext && k + 8 <= g.K;
      ra[q] = *(const uint4*)(g.A + (int64_t)min(r, g.a_ext - 1) * g.lda + min(k, g.K - 8));
    }
#pragma unroll
    for (int q = 0; q < 2 * TQ; ++q) {
      const int c = tid + 256 * q, r = n0 + c / CR, k = k0 + (c % CR) * 8;
      ob[q] = r < g.b_ext && k + 8 <= g.K;
      rb[q] = *(const uint4*)(g.B + (int64_t)min(r, g.b_ext - 1) * g.ldb + min(k, g.K - 8));
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < TQ; ++q) {
      const int c = tid + 256 * q;
      *(uint4*)(As[buf] + (c / CR) * LDK + (c % CR) * 8) = oa[q] ? ra[q] : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 2 * TQ; ++q) {
      const int c = tid + 256 * q;
      *(uint4*)(Bs[buf] + (c / CR) * LDK + (c % CR) * 8) = ob[q] ? rb[q] : make_uint4(0, 0, 0, 0);
    }
  };
  const int fr = lane & 31, fk = (lane >> 5) * 8;
  gload(0);
  sstore(0);
  __syncthreads();
  const int nk = (g.K + BK - 1) / BK;
  for (int s = 0; s < nk; ++s) {
    const int cur = s & 1;
    const bool more = s + 1 < nk;
    if (more) gload((s + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      bf16x8 a[2], b[4];
#pragma unroll
      for (int t = 0; t < 2; ++t) a[t] = *(const bf16x8*)(As[cur] + (wm + t * 32 + fr) * LDK + kk + fk);
#pragma unroll
      for (int t = 0; t < 4; ++t) b[t] = *(const bf16x8*)(Bs[cur] + (wn + t * 32 + fr) * LDK + kk + fk);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) sstore(cur ^ 1);
    __syncthreads();
  }
  // per-column operands loaded once, before the element loop (clamped
  // indices; out-of-range elements are not stored)
  float bj[4], mj[4], sj[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int n = min(n0 + wn + j * 32 + (lane & 31), g.N - 1);
    bj[j] = g.bias[n];
    mj[j] = EPI == EPI_FWD_OUT && g.mu ? g.mu[n] : 0.0f;
    sj[j] = EPI == EPI_FWD_OUT && g.mu ? g.sigma[n] : 1.0f;
  }
  // a tile inside the matrix stores without per-element tests, and the
  // optional output (pre-activations, resp. de-standardisation) is chosen
  // once: straight-line code, no waits for earlier stores between elements
  const bool full = m0 + FBM <= g.M && n0 + FBN <= g.N;
  const bool opt = EPI == EPI_FWD_GELU ? g.zout != nullptr : g.mu != nullptr;
  auto epi = [&](auto checked, auto with) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int m = m0 + wm + i * 32 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
        const int n = n0 + wn + j * 32 + (lane & 31);
        if (decltype(checked)::value && (m >= g.M || n >= g.N)) continue;
        const float s = acc[i][j][v] + bj[j];
        const int64_t o = (int64_t)m * g.ldo + n;
        if (EPI == EPI_FWD_GELU) {
          if (decltype(with)::value) g.zout[o] = s;
          g.outh[o] = f2bf(gelu(s));
        } else {
          g.outf[o] = decltype(with)::value ? mj[j] + sj[j] * s : s;
        }
      }
  };
  if (full && opt)
    epi(std::false_type{}, std::true_type{});
  else if (full)
    epi(std::false_type{}, std::false_type{});
  else if (opt)
    epi(std::true_type{}, std::true_type{});
  else
    epi(std::true_type{}, std::false_type{});
}

// inputs: X0[r][j] = 2 (x - lo) / (hi - lo) - 1 for r < m and j < n_in; 0 for
// the padding columns up to KPAD and the padding rows m <= r < mp
// (rows picked by idx outside [0, nrows) read zeros and set *err)
__global__ void k_prep_x(const float* __restrict__ x, int nrows, const int32_t* __restrict__ idx, int m, int mp,
                         int nin, const float* __restrict__ lo, const float* __restrict__ hi,
                         uint16_t* __restrict__ X0, int* __restrict__ err) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)mp * KPAD) return;
  const int r = (int)(e / KPAD), j = (int)(e % KPAD);
  float v = 0.0f;
  if (j < nin && r < m) {
    const int64_t src = idx ? idx[r] : r;
    if (src >= 0 && src < nrows)
      v = 2.0f * (x[src * nin + j] - lo[j]) / (hi[j] - lo[j]) - 1.0f;
    else
      atomicOr(err, 1);
  }
  X0[e] = f2bf(v);
}

// standardised targets tn = (t - mu) / sigma
__global__ void k_prep_t(const float* __restrict__ t, int nrows, const int32_t* __restrict__ idx, int m, int nout,
                         const float* __restrict__ mu, const float* __restrict__ sigma, float* __restrict__ tn) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)m * nout) return;
  const int r = (int)(e / nout), j = (int)(e % nout);
  const int64_t src = idx ? idx[r] : r;
  tn[e] = (src >= 0 && src < nrows) ? (t[src * nout + j] - mu[j]) / sigma[j] : 0.0f;
}

// loss = mean (y - tn)^2; dy = 2 (y - tn) / count in BF16
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ y, const float* __restrict__ tn, int64_t n,
                                              uint16_t* __restrict__ dy, double* __restrict__ loss) {
  __shared__ double part[256];
  // grid-stride over the elements: a capped grid keeps the atomics on the
  // one loss word few
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const float d = y[e] - tn[e];
    dy[e] = f2bf(2.0f * d / (float)n);
    s += (double)d * (double)d;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss, part[0] / (double)n);
}

// Bias gradients db[j] = sum_r dz[r][j] in two deterministic passes: the
// rows in chunks of CROWS, one workgroup row per chunk (so a large batch
// spreads over many workgroups instead of one column-thread walking every
// row), then the chunks' partial sums added in chunk order.
constexpr int CROWS = 64;
__global__ void k_colsum_part(const uint16_t* __restrict__ dz, int m, int n, float* __restrict__ part) {
  const int j = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (j >= n) return;
  const int r0 = (int)blockIdx.y * CROWS, r1 = min(m, r0 + CROWS);
  float s = 0.0f;
  if (r1 - r0 == CROWS) {   // a whole chunk: all its loads in flight at once
    uint16_t v[CROWS];
#pragma unroll
    for (int r = 0; r < CROWS; ++r) v[r] = dz[(int64_t)(r0 + r) * n + j];
#pragma unroll
    for (int r = 0; r < CROWS; ++r) s += __uint_as_float((uint32_t)v[r] << 16);
  } else {
    for (int r = r0; r < r1; ++r) s += __uint_as_float((uint32_t)dz[(int64_t)r * n + j] << 16);
  }
  part[(int64_t)blockIdx.y * n + j] = s;
}
__global__ void k_colsum_fin(const float* __restrict__ part, int nchunk, int n, float* __restrict__ db) {
  const int j = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (j >= n) return;
  float s = 0.0f;
#pragma unroll 16
  for (int q = 0; q < nchunk; ++q) s += part[(int64_t)q * n + j];
  db[j] = s;
}

struct LayerMap {
  int nl;
  int64_t off[8];       // first parameter of layer l (W then b)
  int64_t woff[8];      // first element of its BF16 weight copy
  int out[8], in[8], kp[8];
};

// BF16 copy of the weights, rows padded to kp columns (the padding stays 0)
__device__ __forceinline__ void to_bf16_copy(const LayerMap& L, int64_t p, float w, uint16_t* wb) {
#pragma unroll 1
  for (int l = 0; l < L.nl; ++l) {
    const int64_t nw = (int64_t)L.out[l] * L.in[l];
    if (p >= L.off[l] && p < L.off[l] + nw) {
      const int64_t q = p - L.off[l];
      wb[L.woff[l] + (q / L.in[l]) * L.kp[l] + q % L.in[l]] = f2bf(w);
      return;
    }
  }
}

__global__ void k_cast(const float* __restrict__ w, int64_t n, LayerMap L, uint16_t* __restrict__ wb) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) to_bf16_copy(L, p, w[p], wb);
}

__global__ void k_adam(float* __restrict__ w, float* __restrict__ m1, float* __restrict__ m2,
                       const float* __restrict__ g, int64_t n, float lr, float b1, float b2, float eps,
                       float bc1, float bc2, LayerMap L, uint16_t* __restrict__ wb) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const float gp = g[p];
  const float a = b1 * m1[p] + (1.0f - b1) * gp;
  const float b = b2 * m2[p] + (1.0f - b2) * gp * gp;
  m1[p] = a;
  m2[p] = b;
  const float wn = w[p] - lr * (a / bc1) / (sqrtf(b / bc2) + eps);
  w[p] = wn;
  to_bf16_copy(L, p, wn, wb);
}


// ---------------------------------------------------------------------------
// Fused inference for width 512 and 512 outputs (the surrogate's shape)
// ---------------------------------------------------------------------------
// One 1024-lane workgroup (16 waves, four per SIMD) per 128 rows holds the
// rows' activations in LDS (128 x 512 BF16, row pitch padded by 16 bytes)
// from the input normalisation to the output layer, so hidden activations
// never travel to HBM.  Wave w computes output columns 32 w .. 32 w + 31 of
// every layer (4 x 1 MFMA tiles of 32 x 32): activation fragments come from
// LDS one k-step ahead, weight fragments stream from L2 in fragment order two
// k-steps ahead of the MFMAs that use them (a phase's first two before the
// barrier that ends the phase before).  The GELU epilogue writes the
// layer's output over its input in LDS between two barriers.
constexpr int MR = 128, MWID = 512, APITCH = MWID + 8;

// weights in MFMA fragment order: element ((ks N/32 + nt) 64 + lane) 8 + e of
// layer l (N outputs, depth K = kp) is W[32 nt + lane % 32][16 ks + 8 (lane / 32) + e],
// so the 64 lanes of a wave read one tile's k-step as 1 KB in a row, and the
// N/32 tiles of one k-step lie side by side: the waves of every workgroup,
// which read the same k-step of different tiles at about the same time,
// spread over all L2 channels instead of meeting in the few that addresses
// a power-of-two distance apart share
__global__ void k_frag(const uint16_t* __restrict__ wb, LayerMap L, int64_t n, uint16_t* __restrict__ wf) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int l = 0;
  while (l + 1 < L.nl && p >= L.woff[l + 1]) ++l;
  const int64_t q = p - L.woff[l];
  const int K = L.kp[l];
  const int e = (int)(q & 7), lane = (int)((q >> 3) & 63);
  const int64_t t = q >> 9;
  const int NT = L.out[l] / 32;
  const int nt = (int)(t % NT), ks = (int)(t / NT);
  wf[p] = wb[L.woff[l] + (int64_t)(nt * 32 + (lane & 31)) * K + ks * 16 + (lane >> 5) * 8 + e];
}

// The same fragment-order copy straight from FP32 parameters (the
// composition of the BF16 cast with rows padded to kp, and k_frag, element
// for element): used by the allocation-free inference, whose fragments live
// in a static device array rather than a context's memory.
__global__ void k_frag_f32(const float* __restrict__ w, LayerMap L, int64_t n, uint16_t* __restrict__ wf) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int l = 0;
  while (l + 1 < L.nl && p >= L.woff[l + 1]) ++l;
  const int64_t q = p - L.woff[l];
  const int e = (int)(q & 7), lane = (int)((q >> 3) & 63);
  const int64_t t = q >> 9;
  const int NT = L.out[l] / 32;
  const int nt = (int)(t % NT), ks = (int)(t / NT);
  const int row = nt * 32 + (lane & 31), col = ks * 16 + (lane >> 5) * 8 + e;
  wf[p] = col < L.in[l] ? f2bf(w[L.off[l] + (int64_t)row * L.in[l] + col]) : (uint16_t)0;
}

// Scratch of the allocation-free inference: the fragment-order BF16 weights
// of one network (at most NOALLOC_WEIGHTS values: n_in <= 32, width 512,
// up to 7 hidden layers, 512 outputs need 1 851 392).  One copy per GPU for
// the life of the process; every call on a GPU shares it.
constexpr int64_t NOALLOC_WEIGHTS = (int64_t)2 << 20;
__device__ __align__(256) uint16_t scratch[NOALLOC_WEIGHTS];

struct MlpArgs {
  const float* x;       // m x nin inputs
  int m, nin;
  const float* lo;
  const float* hi;
  const uint16_t* wf;   // weights in fragment order (layout of wb)
  const float* w;       // FP32 parameters (biases)
  LayerMap L;
  const float* mu;
  const float* sigma;
  float* y;             // m x 512 physical outputs
};

// GELU for the inference epilogue, the same A&S 7.1.26 tail as phi_cdf
// rearranged: with q = (1 - erf(|z| / sqrt 2)) / 2 the upper tail,
// z Phi(z) = max(z, 0) - |z| q for either sign of z, so no select is needed;
// the constants absorb 1 / sqrt 2, the 1/2 of q and log2 e (v_exp_f32 is a
// power of two).  Eleven VALU instructions and two transcendentals.
__device__ __forceinline__ float gelu_epi(float z) {
  const float t = __builtin_amdgcn_rcpf(fmaf(fabsf(z), 0.3275911f * 0.70710678118654752f, 1.0f));
  const float poly =
      0.5f * 0.254829592f +
      t * (0.5f * -0.284496736f + t * (0.5f * 1.421413741f + t * (0.5f * -1.453152027f + t * (0.5f * 1.061405429f))));
  const float e = __builtin_amdgcn_exp2f((z * -0.72134752044448170f) * z);   // exp(-z^2 / 2)
  // max(z, 0) as a median: one instruction, where fmaxf adds a canonicalising max
  return fmaf(-(fabsf(z) * t) * poly, e, __builtin_amdgcn_fmed3f(z, 0.0f, 3.0e38f));
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// The workgroup's 128 rows are two halves of 64, each a pipeline of its own
// through the layers: one phase multiplies one half's layer while the same
// waves, between those products, run the other half's GELU epilogue of the
// layer before, so the vector ALUs work while the matrix cores do.
// Activations stay in LDS and are overwritten in place; the two halves
// touch disjoint rows and one barrier separates the phases.

// compile-time loop: f(integral_constant<int, k>) for k = B .. E - 1
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// GELU of accumulator n (0..32 NJ - 1, in (i, j, v) order) of a half's (column,
// row) tiles; every fourth one stores the group of four as one 8-byte LDS
// write (lane l: row i 32 + l % 32, columns 8 (v / 4) + 4 (l / 32) .. + 3 of
// tile j).
template <int NJ, int N>
__device__ __forceinline__ void epi_value(const f32x16 (&acc)[2][NJ], float (&gv)[4], uint16_t* act, int wv,
                                          int lane) {
  constexpr int i = N / (16 * NJ), j = (N / 16) % NJ, v = N & 15;
  gv[N & 3] = gelu_epi(acc[i][j][v]);
  if ((N & 3) == 3) {
    const int row = i * 32 + (lane & 31), col = (NJ * wv + j) * 32 + 8 * (v >> 2) + 4 * (lane >> 5);
    // hardware round-to-nearest-even conversion, two values at a time
    const bf16x2 lo = __builtin_convertvector((f32x2){gv[0], gv[1]}, bf16x2);
    const bf16x2 hi = __builtin_convertvector((f32x2){gv[2], gv[3]}, bf16x2);
    *(uint2*)(act + row * APITCH + col) = make_uint2(__builtin_bit_cast(uint32_t, lo), __builtin_bit_cast(uint32_t, hi));
  }
}

template <int NJ, int N0, int PER>
__device__ __forceinline__ void epi_values(const f32x16 (&acc)[2][NJ], float (&gv)[4], uint16_t* act, int wv, int lane) {
  if constexpr (PER > 0) {
    epi_value<NJ, N0>(acc, gv, act, wv, lane);
    epi_values<NJ, N0 + 1, PER - 1>(acc, gv, act, wv, lane);
  }
}

// the weight fragments of a phase's first two k-steps (depth 16 NKS >= 2),
// loaded before the barrier that precedes the phase: weights do not depend
// on the activations the barrier orders
template <int NJ, int NKS>
__device__ __forceinline__ void mlp_pre(bf16x8 (&pre)[2][NJ], const uint16_t* wf, int wv, int lane) {
  constexpr int NT = MWID / 32;
  const __amdgpu_buffer_rsrc_t W = __builtin_amdgcn_make_buffer_rsrc((void*)wf, (short)0, NT * 64 * 16 * NKS, 0x00020000);
  const int wlane = ((NJ * wv) * 64 + lane) * 16;
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    pre[0][j] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(W, wlane, j * 64 * 16, 0));
    pre[1][j] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(W, wlane, (NT * 64 + j * 64) * 16, 0));
  }
}

// One phase: the products of one layer (depth 16 KS) for one half (two
// 32-row blocks, rows at actM) and this wave's 32 NJ output columns into accM,
// the first k-step taking the bias tiles bt as its accumulator input; with
// DRAIN the epilogue of the other half (accE, rows at actE) is spread over
// the k-steps.  pre holds the weight fragments of the first two k-steps on
// entry and, with NKS > 0, those of the next phase (weights wf_next, depth
// 16 NKS) on exit.  TR: the weights are the A operand and the activations the B
// operand, so a tile holds (output column, row) and lane l has row l % 32
// and four consecutive columns per group of four accumulators.  !TR: (row,
// output column), lane l has column l % 32 (the output layer, whose FP32
// rows leave in 128-byte runs).
template <int NJ, bool TR, int KS, bool DRAIN, int NKS>
__device__ __forceinline__ void mlp_phase(f32x16 (&accM)[2][NJ], const f32x16 (&bt)[NJ], const uint16_t* actM,
                                          const uint16_t* wf, const f32x16 (&accE)[2][NJ], uint16_t* actE, int wv,
                                          int lane, bf16x8 (&pre)[2][NJ], const uint16_t* wf_next) {
  const int fr = lane & 31, fk = (lane >> 5) * 8;
  constexpr int NT = MWID / 32;   // column tiles of a layer
  // weight fragments through a buffer resource over this layer's fragments
  // (out of range reads return zero): the lane's byte offset in a VGPR, the
  // k-step's in the scalar offset, so the unrolled k-steps need no 64-bit
  // address registers of their own (dword 3: 32-bit data format)
  const __amdgpu_buffer_rsrc_t W = __builtin_amdgcn_make_buffer_rsrc((void*)wf, (short)0, NT * 64 * 16 * KS, 0x00020000);
  const int wlane = ((NJ * wv) * 64 + lane) * 16;
  auto ldw = [&](int off) { return __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(W, wlane, off, 0)); };
  const uint16_t* arow = actM + fr * APITCH + fk;
  bf16x8 b[3][NJ], af[2][2];
  float gv[4];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {   // the first two k-steps' weights came with the phase before
    b[0][j] = pre[0][j];
    b[1][j] = pre[1][j];
  }
  af[0][0] = *(const bf16x8*)arow;
  af[0][1] = *(const bf16x8*)(arow + 32 * APITCH);
  static_for<0, KS>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    if constexpr (c + 2 < KS) {   // weights two k-steps ahead
#pragma unroll
      for (int j = 0; j < NJ; ++j) b[(c + 2) % 3][j] = ldw(((c + 2) * NT * 64 + j * 64) * 16);
    }
    if constexpr (c + 1 < KS) {   // next k-step's activations in flight
      af[(c + 1) & 1][0] = *(const bf16x8*)(arow + (c + 1) * 16);
      af[(c + 1) & 1][1] = *(const bf16x8*)(arow + 32 * APITCH + (c + 1) * 16);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const bf16x8 x = af[c & 1][i];
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const f32x16 c0 = c == 0 ? bt[j] : accM[i][j];
        if (TR)
          accM[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[c % 3][j], x, c0, 0, 0, 0);
        else
          accM[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, b[c % 3][j], c0, 0, 0, 0);
      }
    }
    if constexpr (DRAIN) epi_values<NJ, c * (32 * NJ / KS), 32 * NJ / KS>(accE, gv, actE, wv, lane);
  });
  if constexpr (NKS > 0) mlp_pre<NJ, NKS>(pre, wf_next, wv, lane);
}

// column tiles per wave: 1 (16 waves, at most 128 VGPRs each) ran the
// network in 178-182 us per 65 536 rows, 2 (8 waves with twice the
// accumulators) in 190, both before the cross-barrier weight loads
constexpr int FWD_NJ = 1, FWD_THREADS = 64 * (MWID / 32) / FWD_NJ;
__global__ __launch_bounds__(FWD_THREADS) void k_mlp_fwd(MlpArgs a) {
  constexpr int NJ = FWD_NJ;
  __shared__ __attribute__((aligned(16))) uint16_t act[MR * APITCH];
  const int tid = (int)threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r0 = (int)blockIdx.x * MR;
  // inputs normalised as k_prep_x does; padding columns and rows are zero
  for (int e = tid; e < MR * KPAD; e += FWD_THREADS) {
    const int r = e / KPAD, j = e % KPAD;
    float v = 0.0f;
    if (j < a.nin && r0 + r < a.m)
      v = 2.0f * (a.x[(int64_t)(r0 + r) * a.nin + j] - a.lo[j]) / (a.hi[j] - a.lo[j]) - 1.0f;
    act[r * APITCH + j] = f2bf(v);
  }
  __syncthreads();
  const int fr = lane & 31, fh = lane >> 5;
  uint16_t* const actA = act;
  uint16_t* const actB = act + 64 * APITCH;
  auto bias_of = [&](int l) { return a.w + a.L.off[l] + (int64_t)a.L.out[l] * a.L.in[l]; };
  // hidden-layer bias tiles: accumulator v of lane l is column
  // 8 (v / 4) + 4 (l / 32) + v % 4 of the (column, row) tile
  auto bias_tr = [&](int l, f32x16 (&bt)[NJ]) {
    const float* bias = bias_of(l);
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const float4 bv = *(const float4*)(bias + (NJ * wv + j) * 32 + 8 * g + 4 * fh);
        bt[j][4 * g + 0] = bv.x;
        bt[j][4 * g + 1] = bv.y;
        bt[j][4 * g + 2] = bv.z;
        bt[j][4 * g + 3] = bv.w;
      }
  };
  // output-layer bias tiles: column l % 32 of the (row, column) tile
  auto bias_out = [&](f32x16 (&bt)[NJ]) {
    const float* bias = bias_of(a.L.nl - 1);
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const float bj = bias[(NJ * wv + j) * 32 + fr];
#pragma unroll
      for (int v = 0; v < 16; ++v) bt[j][v] = bj;
    }
  };
  auto wf_of = [&](int l) { return a.wf + a.L.woff[l]; };
  const int nl = a.L.nl;
  f32x16 accA[2][NJ], accB[2][NJ];
  constexpr int K0 = KPAD / 16, KH = MWID / 16;
  // phase 2l: half A's products of layer l beside half B's epilogue of
  // layer l - 1; phase 2l + 1: half B's products of layer l beside half A's
  // epilogue of layer l.  A barrier ends every phase: the rows a phase
  // drains into were read by the products of the phase before, and the rows
  // it multiplies were drained into by the phase before.
  bf16x8 pre[2][NJ];
  mlp_pre<NJ, K0>(pre, wf_of(0), wv, lane);
  {
    f32x16 bt[NJ];
    bias_tr(0, bt);
    mlp_phase<NJ, true, K0, false, K0>(accA, bt, actA, wf_of(0), accB, actB, wv, lane, pre, wf_of(0));
    __syncthreads();
    bias_tr(0, bt);
    mlp_phase<NJ, true, K0, true, KH>(accB, bt, actB, wf_of(0), accA, actA, wv, lane, pre, wf_of(1));
    __syncthreads();
  }
  for (int l = 1; l + 1 < nl; ++l) {
    {
      f32x16 bt[NJ];
      bias_tr(l, bt);
      mlp_phase<NJ, true, KH, true, KH>(accA, bt, actA, wf_of(l), accB, actB, wv, lane, pre, wf_of(l));
    }
    __syncthreads();
    {
      f32x16 bt[NJ];
      bias_tr(l, bt);
      mlp_phase<NJ, true, KH, true, KH>(accB, bt, actB, wf_of(l), accA, actA, wv, lane, pre, wf_of(l + 1));
    }
    __syncthreads();
  }
  {
    f32x16 bt[NJ];
    bias_out(bt);
    mlp_phase<NJ, false, KH, true, KH>(accA, bt, actA, wf_of(nl - 1), accB, actB, wv, lane, pre, wf_of(nl - 1));
    __syncthreads();
    bias_out(bt);
    mlp_phase<NJ, false, KH, false, 0>(accB, bt, actB, wf_of(nl - 1), accA, actA, wv, lane, pre, wf_of(nl - 1));
  }
  const bool full = r0 + MR <= a.m;   // uniform: only the last workgroup may be ragged
  auto store = [&](const f32x16 (&acc)[2][NJ], int rb, auto checked) {
    float* yb = a.y + (int64_t)(r0 + rb) * MWID;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int col = (NJ * wv + j) * 32 + fr;
      const float mj = a.mu[col], sj = a.sigma[col];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int row = i * 32 + (v >> 2) * 8 + fh * 4 + (v & 3);
          if (!decltype(checked)::value || r0 + rb + row < a.m) yb[row * MWID + col] = fmaf(sj, acc[i][j][v], mj);
        }
    }
  };
  if (full) {
    store(accA, 0, std::false_type{});
    store(accB, 64, std::false_type{});
  } else {
    store(accA, 0, std::true_type{});
    store(accB, 64, std::true_type{});
  }
}

}  // namespace sur

using namespace sur;

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

struct lbm_sur_ctx {
  lbm_sur_config cfg;
  hipStream_t stream;
  std::string err;
  LayerMap L;
  int64_t np, nwb;
  // device regions
  float *w, *m1, *m2, *g, *lo, *hi, *mu, *sigma, *Y, *Tn;
  float* cpart;         // partial column sums of the bias gradients
  float* wpart;         // partial weight gradients of a depth-split product
  uint16_t *wb, *wf, *X0, *dz[2];
  int64_t wgen, fgen;   // weight updates so far; the update wf was last built from
  uint16_t* H[8];
  float* Z[8];
  double* loss;
  int* errw;            // device error word (bit 0: index out of range)
  int64_t step;
  // timing
  bool timing;
  std::vector<hipEvent_t> ev;
  int nev;
  int64_t launches;
  double flops, ms;
};

namespace {

lbm_status fail(lbm_sur_ctx* c, lbm_status s, const std::string& m) {
  if (c) c->err = m;
  return s;
}

// allocation-free inference: the static fragment buffer's address per device
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};
thread_local std::string g_static_err;   // last failure of a context-free call

#define SURCHK(c, x)                                                               \
  do {                                                                             \
    hipError_t e_ = (x);                                                           \
    if (e_ != hipSuccess) return fail(c, LBM_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

bool valid_cfg(const lbm_sur_config* c) {
  return c && c->n_in >= 1 && c->n_in <= KPAD && c->width >= 32 && c->width % 32 == 0 && c->n_hidden >= 1 &&
         c->n_hidden <= 7 && c->n_out >= 32 && c->n_out % 32 == 0 && c->max_batch >= 1 && c->train_batch >= 8 &&
         c->train_batch % 8 == 0 && c->max_batch <= (1 << 22) && c->train_batch <= (1 << 20);
}

LayerMap layer_map(const lbm_sur_config& c, int64_t& np, int64_t& nwb) {
  LayerMap L;
  std::memset(&L, 0, sizeof L);
  L.nl = c.n_hidden + 1;
  np = 0;
  nwb = 0;
  for (int l = 0; l < L.nl; ++l) {
    L.in[l] = l == 0 ? c.n_in : c.width;
    L.out[l] = l == L.nl - 1 ? c.n_out : c.width;
    L.kp[l] = l == 0 ? KPAD : c.width;
    L.off[l] = np;
    L.woff[l] = nwb;
    np += (int64_t)L.out[l] * L.in[l] + L.out[l];
    nwb += (int64_t)L.out[l] * L.kp[l];
  }
  return L;
}

struct Plan {
  size_t w, m1, m2, g, wb, wf, lo, hi, mu, sigma, X0, H[8], Z[8], Y, Tn, dz[2], cpart, wpart, loss, errw, total;
};

// depth split of a weight-gradient product over the batch rows: one slice
// per 256 rows, at most 16 (a product of 512 x 512 outputs has only 16 tiles)
int wgrad_split(int K) { return std::min(16, std::max(1, K / 256)); }
// depth split of a backward data product (depth 512) of few rows, whose few
// workgroups would each walk all 8 k-steps
constexpr int BWD_SPLIT = 4, BWD_SPLIT_ROWS = 1024;
int bwd_split(int M) { return M <= BWD_SPLIT_ROWS ? BWD_SPLIT : 1; }

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

Plan plan(const lbm_sur_config& c) {
  int64_t np, nwb;
  layer_map(c, np, nwb);
  Plan p;
  std::memset(&p, 0, sizeof p);
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = al(o + bytes); return r; };
  const size_t rows_inf = (size_t)c.max_batch, rows_tr = (size_t)c.train_batch;
  const size_t rows = rows_inf > rows_tr ? rows_inf : rows_tr;
  p.w = take(np * 4);
  p.m1 = take(np * 4);
  p.m2 = take(np * 4);
  p.g = take(np * 4);
  p.wb = take(nwb * 2);
  p.wf = take(nwb * 2);
  p.lo = take(KPAD * 4);
  p.hi = take(KPAD * 4);
  p.mu = take((size_t)c.n_out * 4);
  p.sigma = take((size_t)c.n_out * 4);
  p.X0 = take(rows * KPAD * 2);
  // hidden activations: every layer's for training, a ping-pong pair for
  // inference
  for (int l = 0; l < c.n_hidden; ++l) {
    const size_t r = l < 2 ? rows : rows_tr;
    p.H[l] = take(r * (size_t)c.width * 2);
  }
  for (int l = 0; l < c.n_hidden; ++l) p.Z[l] = take(rows_tr * (size_t)c.width * 4);
  p.Y = take(rows_tr * (size_t)c.n_out * 4);
  p.Tn = take(rows_tr * (size_t)c.n_out * 4);
  const size_t wmax = (size_t)(c.width > c.n_out ? c.width : c.n_out);
  p.dz[0] = take(rows_tr * wmax * 2);
  p.dz[1] = take(rows_tr * wmax * 2);
  p.cpart = take((rows_tr + CROWS - 1) / CROWS * wmax * 4);
  {
    // partial products of a depth split: weight gradients (nout x nin) or
    // backward data products (rows x width)
    const int s = wgrad_split((int)((rows_tr + 7) / 8 * 8));
    const size_t win = (size_t)(c.width > KPAD ? c.width : KPAD);
    const size_t wg = s > 1 ? (size_t)s * wmax * win : 0;
    const size_t bw = (size_t)BWD_SPLIT * std::min(rows_tr, (size_t)BWD_SPLIT_ROWS) * (size_t)c.width;
    p.wpart = take((wg > bw ? wg : bw) * 4);
  }
  p.loss = take(8);
  p.errw = take(4);
  p.total = o;
  return p;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

template <bool AKC, bool BKC, int EPI>
lbm_status gemm(lbm_sur_ctx* c, const GemmArgs& a) {
  // the tile loaders read 16-byte chunks: rows and depth in multiples of 8
  if (a.K % 8 || a.lda % 8 || a.ldb % 8 || !aligned16(a.A) || !aligned16(a.B) || (!AKC && a.a_ext % 8) ||
      (!BKC && a.b_ext % 8) || a.M <= 0 || a.N <= 0)
    return fail(c, LBM_E_INVAL, "matrix product shape or alignment not supported");
  const bool t = c->timing && c->nev + 2 <= (int)c->ev.size();
  if (t) SURCHK(c, hipEventRecord(c->ev[c->nev], c->stream));
  // forward products of few rows take the 128 x 128 tiles: twice the
  // workgroups, half the epilogue each (a latency-bound chain either way)
  constexpr bool fwd_form = AKC && BKC && (EPI == EPI_FWD_GELU || EPI == EPI_FWD_OUT);
  bool use_fwd = false;
  if constexpr (fwd_form) use_fwd = a.M > FWD_SMALL_M;
  if (use_fwd) {
    if constexpr (fwd_form) {
      dim3 grid((a.N + FBN - 1) / FBN, (a.M + FBM - 1) / FBM);
      hipLaunchKernelGGL((k_gemm_fwd<EPI>), grid, dim3(256), 0, c->stream, a);
    }
  } else {
    GemmArgs b = a;
    b.ksplit = EPI == EPI_WGRAD ? wgrad_split(a.K) : EPI == EPI_BWD_GELU ? bwd_split(a.M) : 1;
    b.part = c->wpart;
    dim3 grid((a.N + BN - 1) / BN, (a.M + BM - 1) / BM, b.ksplit);
    hipLaunchKernelGGL((k_gemm<AKC, BKC, EPI>), grid, dim3(256), 0, c->stream, b);
    SURCHK(c, hipGetLastError());
    const dim3 eg((unsigned)(((int64_t)a.M * a.N + 255) / 256));
    if (b.ksplit > 1 && EPI == EPI_WGRAD)
      hipLaunchKernelGGL(k_sum_parts, eg, dim3(256), 0, c->stream, c->wpart, b.ksplit, a.M, a.N, a.outf, a.ldo);
    if (b.ksplit > 1 && EPI == EPI_BWD_GELU)
      hipLaunchKernelGGL(k_sum_parts_bwd, eg, dim3(256), 0, c->stream, c->wpart, b.ksplit, a.M, a.N, a.zin, a.outh,
                         a.ldo);
  }
  SURCHK(c, hipGetLastError());
  if (t) {
    SURCHK(c, hipEventRecord(c->ev[c->nev + 1], c->stream));
    c->nev += 2;
    c->flops += 2.0 * a.M * (double)a.N * a.K;
  }
  return LBM_OK;
}

#define TRY(x)                      \
  do {                              \
    lbm_status s_ = (x);            \
    if (s_ != LBM_OK) return s_;    \
  } while (0)

unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// forward pass over m rows from X0; training keeps Z and every H, inference
// ping-pongs two H buffers and writes physical outputs to y
lbm_status forward(lbm_sur_ctx* c, int m, bool train, float* y) {
  const lbm_sur_config& C = c->cfg;
  const uint16_t* in = c->X0;
  int64_t ldin = KPAD;
  for (int l = 0; l < C.n_hidden; ++l) {
    GemmArgs a;
    std::memset(&a, 0, sizeof a);
    uint16_t* out = train ? c->H[l] : c->H[l & 1];
    a.A = in; a.lda = ldin; a.a_ext = m;
    a.B = c->wb + c->L.woff[l]; a.ldb = c->L.kp[l]; a.b_ext = C.width;
    a.M = m; a.N = C.width; a.K = (int)ldin;
    a.bias = c->w + c->L.off[l] + (int64_t)c->L.out[l] * c->L.in[l];
    a.outh = out; a.zout = train ? c->Z[l] : nullptr; a.ldo = C.width;
    TRY((gemm<true, true, EPI_FWD_GELU>(c, a)));
    in = out;
    ldin = C.width;
  }
  const int l = C.n_hidden;
  GemmArgs a;
  std::memset(&a, 0, sizeof a);
  a.A = in; a.lda = ldin; a.a_ext = m;
  a.B = c->wb + c->L.woff[l]; a.ldb = c->L.kp[l]; a.b_ext = C.n_out;
  a.M = m; a.N = C.n_out; a.K = (int)ldin;
  a.bias = c->w + c->L.off[l] + (int64_t)c->L.out[l] * c->L.in[l];
  a.outf = train ? c->Y : y; a.ldo = C.n_out;
  a.mu = train ? nullptr : c->mu;
  a.sigma = train ? nullptr : c->sigma;
  return gemm<true, true, EPI_FWD_OUT>(c, a);
}

lbm_status check_batch(lbm_sur_ctx* c, const float* x, int m, int limit) {
  if (!x || ((uintptr_t)x & 3)) return fail(c, LBM_E_INVAL, "input rows must be a 4-byte aligned device pointer");
  if (m < 1 || m > limit) return fail(c, LBM_E_INVAL, "row count outside [1, configured batch]");
  return LBM_OK;
}

// forward, loss and backward into c->g; the loss lands in c->loss
lbm_status grad_pass(lbm_sur_ctx* c, const float* x, const float* t, int nrows, const int32_t* idx, int m) {
  const lbm_sur_config& C = c->cfg;
  TRY(check_batch(c, x, m, C.train_batch));
  if (!t || ((uintptr_t)t & 3)) return fail(c, LBM_E_INVAL, "targets must be a 4-byte aligned device pointer");
  if (nrows < 1 || (!idx && nrows < m)) return fail(c, LBM_E_INVAL, "fewer data rows than batch rows");
  // the weight-gradient product reduces over the rows in chunks of 8: pad
  // the batch's activations with zero rows up to a multiple of 8
  const int mp = (m + 7) / 8 * 8;
  hipLaunchKernelGGL(k_prep_x, dim3(blocks((int64_t)mp * KPAD, 256)), dim3(256), 0, c->stream, x, nrows, idx, m,
                     mp, C.n_in, c->lo, c->hi, c->X0, c->errw);
  SURCHK(c, hipGetLastError());
  hipLaunchKernelGGL(k_prep_t, dim3(blocks((int64_t)m * C.n_out, 256)), dim3(256), 0, c->stream, t, nrows, idx, m,
                     C.n_out, c->mu, c->sigma, c->Tn);
  SURCHK(c, hipGetLastError());
  TRY(forward(c, m, true, nullptr));
  SURCHK(c, hipMemsetAsync(c->loss, 0, 8, c->stream));
  hipLaunchKernelGGL(k_loss, dim3(std::min(blocks((int64_t)m * C.n_out, 256), 512u)), dim3(256), 0, c->stream, c->Y, c->Tn,
                     (int64_t)m * C.n_out, c->dz[0], c->loss);
  SURCHK(c, hipGetLastError());
  int cur = 0;
  for (int l = C.n_hidden; l >= 0; --l) {
    const int nout = c->L.out[l], nin = c->L.in[l];
    const uint16_t* hin = l == 0 ? c->X0 : c->H[l - 1];
    const int64_t ldh = l == 0 ? KPAD : C.width;
    // dW_l = dz^T h_{l-1}: (nout x m) (m x nin), reduction over the rows
    GemmArgs a;
    std::memset(&a, 0, sizeof a);
    a.A = c->dz[cur]; a.lda = nout; a.a_ext = nout;
    a.B = hin; a.ldb = ldh; a.b_ext = (int)ldh;
    a.M = nout; a.N = nin; a.K = mp;
    a.outf = c->g + c->L.off[l]; a.ldo = nin;
    TRY((gemm<false, false, EPI_WGRAD>(c, a)));
    const int nchunk = (m + CROWS - 1) / CROWS;
    hipLaunchKernelGGL(k_colsum_part, dim3(blocks(nout, 256), nchunk), dim3(256), 0, c->stream, c->dz[cur], m, nout,
                       c->cpart);
    SURCHK(c, hipGetLastError());
    hipLaunchKernelGGL(k_colsum_fin, dim3(blocks(nout, 256)), dim3(256), 0, c->stream, c->cpart, nchunk, nout,
                       c->g + c->L.off[l] + (int64_t)nout * nin);
    SURCHK(c, hipGetLastError());
    if (l == 0) break;
    // dz_{l-1} = (dz W_l) * GELU'(z_{l-1}): (m x nout) (nout x nin)
    std::memset(&a, 0, sizeof a);
    a.A = c->dz[cur]; a.lda = nout; a.a_ext = m;
    a.B = c->wb + c->L.woff[l]; a.ldb = c->L.kp[l]; a.b_ext = nin;
    a.M = m; a.N = nin; a.K = nout;
    a.zin = c->Z[l - 1]; a.outh = c->dz[cur ^ 1]; a.ldo = nin;
    TRY((gemm<true, false, EPI_BWD_GELU>(c, a)));
    cur ^= 1;
  }
  return LBM_OK;
}

// rows m..mp of the padded batch must be zero in every operand of the
// weight-gradient product: dz (loss gradient and backward products) and h
lbm_status zero_tail(lbm_sur_ctx* c, int m) {
  const lbm_sur_config& C = c->cfg;
  const int mp = (m + 7) / 8 * 8;
  if (mp == m) return LBM_OK;
  // dz holds rows of pitch n_out (loss gradient) or width (backward
  // products): clear from the smaller pitch's row m to the larger's row mp
  const size_t wmax = (size_t)(C.width > C.n_out ? C.width : C.n_out);
  const size_t wmin = (size_t)(C.width < C.n_out ? C.width : C.n_out);
  for (int k = 0; k < 2; ++k)
    SURCHK(c, hipMemsetAsync(c->dz[k] + (size_t)m * wmin, 0, ((size_t)mp * wmax - (size_t)m * wmin) * 2, c->stream));
  for (int l = 0; l < C.n_hidden; ++l)
    SURCHK(c, hipMemsetAsync(c->H[l] + (size_t)m * C.width, 0, (size_t)(mp - m) * C.width * 2, c->stream));
  return LBM_OK;
}

}  // namespace

extern "C" lbm_status lbm_sur_sync(lbm_sur_ctx* c);

namespace {
lbm_status read_loss(lbm_sur_ctx* c, double* loss) {
  TRY(lbm_sur_sync(c));
  SURCHK(c, hipMemcpy(loss, c->loss, 8, hipMemcpyDeviceToHost));
  return LBM_OK;
}
// the whole network in one kernel (k_mlp_fwd) when the hidden width and
// the output count are 512
bool fused_shape(const lbm_sur_config& C) { return C.width == MWID && C.n_out == MWID; }

lbm_status predict_fused(lbm_sur_ctx* c, const float* x, int m, float* y) {
  if (c->fgen != c->wgen) {   // weights changed: rebuild the fragment-order copy
    hipLaunchKernelGGL(k_frag, dim3(blocks(c->nwb, 256)), dim3(256), 0, c->stream, c->wb, c->L, c->nwb, c->wf);
    SURCHK(c, hipGetLastError());
    c->fgen = c->wgen;
  }
  MlpArgs g;
  g.x = x; g.m = m; g.nin = c->cfg.n_in; g.lo = c->lo; g.hi = c->hi;
  g.wf = c->wf; g.w = c->w; g.L = c->L; g.mu = c->mu; g.sigma = c->sigma; g.y = y;
  const bool t = c->timing && c->nev + 2 <= (int)c->ev.size();
  if (t) SURCHK(c, hipEventRecord(c->ev[c->nev], c->stream));
  hipLaunchKernelGGL(k_mlp_fwd, dim3(blocks(m, MR)), dim3(FWD_THREADS), 0, c->stream, g);
  SURCHK(c, hipGetLastError());
  if (t) {
    SURCHK(c, hipEventRecord(c->ev[c->nev + 1], c->stream));
    c->nev += 2;
    for (int l = 0; l < c->L.nl; ++l) c->flops += 2.0 * m * (double)c->L.out[l] * c->L.kp[l];
  }
  return LBM_OK;
}

}  // namespace

extern "C" {

int64_t lbm_sur_num_params(const lbm_sur_config* cfg) {
  if (!valid_cfg(cfg)) return -1;
  int64_t np, nwb;
  layer_map(*cfg, np, nwb);
  return np;
}

lbm_status lbm_sur_query_sizes(const lbm_sur_config* cfg, size_t* bytes) {
  if (!valid_cfg(cfg) || !bytes) return LBM_E_INVAL;
  *bytes = plan(*cfg).total;
  return LBM_OK;
}

lbm_status lbm_sur_init(const lbm_sur_config* cfg, void* mem, size_t bytes, void* stream, lbm_sur_ctx** out) {
  if (!out) return LBM_E_INVAL;
  *out = nullptr;
  if (!valid_cfg(cfg) || !mem || ((uintptr_t)mem & 255)) return LBM_E_INVAL;
  const Plan p = plan(*cfg);
  if (bytes < p.total) return LBM_E_INVAL;
  lbm_sur_ctx* c = new lbm_sur_ctx();
  c->cfg = *cfg;
  c->stream = (hipStream_t)stream;
  c->L = layer_map(*cfg, c->np, c->nwb);
  char* b = (char*)mem;
  c->w = (float*)(b + p.w); c->m1 = (float*)(b + p.m1); c->m2 = (float*)(b + p.m2); c->g = (float*)(b + p.g);
  c->wb = (uint16_t*)(b + p.wb);
  c->wf = (uint16_t*)(b + p.wf);
  c->wgen = 0;
  c->fgen = -1;
  c->lo = (float*)(b + p.lo); c->hi = (float*)(b + p.hi); c->mu = (float*)(b + p.mu); c->sigma = (float*)(b + p.sigma);
  c->X0 = (uint16_t*)(b + p.X0);
  for (int l = 0; l < cfg->n_hidden; ++l) {
    c->H[l] = (uint16_t*)(b + p.H[l]);
    c->Z[l] = (float*)(b + p.Z[l]);
  }
  c->Y = (float*)(b + p.Y); c->Tn = (float*)(b + p.Tn);
  c->dz[0] = (uint16_t*)(b + p.dz[0]); c->dz[1] = (uint16_t*)(b + p.dz[1]);
  c->cpart = (float*)(b + p.cpart);
  c->wpart = (float*)(b + p.wpart);
  c->loss = (double*)(b + p.loss);
  c->errw = (int*)(b + p.errw);
  c->step = 0;
  c->timing = false;
  c->nev = 0;
  c->launches = 0;
  c->flops = c->ms = 0.0;
  // zero everything once (padding columns of the BF16 weights and of X0,
  // Adam moments, scaling); synchronous so the context is ready on return
  hipError_t e = hipMemsetAsync(mem, 0, p.total, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    delete c;
    return LBM_E_DEVICE;
  }
  *out = c;
  return LBM_OK;
}

lbm_status lbm_sur_set_params(lbm_sur_ctx* c, const double* theta, int64_t n) {
  if (!c || !theta) return LBM_E_INVAL;
  if (n != c->np) return fail(c, LBM_E_INVAL, "parameter count does not match the network");
  std::vector<float> h(n);
  for (int64_t k = 0; k < n; ++k) h[k] = (float)theta[k];
  SURCHK(c, hipStreamSynchronize(c->stream));
  SURCHK(c, hipMemcpy(c->w, h.data(), n * 4, hipMemcpyHostToDevice));
  SURCHK(c, hipMemsetAsync(c->m1, 0, n * 4, c->stream));
  SURCHK(c, hipMemsetAsync(c->m2, 0, n * 4, c->stream));
  hipLaunchKernelGGL(k_cast, dim3(blocks(n, 256)), dim3(256), 0, c->stream, c->w, n, c->L, c->wb);
  SURCHK(c, hipGetLastError());
  SURCHK(c, hipStreamSynchronize(c->stream));
  c->step = 0;
  c->wgen += 1;
  return LBM_OK;
}

lbm_status lbm_sur_get_params(lbm_sur_ctx* c, double* theta, int64_t n) {
  if (!c || !theta) return LBM_E_INVAL;
  if (n != c->np) return fail(c, LBM_E_INVAL, "parameter count does not match the network");
  std::vector<float> h(n);
  SURCHK(c, hipStreamSynchronize(c->stream));
  SURCHK(c, hipMemcpy(h.data(), c->w, n * 4, hipMemcpyDeviceToHost));
  for (int64_t k = 0; k < n; ++k) theta[k] = h[k];
  return LBM_OK;
}

lbm_status lbm_sur_set_scaling(lbm_sur_ctx* c, const double* lo, const double* hi, const double* mu,
                               const double* sigma) {
  if (!c || !lo || !hi || !mu || !sigma) return LBM_E_INVAL;
  const lbm_sur_config& C = c->cfg;
  std::vector<float> a(KPAD, 0.0f), b(KPAD, 1.0f), m(C.n_out), s(C.n_out);
  for (int j = 0; j < C.n_in; ++j) {
    if (!(hi[j] > lo[j])) return fail(c, LBM_E_INVAL, "input box needs lo < hi");
    a[j] = (float)lo[j];
    b[j] = (float)hi[j];
  }
  for (int j = 0; j < C.n_out; ++j) {
    if (!(sigma[j] > 0)) return fail(c, LBM_E_INVAL, "output scales must be positive");
    m[j] = (float)mu[j];
    s[j] = (float)sigma[j];
  }
  SURCHK(c, hipStreamSynchronize(c->stream));
  SURCHK(c, hipMemcpy(c->lo, a.data(), KPAD * 4, hipMemcpyHostToDevice));
  SURCHK(c, hipMemcpy(c->hi, b.data(), KPAD * 4, hipMemcpyHostToDevice));
  SURCHK(c, hipMemcpy(c->mu, m.data(), C.n_out * 4, hipMemcpyHostToDevice));
  SURCHK(c, hipMemcpy(c->sigma, s.data(), C.n_out * 4, hipMemcpyHostToDevice));
  return LBM_OK;
}

lbm_status lbm_sur_grad(lbm_sur_ctx* c, const float* x, const float* t, int32_t n_rows, const int32_t* idx,
                        int32_t m, float* grad, double* loss) {
  if (!c || !grad) return LBM_E_INVAL;
  if (m < 1 || m > c->cfg.train_batch) return fail(c, LBM_E_INVAL, "row count outside [1, training batch]");
  TRY(zero_tail(c, m));
  TRY(grad_pass(c, x, t, n_rows, idx, m));
  SURCHK(c, hipMemcpyAsync(grad, c->g, c->np * 4, hipMemcpyDeviceToDevice, c->stream));
  if (loss) TRY(read_loss(c, loss));
  return LBM_OK;
}

lbm_status lbm_sur_train_step(lbm_sur_ctx* c, const float* x, const float* t, int32_t n_rows,
                              const int32_t* idx, int32_t m, double lr, double b1, double b2, double eps,
                              double* loss) {
  if (!c) return LBM_E_INVAL;
  if (!(lr >= 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0))
    return fail(c, LBM_E_INVAL, "Adam needs lr >= 0, 0 <= b1, b2 < 1, eps > 0");
  if (m < 1 || m > c->cfg.train_batch) return fail(c, LBM_E_INVAL, "row count outside [1, training batch]");
  TRY(zero_tail(c, m));
  TRY(grad_pass(c, x, t, n_rows, idx, m));
  c->step += 1;
  const float bc1 = (float)(1.0 - std::pow(b1, (double)c->step));
  const float bc2 = (float)(1.0 - std::pow(b2, (double)c->step));
  hipLaunchKernelGGL(k_adam, dim3(blocks(c->np, 256)), dim3(256), 0, c->stream, c->w, c->m1, c->m2, c->g, c->np,
                     (float)lr, (float)b1, (float)b2, (float)eps, bc1, bc2, c->L, c->wb);
  SURCHK(c, hipGetLastError());
  c->wgen += 1;
  if (loss) TRY(read_loss(c, loss));
  return LBM_OK;
}

lbm_status lbm_sur_predict(lbm_sur_ctx* c, const float* x, int32_t m, float* y) {
  if (!c || !y) return LBM_E_INVAL;
  TRY(check_batch(c, x, m, c->cfg.max_batch));
  if (fused_shape(c->cfg)) return predict_fused(c, x, m, y);
  hipLaunchKernelGGL(k_prep_x, dim3(blocks((int64_t)m * KPAD, 256)), dim3(256), 0, c->stream, x, m, nullptr, m, m,
                     c->cfg.n_in, c->lo, c->hi, c->X0, c->errw);
  SURCHK(c, hipGetLastError());
  return forward(c, m, false, y);
}

lbm_status lbm_sur_set_timing(lbm_sur_ctx* c, int32_t on) {
  if (!c) return LBM_E_INVAL;
  SURCHK(c, hipStreamSynchronize(c->stream));
  if (on && c->ev.empty()) {
    c->ev.resize(2048);
    for (auto& e : c->ev) SURCHK(c, hipEventCreate(&e));
  }
  c->timing = on != 0;
  c->nev = 0;
  c->launches = 0;
  c->flops = c->ms = 0.0;
  return LBM_OK;
}

lbm_status lbm_sur_gemm_time(lbm_sur_ctx* c, int64_t* launches, double* ms, double* flops) {
  if (!c || !launches || !ms || !flops) return LBM_E_INVAL;
  SURCHK(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k + 1 < c->nev; k += 2) {
    float t = 0.0f;
    SURCHK(c, hipEventElapsedTime(&t, c->ev[k], c->ev[k + 1]));
    c->ms += t;
    c->launches += 1;
  }
  c->nev = 0;
  *launches = c->launches;
  *ms = c->ms;
  *flops = c->flops;
  return LBM_OK;
}

lbm_status lbm_sur_sync(lbm_sur_ctx* c) {
  if (!c) return LBM_E_INVAL;
  SURCHK(c, hipStreamSynchronize(c->stream));
  int e = 0;
  SURCHK(c, hipMemcpy(&e, c->errw, 4, hipMemcpyDeviceToHost));
  if (e) {
    SURCHK(c, hipMemset(c->errw, 0, 4));
    return fail(c, LBM_E_INVAL, "a batch index was outside [0, n_rows)");
  }
  return LBM_OK;
}

const char* lbm_sur_last_error(const lbm_sur_ctx* c) {
  return c ? c->err.c_str() : (g_static_err.empty() ? "null context" : g_static_err.c_str());
}

lbm_status lbm_sur_predict_static(const lbm_sur_config* cfg, const float* theta, const float* lo, const float* hi,
                                  const float* mu, const float* sigma, const float* x, int32_t m, float* y,
                                  void* stream) {
  auto bad = [](lbm_status st, const char* msg) {
    g_static_err = msg;
    return st;
  };
  if (!cfg || !theta || !lo || !hi || !mu || !sigma || !x || !y) return bad(LBM_E_INVAL, "NULL argument");
  for (const void* q : {(const void*)theta, (const void*)lo, (const void*)hi, (const void*)mu, (const void*)sigma,
                        (const void*)x, (const void*)y})
    if ((uintptr_t)q & 3) return bad(LBM_E_INVAL, "device arrays must be 4-byte aligned");
  if (cfg->n_in < 1 || cfg->n_in > KPAD || cfg->width != MWID || cfg->n_out != MWID || cfg->n_hidden < 1 ||
      cfg->n_hidden > 7)
    return bad(LBM_E_INVAL, "allocation-free inference takes n_in <= 32, width 512, 1..7 hidden layers, 512 outputs");
  if (m < 0 || m > (1 << 22)) return bad(LBM_E_INVAL, "row count outside [0, 2^22]");
  int64_t np = 0, nwb = 0;
  const LayerMap L = layer_map(*cfg, np, nwb);
  if (nwb > NOALLOC_WEIGHTS) return bad(LBM_E_INVAL, "network larger than the static fragment buffer");
  if (m == 0) return LBM_OK;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES)
    return bad(LBM_E_DEVICE, "no current device");
  uint16_t* wf = nullptr;
  {
    // the array's device address on this GPU, looked up once per device
    // (with that device current); host code never uses the symbol itself
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void* ptr = nullptr;
      if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
        return bad(LBM_E_DEVICE, "hipGetSymbolAddress of the static fragment buffer failed");
      g_scratch_ptr[dev] = ptr;
    }
    wf = (uint16_t*)g_scratch_ptr[dev];
  }
  hipStream_t s = (hipStream_t)stream;
  // every call rebuilds the fragments from the caller's parameters, so the
  // buffer holds nothing that must start at zero
  hipLaunchKernelGGL(k_frag_f32, dim3(blocks(nwb, 256)), dim3(256), 0, s, theta, L, nwb, wf);
  if (hipGetLastError() != hipSuccess) return bad(LBM_E_DEVICE, "fragment kernel launch failed");
  MlpArgs g;
  g.x = x; g.m = m; g.nin = cfg->n_in; g.lo = lo; g.hi = hi;
  g.wf = wf; g.w = theta; g.L = L; g.mu = mu; g.sigma = sigma; g.y = y;
  hipLaunchKernelGGL(k_mlp_fwd, dim3(blocks(m, MR)), dim3(FWD_THREADS), 0, s, g);
  if (hipGetLastError() != hipSuccess) return bad(LBM_E_DEVICE, "inference kernel launch failed");
  return LBM_OK;
}

lbm_status lbm_sur_destroy(lbm_sur_ctx* c) {
  if (!c) return LBM_E_INVAL;
  (void)hipStreamSynchronize(c->stream);
  for (auto& e : c->ev) (void)hipEventDestroy(e);
  delete c;
  return LBM_OK;
}

}  // extern "C"
