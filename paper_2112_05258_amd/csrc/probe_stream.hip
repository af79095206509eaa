// Practical HBM ceiling of the collide-stream access pattern: per cell, 19
// structure-of-arrays loads and 19 stores with the AA pattern's addressing
// (even step: the cell's own slots; odd step: neighbour-shifted slots), with
// next to no arithmetic.  Prints one line per case: element type, box, and
// the achieved GB/s of each parity (bytes = 2 * 19 * cells * element size).
// Measurement aid of the benchmark, not part of the method.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

namespace {

__device__ constexpr int PX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
__device__ constexpr int PY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__device__ constexpr int PZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
__device__ constexpr int PO[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};

#define CHECK(x)                                                                 \
  do {                                                                           \
    hipError_t e_ = (x);                                                         \
    if (e_ != hipSuccess) {                                                      \
      std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));              \
      std::exit(1);                                                              \
    }                                                                            \
  } while (0)

// cells [lo, hi) keep every neighbour-shifted index inside [0, NT)
template <class T, bool ODD>
__global__ __launch_bounds__(256) void k_stream(T* A, long NT, int nx, int ny, long lo, long hi) {
  const long c = lo + (long)blockIdx.x * 256 + threadIdx.x;
  if (c >= hi) return;
  const long sy = nx, sz = (long)nx * ny;
  float g[19];
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const long o = PX[i] + PY[i] * sy + PZ[i] * sz;
    g[i] = (float)(ODD ? A[PO[i] * NT + c - o] : A[i * NT + c]);
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 19; ++i) s += g[i];
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const long o = PX[i] + PY[i] * sy + PZ[i] * sz;
    const float v = g[i] * 0.999f + s * 1e-6f;
    if (ODD)
      A[i * NT + c + o] = (T)v;
    else
      A[PO[i] * NT + c] = (T)v;
  }
}

template <class T>
void run(const char* name, int nx, int ny, int nz) {
  const long NT = (long)nx * ny * nz, sz = (long)nx * ny;
  const long lo = sz + nx + 1, hi = NT - sz - nx - 1;
  T* A = nullptr;
  CHECK(hipMalloc(&A, 19 * NT * sizeof(T)));
  CHECK(hipMemset(A, 0, 19 * NT * sizeof(T)));
  const unsigned nb = (unsigned)((hi - lo + 255) / 256);
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  for (int w = 0; w < 4; ++w) {
    k_stream<T, false><<<nb, 256>>>(A, NT, nx, ny, lo, hi);
    k_stream<T, true><<<nb, 256>>>(A, NT, nx, ny, lo, hi);
  }
  CHECK(hipGetLastError());
  const int reps = 40;
  float ms[2];
  for (int odd = 0; odd < 2; ++odd) {
    CHECK(hipEventRecord(e0));
    for (int r = 0; r < reps; ++r) {
      if (odd)
        k_stream<T, true><<<nb, 256>>>(A, NT, nx, ny, lo, hi);
      else
        k_stream<T, false><<<nb, 256>>>(A, NT, nx, ny, lo, hi);
    }
    CHECK(hipEventRecord(e1));
    CHECK(hipEventSynchronize(e1));
    CHECK(hipEventElapsedTime(&ms[odd], e0, e1));
    ms[odd] /= reps;
  }
  const double bytes = 2.0 * 19 * (double)(hi - lo) * sizeof(T);
  std::printf("%s %dx%dx%d even_us %.1f even_GBs %.0f odd_us %.1f odd_GBs %.0f\n", name, nx, ny, nz, ms[0] * 1e3,
              bytes / (ms[0] * 1e-3) / 1e9, ms[1] * 1e3, bytes / (ms[1] * 1e-3) / 1e9);
  CHECK(hipEventDestroy(e0));
  CHECK(hipEventDestroy(e1));
  CHECK(hipFree(A));
}

}  // namespace

int main() {
  run<float>("fp32", 128, 128, 512);
  run<__half>("fp16", 128, 128, 512);
  run<float>("fp32", 256, 256, 512);
  run<__half>("fp16", 256, 256, 512);
  return 0;
}
