// Host code of the solver library under AddressSanitizer and
// UndefinedBehaviorSanitizer, without a GPU: the geometry checks and sizes
// (lbm_query_sizes) on a real workload's cell types, single and batched,
// with the extrapolation variants, and the rejections of bad inputs.  The
// device launchers are replaced by stubs that fail (no context is ever
// created here, so none of them is reached).
//
// Input file (written by the test): int32 nx, ny, nz, then nx*ny*nz cell-type
// bytes.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "lbm0d3d.h"
#include "lbm_internal.h"

namespace lbm {
hipError_t launch_reduce(const Dev&, int, int, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_collide(const Dev&, int, int, int, int, bool, const CTile*, int, int, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_band(const Dev&, int, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_collide_count(const Dev&, int, bool, const CTile*, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_reduce_band(const Dev&, int, int, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_wall(const Dev&, int, int, int, int, bool, const int32_t*, int, int, int, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_band_rebuild(const Dev&, int, float, const int[3], int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_wss(const Dev&, int, int, int, int64_t, double, double, double*, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_motion(const Dev&, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_membrane(const Dev&, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_fill_rest(const Dev&, int, int64_t, int64_t, double, hipStream_t) { return hipErrorNotSupported; }
}  // namespace lbm

static int fails = 0;
static void expect(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s\n", what);
    ++fails;
  }
}

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t n[3];
  if (std::fread(n, 4, 3, f) != 3) return 2;
  const size_t nc = (size_t)n[0] * n[1] * n[2];
  std::vector<uint8_t> flags(nc);
  if (std::fread(flags.data(), 1, nc, f) != nc) return 2;
  std::fclose(f);

  lbm_config c{};
  c.nx = n[0]; c.ny = n[1]; c.nz = n[2];
  c.tau = 0.6;
  c.precision = LBM_FP32;
  c.flags = flags.data();
  size_t pb = 0, wb = 0;
  for (int v = 0; v < 2; ++v)
    for (int p = 0; p < 4; ++p) {
      c.nee_variant = v;
      c.precision = p;
      expect(lbm_query_sizes(&c, 1, &pb, &wb) == LBM_OK && pb > 0 && wb > 0, "sizes of the workload");
    }
  std::vector<lbm_config> two(2, c);
  two[1].nee_variant = 0;
  expect(lbm_query_sizes(two.data(), 2, &pb, &wb) == LBM_OK, "sizes of a batch of two");

  // rejections
  lbm_config bad = c;
  bad.tau = 0.5;
  expect(lbm_query_sizes(&bad, 1, &pb, &wb) == LBM_E_INVAL, "tau 0.5 rejected");
  bad = c;
  bad.nx = 2;
  expect(lbm_query_sizes(&bad, 1, &pb, &wb) == LBM_E_INVAL, "box of 2 rejected");
  std::vector<uint8_t> face = flags;
  face[(size_t)n[0] * n[1] * (n[2] / 2)] = 0;  // a FLUID cell on a box face
  bad = c;
  bad.flags = face.data();
  expect(lbm_query_sizes(&bad, 1, &pb, &wb) == LBM_E_INVAL, "FLUID on a box face rejected");
  std::vector<uint8_t> type = flags;
  type[nc / 2] = 7;  // no such cell type
  bad.flags = type.data();
  expect(lbm_query_sizes(&bad, 1, &pb, &wb) == LBM_E_INVAL, "unknown cell type rejected");
  expect(lbm_query_sizes(nullptr, 1, &pb, &wb) == LBM_E_INVAL, "NULL configs rejected");
  expect(lbm_query_sizes(&c, 0, &pb, &wb) == LBM_E_INVAL, "zero instances rejected");
  lbm_ctx* ctx = nullptr;
  expect(lbm_init(&c, 1, nullptr, nullptr, &ctx) != LBM_OK && ctx == nullptr, "lbm_init without buffers rejected");
  std::printf("host driver: %d failure(s)\n", fails);
  return fails ? 1 : 0;
}
