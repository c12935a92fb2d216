// Host-side checks of libuot's C ABI without a GPU: argument validation,
// plan building and workspace sizing, on valid, edge and invalid inputs.
// Built with AddressSanitizer and UndefinedBehaviorSanitizer on the host code
// only (tests/test_host_sanitizer.py); every call must return the documented
// code, and the sanitizers must stay silent.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "uot.h"

static int failures = 0;
#define EXPECT(cond)                                                      \
  do {                                                                    \
    if (!(cond)) {                                                        \
      std::fprintf(stderr, "FAILED %s:%d: %s (%s)\n", __FILE__, __LINE__, #cond, uot_last_error()); \
      ++failures;                                                         \
    }                                                                     \
  } while (0)

static const void* const kDev = reinterpret_cast<const void*>(0x10000);   // never dereferenced on the host

static uot_problem points(int dtype, int dim, int64_t N, int64_t M) {
  uot_problem pb;
  std::memset(&pb, 0, sizeof(pb));
  pb.dtype = dtype;
  pb.geom.kind = UOT_GEOM_POINTS;
  pb.geom.dim = dim;
  pb.geom.N = N;
  pb.geom.M = M;
  pb.geom.x = pb.geom.y = kDev;
  pb.p = pb.q = pb.dx = pb.dy = kDev;
  pb.F1.kind = pb.F2.kind = UOT_DIV_KL;
  pb.F1.lambda = pb.F2.lambda = 1.0;
  return pb;
}

static uot_problem grid(int dtype, int dim, const int64_t* n) {
  uot_problem pb;
  std::memset(&pb, 0, sizeof(pb));
  pb.dtype = dtype;
  pb.geom.kind = UOT_GEOM_GRID;
  pb.geom.dim = dim;
  for (int k = 0; k < dim; ++k) {
    pb.geom.n[k] = n[k];
    pb.geom.h[k] = 1.0 / double(n[k]);
  }
  pb.p = pb.q = pb.dx = pb.dy = kDev;
  pb.F1.kind = pb.F2.kind = UOT_DIV_KL;
  pb.F1.lambda = pb.F2.lambda = 0.1;
  return pb;
}

int main() {
  size_t n = 0;
  EXPECT(uot_abi_version() == 3);
  for (int s = -6; s <= 2; ++s) EXPECT(uot_status_string(s) != nullptr && std::strlen(uot_status_string(s)) > 0);

  // point clouds: every dtype, dimension and a range of sizes
  for (int dt : {UOT_F32, UOT_F64})
    for (int dim = 1; dim <= 3; ++dim)
      for (int64_t N : {1LL, 2LL, 255LL, 256LL, 2048LL, 20000LL, 1LL << 20})
        for (int64_t M : {1LL, 3LL, 4096LL, 30001LL}) {
          uot_problem pb = points(dt, dim, N, M);
          EXPECT(uot_workspace_size(&pb, &n) == UOT_OK);
          EXPECT(n >= (size_t)(N + M) * (dt == UOT_F32 ? 4 : 8));
        }
  {
    uot_problem pb = points(UOT_F32, 4, 100, 100);
    EXPECT(uot_workspace_size(&pb, &n) == UOT_E_UNSUPPORTED);
    pb = points(UOT_F32, 2, 0, 100);
    EXPECT(uot_workspace_size(&pb, &n) == UOT_E_INVALID);
    pb = points(7, 2, 10, 10);
    EXPECT(uot_workspace_size(&pb, &n) == UOT_E_INVALID);
    pb = points(UOT_F32, 2, 10, 10);
    EXPECT(uot_workspace_size(&pb, nullptr) == UOT_E_INVALID);
    EXPECT(uot_workspace_size(nullptr, &n) == UOT_E_INVALID);
    pb.geom.cost = UOT_COST_WF;   // needs a cut > 0
    EXPECT(uot_workspace_size(&pb, &n) == UOT_E_INVALID);
    pb.geom.cut = 0.3;
    EXPECT(uot_workspace_size(&pb, &n) == UOT_OK);
  }
  // grids of 1 to 3 axes, fields of them
  {
    const int64_t shapes[][3] = {{1, 0, 0}, {16, 0, 0}, {3000, 0, 0}, {256, 256, 0}, {64, 48, 0}, {1, 1, 0},
                                 {64, 32, 32}, {17, 33, 5}, {128, 128, 128}};
    const int dims[] = {1, 1, 1, 2, 2, 2, 3, 3, 3};
    for (int k = 0; k < 9; ++k)
      for (int dt : {UOT_F32, UOT_F64}) {
        uot_problem pb = grid(dt, dims[k], shapes[k]);
        EXPECT(uot_workspace_size(&pb, &n) == UOT_OK);
        for (int nb : {1, 2, 256}) EXPECT(uot_fields_workspace_size(&pb, nb, &n) == UOT_OK);
        EXPECT(uot_fields_workspace_size(&pb, 0, &n) == UOT_E_INVALID);
      }
    int64_t bad[3] = {64, 0, 0};
    uot_problem pb = grid(UOT_F32, 2, bad);
    EXPECT(uot_workspace_size(&pb, &n) == UOT_E_UNSUPPORTED);   // axes of 1..4096 cells
    int64_t wide[3] = {8192, 0, 0};
    pb = grid(UOT_F32, 1, wide);
    EXPECT(uot_workspace_size(&pb, &n) == UOT_E_UNSUPPORTED);
    pb = grid(UOT_F32, 2, shapes[3]);
    pb.geom.h[1] = -1.0;
    EXPECT(uot_workspace_size(&pb, &n) == UOT_E_INVALID);
    pb = grid(UOT_F32, 2, shapes[3]);
    pb.geom.cost = UOT_COST_WF;
    pb.geom.cut = 0.5;
    EXPECT(uot_workspace_size(&pb, &n) == UOT_E_UNSUPPORTED);   // not separable beyond 1-D
  }
  // barycentres
  {
    uot_bary_problem bp;
    std::memset(&bp, 0, sizeof(bp));
    bp.dtype = UOT_F32;
    bp.n = 8;
    bp.geom.kind = UOT_GEOM_GRID;
    bp.geom.dim = 2;
    bp.geom.n[0] = bp.geom.n[1] = 128;
    bp.geom.h[0] = bp.geom.h[1] = 1.0 / 128;
    EXPECT(uot_bary_workspace_size(&bp, &n) == UOT_OK);
    bp.n = 0;
    EXPECT(uot_bary_workspace_size(&bp, &n) == UOT_E_INVALID);
  }
  // ragged batches: offsets on the host
  {
    std::vector<int64_t> offN{0}, offM{0};
    for (int b = 0; b < 4096; ++b) {
      offN.push_back(offN.back() + 64 + (b * 37) % 4033);
      offM.push_back(offM.back() + 64 + (b * 53) % 4033);
    }
    uot_batch_problem pb;
    std::memset(&pb, 0, sizeof(pb));
    pb.dtype = UOT_F32;
    pb.dim = 2;
    pb.B = 4096;
    pb.offN = offN.data();
    pb.offM = offM.data();
    pb.x = pb.y = pb.p = pb.q = pb.dx = pb.dy = kDev;
    pb.F1.kind = pb.F2.kind = UOT_DIV_KL;
    pb.F1.lambda = pb.F2.lambda = 1.0;
    EXPECT(uot_batch_workspace_size(&pb, &n) == UOT_OK);
    EXPECT(n >= (size_t)(offN.back() + offM.back()) * 4);
    size_t nf = 0;
    EXPECT(uot_cloud_features_workspace_size(&pb, &nf) == UOT_OK && nf > n);
    pb.dtype = UOT_F64;
    EXPECT(uot_batch_workspace_size(&pb, &n) == UOT_OK);
    EXPECT(uot_cloud_features_workspace_size(&pb, &nf) == UOT_OK);   // sizing only; the call rejects FP64
    pb.dtype = UOT_F32;
    std::vector<int64_t> empty{0, 10, 10, 20};                  // a problem with N = 0
    pb.offN = empty.data();
    pb.B = 3;
    EXPECT(uot_batch_workspace_size(&pb, &n) == UOT_E_INVALID);
    std::vector<int64_t> shifted{5, 10, 20, 30};                // offsets must start at 0
    pb.offN = shifted.data();
    EXPECT(uot_batch_workspace_size(&pb, &n) == UOT_E_INVALID);
    pb.offN = nullptr;
    EXPECT(uot_batch_workspace_size(&pb, &n) == UOT_E_INVALID);
    pb.offN = offN.data();
    pb.B = 0;
    EXPECT(uot_batch_workspace_size(&pb, &n) == UOT_E_INVALID);
    pb.B = 3;
    pb.dim = 4;
    EXPECT(uot_batch_workspace_size(&pb, &n) == UOT_E_UNSUPPORTED);
  }
  // networks and GEMMs
  {
    uot_net net;
    std::memset(&net, 0, sizeof(net));
    net.n_in = 8192;
    net.width = 256;
    net.n_out = 4096;
    net.in_scale = 1.f;
    int64_t count = 0;
    EXPECT(uot_net_param_count(&net, &count) == UOT_OK);
    EXPECT(count == 8192LL * 256 + 256 + 2 * (256LL * 256 + 256) + 256LL * 4096 + 4096);
    EXPECT(uot_net_workspace_size(&net, 256, &n) == UOT_OK);
    net.n_in = 12;   // not a multiple of 8
    EXPECT(uot_net_param_count(&net, &count) == UOT_E_UNSUPPORTED);
    net.n_in = 16;
    net.n_out = 0;
    EXPECT(uot_net_param_count(&net, &count) == UOT_E_INVALID);
    for (int K : {32, 256, 4096, 8192}) EXPECT(uot_gemm_workspace_size(256, 256, K, &n) == UOT_OK);
    EXPECT(uot_gemm_workspace_size(0, 256, 256, &n) == UOT_E_INVALID);
  }
  // calls that need a context or device buffers are refused on the host
  {
    uot_problem pb = points(UOT_F32, 2, 10, 10);
    uot_params pr;
    std::memset(&pr, 0, sizeof(pr));
    pr.eps = 0.1;
    pr.max_iter = 10;
    pr.check_every = 10;
    uot_result res;
    EXPECT(uot_solve(nullptr, &pb, &pr, nullptr, nullptr, nullptr, 0, &res) == UOT_E_INVALID);
    EXPECT(uot_solve_async(nullptr, &pb, &pr, nullptr, nullptr, nullptr, 0) == UOT_E_INVALID);
    EXPECT(uot_sync_result(nullptr, &res) == UOT_E_INVALID);
    EXPECT(uot_destroy(nullptr) == UOT_OK);
  }
  // a context without a device: creation fails and cleans up after itself
  {
    uot_ctx* ctx = nullptr;
    const int rc = uot_create(&ctx, nullptr);
    if (rc == UOT_OK) {   // (a machine with a GPU)
      EXPECT(uot_destroy(ctx) == UOT_OK);
    } else {
      EXPECT(rc == UOT_E_HIP && ctx == nullptr);
    }
    EXPECT(uot_create(nullptr, nullptr) == UOT_E_INVALID);
  }
  if (failures) {
    std::fprintf(stderr, "%d host check(s) failed\n", failures);
    return 1;
  }
  std::printf("host checks passed\n");
  return 0;
}
