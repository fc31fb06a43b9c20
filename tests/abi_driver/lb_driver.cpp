// Drives the D2Q37 library through its C ABI alone (include/lb.h): no
// PyTorch, device memory from hipMalloc, work on a stream of its own.
//
//   lb_driver <in.bin> <out.bin> <lx> <ly> <steps> <kernel: 0 fused | 1 split>
//
// in.bin: rho0, ux0, uy0, T0 as FP64 [lx][ly] each, back to back.
// out.bin: rho, ux, uy, T after `steps` steps, same layout.
// Also checks, before any device work, that lb_init rejects a workspace one
// byte short and a misaligned one.  Exit status 0 on success; on failure
// prints the library's message and exits 1.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#include "lb.h"

namespace {

int fail(const char* what, int rc) {
  std::fprintf(stderr, "lb_driver: %s returned %d (%s)\n", what, rc, lb_last_error());
  return 1;
}

bool hip_ok(hipError_t e, const char* what) {
  if (e == hipSuccess) return true;
  std::fprintf(stderr, "lb_driver: %s: %s\n", what, hipGetErrorString(e));
  return false;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 7) {
    std::fprintf(stderr, "usage: lb_driver in.bin out.bin lx ly steps kernel\n");
    return 2;
  }
  const int lx = std::atoi(argv[3]), ly = std::atoi(argv[4]), steps = std::atoi(argv[5]);
  const int kernel = std::atoi(argv[6]);
  const size_t n = size_t(lx) * size_t(ly);
  if (lx < 6 || ly < 6 || steps < 0 || n > (size_t(1) << 26)) {
    std::fprintf(stderr, "lb_driver: bad sizes\n");
    return 2;
  }

  std::vector<double> host(4 * n);
  FILE* in = std::fopen(argv[1], "rb");
  if (!in || std::fread(host.data(), sizeof(double), host.size(), in) != host.size()) {
    std::fprintf(stderr, "lb_driver: cannot read %s\n", argv[1]);
    return 2;
  }
  std::fclose(in);

  lb_lattice lat = {lx, ly, LB_FP64, LB_Y_WALLS, LB_LAYOUT_COLUMN, 0};
  lb_params par = {0.7, 0.0, -1e-4, 1.5, 0.5, 1.0, 1, kernel, 0, 0};
  size_t ws_bytes = 0;
  int rc = lb_workspace_bytes(&lat, &par, &ws_bytes);
  if (rc != LB_OK) return fail("lb_workspace_bytes", rc);

  hipStream_t stream = nullptr;
  void* ws = nullptr;
  double* fields = nullptr;  // rho0, ux0, uy0, T0, then the four outputs
  if (!hip_ok(hipStreamCreate(&stream), "hipStreamCreate") ||
      !hip_ok(hipMalloc(&ws, ws_bytes + 256), "hipMalloc workspace") ||
      !hip_ok(hipMalloc(&fields, 8 * n * sizeof(double)), "hipMalloc fields") ||
      !hip_ok(hipMemcpy(fields, host.data(), 4 * n * sizeof(double), hipMemcpyHostToDevice),
              "upload"))
    return 1;
  double* f0[4] = {fields, fields + n, fields + 2 * n, fields + 3 * n};
  double* m[4] = {fields + 4 * n, fields + 5 * n, fields + 6 * n, fields + 7 * n};

  lb_ctx* ctx = nullptr;
  // argument checks happen before any device work
  rc = lb_init(&lat, &par, ws, ws_bytes - 1, stream, f0[0], f0[1], f0[2], f0[3], &ctx);
  if (rc != LB_E_WORKSPACE || ctx) return fail("lb_init with a short workspace", rc);
  rc = lb_init(&lat, &par, static_cast<char*>(ws) + 8, ws_bytes, stream, f0[0], f0[1], f0[2],
               f0[3], &ctx);
  if (rc != LB_E_WORKSPACE || ctx) return fail("lb_init with a misaligned workspace", rc);

  rc = lb_init(&lat, &par, ws, ws_bytes, stream, f0[0], f0[1], f0[2], f0[3], &ctx);
  if (rc != LB_OK) return fail("lb_init", rc);
  rc = lb_step(ctx, steps);
  if (rc != LB_OK) return fail("lb_step", rc);
  rc = lb_moments(ctx, m[0], m[1], m[2], m[3]);
  if (rc != LB_OK) return fail("lb_moments", rc);
  if (!hip_ok(hipStreamSynchronize(stream), "sync") ||
      !hip_ok(hipMemcpy(host.data(), m[0], 4 * n * sizeof(double), hipMemcpyDeviceToHost),
              "download"))
    return 1;
  lb_free(ctx);
  if (!hip_ok(hipFree(fields), "hipFree fields") || !hip_ok(hipFree(ws), "hipFree workspace") ||
      !hip_ok(hipStreamDestroy(stream), "hipStreamDestroy"))
    return 1;

  FILE* out = std::fopen(argv[2], "wb");
  if (!out || std::fwrite(host.data(), sizeof(double), host.size(), out) != host.size()) {
    std::fprintf(stderr, "lb_driver: cannot write %s\n", argv[2]);
    return 2;
  }
  std::fclose(out);
  std::printf("lb_driver: %dx%d, %d steps (kernel %d) done\n", lx, ly, steps, kernel);
  return 0;
}
