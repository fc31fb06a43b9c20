// Host-logic check of the C ABI (include/lb.h) with the kernel launchers
// replaced by stand-ins that touch no memory (host_stub_launchers.cpp), built
// with AddressSanitizer and UndefinedBehaviorSanitizer on the host side and
// run without a GPU.  Covers argument validation, workspace carving and
// sizes, call-order rules, every entry point's success path over host-side
// buffers, and the thread-local error message.  Exit status 0 if every
// expectation holds.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "lb.h"

namespace d2q37 {
extern int g_stub_device;  // host_stub_launchers.cpp
}

namespace {

int failures = 0;

void expect(bool ok, const char* what, int line) {
  if (!ok) {
    std::fprintf(stderr, "FAILED line %d: %s (last error: %s)\n", line, what, lb_last_error());
    ++failures;
  }
}

#define EXPECT(cond) expect((cond), #cond, __LINE__)

size_t round256(size_t n) { return (n + 255) / 256 * 256; }

void check_context(int precision, int layout, int kernel, int ybc) {
  const int lx = 40, ly = 30;
  const size_t S = size_t(lx) * ly;
  lb_lattice lat = {lx, ly, precision, ybc, layout, 0};
  lb_params par = {0.7, 1e-4, -1e-4, 1.5, 0.5, 1.0, 1, kernel, 0, 0};
  size_t need = 0;
  const bool local = precision == LB_FP32_COLLIDE || precision == LB_FP32_LOCAL;
  if (local && kernel != LB_KERNEL_FUSED) {  // fused kernel only
    EXPECT(lb_workspace_bytes(&lat, &par, &need) == LB_E_ARG);
    return;
  }
  if (kernel == LB_KERNEL_SPLIT_MFMA && precision != LB_FP64) {  // FP64 matrix cores only
    EXPECT(lb_workspace_bytes(&lat, &par, &need) == LB_E_ARG);
    EXPECT(std::string(lb_last_error()).find("LB_FP64") != std::string::npos);
    return;
  }
  EXPECT(lb_workspace_bytes(&lat, &par, &need) == LB_OK);
  EXPECT(need >= 2 * (local ? 38 : 37) * S * (precision == LB_FP64 ? 8 : 4));
  void* ws = std::aligned_alloc(256, round256(need) + 256);
  std::vector<double> fields(4 * S, 1.0), out(4 * S), lam_a(37 * S), lam_b(37 * S);
  std::vector<double> tape(3 * 4 * S), prof(6 * ly), sc(4), series(3 * 4), pops(37 * S);
  std::vector<char> state(37 * S * 8);
  const double* f = fields.data();
  lb_ctx* ctx = reinterpret_cast<lb_ctx*>(1);

  EXPECT(lb_init(&lat, &par, ws, need - 1, nullptr, f, f + S, f + 2 * S, f + 3 * S, &ctx) ==
         LB_E_WORKSPACE);
  EXPECT(ctx == nullptr);
  EXPECT(lb_init(&lat, &par, static_cast<char*>(ws) + 8, need, nullptr, f, f + S, f + 2 * S,
                 f + 3 * S, &ctx) == LB_E_WORKSPACE);
  EXPECT(lb_init(&lat, &par, nullptr, need, nullptr, f, f + S, f + 2 * S, f + 3 * S, &ctx) ==
         LB_E_ARG);
  EXPECT(lb_init(&lat, &par, ws, need, nullptr, f, nullptr, f + 2 * S, f + 3 * S, &ctx) ==
         LB_E_ARG);
  EXPECT(lb_init(&lat, &par, ws, need, nullptr, f, f + S, f + 2 * S, f + 3 * S, nullptr) ==
         LB_E_ARG);
  EXPECT(lb_init(&lat, &par, ws, need, nullptr, f, f + S, f + 2 * S, f + 3 * S, &ctx) == LB_OK);
  EXPECT(ctx != nullptr);

  EXPECT(lb_step(ctx, 0) == LB_OK);
  EXPECT(lb_step(ctx, 3) == LB_OK);
  EXPECT(lb_step(ctx, -1) == LB_E_ARG);
  EXPECT(lb_moments(ctx, out.data(), out.data() + S, nullptr, out.data() + 3 * S) == LB_OK);
  EXPECT(lb_get_state(ctx, nullptr) == LB_E_ARG);
  EXPECT(lb_get_state(ctx, state.data()) == LB_OK);
  EXPECT(lb_set_state(ctx, state.data()) == LB_OK);
  EXPECT(lb_get_populations(ctx, pops.data()) == LB_OK);
  const int split_rc = local ? LB_E_STATE : LB_OK;
  EXPECT(lb_halo(ctx) == LB_OK);
  EXPECT(lb_propagate(ctx) == split_rc && lb_bc(ctx) == split_rc && lb_collide(ctx) == split_rc);
  EXPECT(lb_get_scratch(ctx, state.data()) == split_rc &&
         lb_set_scratch(ctx, state.data()) == split_rc);
  EXPECT(lb_observables(ctx, prof.data(), sc.data()) == LB_OK);
  EXPECT(lb_observables(ctx, nullptr, sc.data()) == LB_OK);
  EXPECT(lb_run_observed(ctx, 12, 4, series.data()) == LB_OK);
  EXPECT(lb_run_observed(ctx, 12, 0, series.data()) == LB_E_ARG);
  EXPECT(lb_run_observed(ctx, 12, 4, nullptr) == LB_E_ARG);
  EXPECT(lb_run_observed(ctx, 3, 4, nullptr) == LB_OK);
  EXPECT(lb_set_stream(ctx, nullptr) == LB_OK);

  lb_params p2 = par;
  p2.tau = 0.45;
  EXPECT(lb_set_params(ctx, &p2) == LB_E_ARG);
  p2 = par;
  p2.rho_ref = 0.5;
  EXPECT(lb_set_params(ctx, &p2) == (precision == LB_FP64 ? LB_OK : LB_E_ARG));
  p2 = par;
  p2.kernel = kernel == LB_KERNEL_FUSED ? LB_KERNEL_SPLIT : LB_KERNEL_FUSED;
  p2.regularize = 0;
  EXPECT(lb_set_params(ctx, &p2) == (local ? LB_E_ARG : LB_OK));
  p2.kernel = kernel;
  EXPECT(lb_set_params(ctx, &p2) == LB_OK);
  EXPECT(lb_step(ctx, 2) == LB_OK);
  // a call made with another device current is refused, not launched there
  d2q37::g_stub_device = 1;
  EXPECT(lb_step(ctx, 1) == LB_E_STATE);
  EXPECT(std::string(lb_last_error()).find("belongs to device 0") != std::string::npos);
  d2q37::g_stub_device = 0;
  EXPECT(lb_step(ctx, 1) == LB_OK);

  double ke = 0.0;
  double* t = tape.data();
  double* la = lam_a.data();
  double* lbuf = lam_b.data();
  if (precision == LB_FP64) {
    EXPECT(lb_step_record(ctx, 3, t) == LB_OK);
    EXPECT(lb_step_record(ctx, 3, nullptr) == LB_E_ARG);
    EXPECT(lb_step_record(ctx, 0, nullptr) == LB_OK);
    EXPECT(lb_loss_ke(ctx, &ke, la) == LB_OK);
    EXPECT(lb_loss_ke(ctx, nullptr, la) == LB_E_ARG);
    EXPECT(lb_adjoint_step(ctx, t, la, lbuf) == LB_OK);
    EXPECT(lb_adjoint_step(ctx, t, la, la) == LB_E_ARG);
    EXPECT(lb_adjoint_step(ctx, nullptr, la, lbuf) == LB_E_ARG);
    size_t adj = 0;
    EXPECT(lb_adjoint_workspace_bytes(ctx, &adj) == LB_OK && adj >= 2 * 37 * S * 8);
    EXPECT(lb_adjoint_workspace_bytes(ctx, nullptr) == LB_E_ARG);
    void* aws = std::aligned_alloc(256, round256(adj));
    EXPECT(lb_adjoint_run(ctx, 3, t, la, aws, adj) == LB_OK);
    EXPECT(lb_adjoint_run(ctx, 0, nullptr, nullptr, nullptr, 0) == LB_OK);
    EXPECT(lb_adjoint_run(ctx, -1, t, la, aws, adj) == LB_E_ARG);
    EXPECT(lb_adjoint_run(ctx, 3, t, la, aws, adj - 1) == LB_E_WORKSPACE);
    EXPECT(lb_adjoint_run(ctx, 3, t, la, static_cast<char*>(aws) + 8, adj) == LB_E_WORKSPACE);
    EXPECT(lb_adjoint_run(ctx, 3, nullptr, la, aws, adj) == LB_E_ARG);
    EXPECT(lb_adjoint_run_static(ctx, -1, t, la) == LB_E_ARG);
    EXPECT(lb_adjoint_run_static(ctx, 0, nullptr, nullptr) == LB_OK);
    EXPECT(lb_adjoint_run_static(ctx, 3, nullptr, la) == LB_E_ARG);
    std::free(aws);
    EXPECT(lb_init_adjoint(ctx, f, f + S, f + 2 * S, f + 3 * S, lbuf, out.data(), nullptr,
                           nullptr, out.data() + 3 * S) == LB_OK);
    EXPECT(lb_init_adjoint(ctx, f, f + S, f + 2 * S, f + 3 * S, nullptr, out.data(), nullptr,
                           nullptr, nullptr) == LB_E_ARG);
  } else {
    EXPECT(lb_step_record(ctx, 3, t) == LB_E_STATE);
    EXPECT(lb_loss_ke(ctx, &ke, la) == LB_E_STATE);
    EXPECT(lb_adjoint_step(ctx, t, la, lbuf) == LB_E_STATE);
    size_t adj = 0;
    EXPECT(lb_adjoint_workspace_bytes(ctx, &adj) == LB_E_STATE);
    EXPECT(lb_adjoint_run(ctx, 2, t, la, nullptr, 0) == LB_E_STATE);
    EXPECT(lb_adjoint_run_static(ctx, 2, t, la) == LB_E_STATE);
    EXPECT(lb_init_adjoint(ctx, f, f + S, f + 2 * S, f + 3 * S, la, nullptr, nullptr, nullptr,
                           nullptr) == LB_E_STATE);
  }
  EXPECT(std::strlen(lb_last_error()) > 0);
  EXPECT(lb_free(ctx) == LB_OK);
  std::free(ws);
}

}  // namespace

int main() {
  EXPECT(lb_version() == 5);
  lb_lattice lat = {64, 48, LB_FP64, LB_Y_WALLS, LB_LAYOUT_COLUMN, 0};
  lb_params par = {0.7, 0.0, -1e-4, 1.5, 0.5, 1.0, 1, LB_KERNEL_FUSED, 0, 0};
  size_t need = 0;
  EXPECT(lb_workspace_bytes(&lat, &par, &need) == LB_OK);
  EXPECT(lb_workspace_bytes(nullptr, &par, &need) == LB_E_ARG);
  EXPECT(lb_workspace_bytes(&lat, nullptr, &need) == LB_E_ARG);
  EXPECT(lb_workspace_bytes(&lat, &par, nullptr) == LB_E_ARG);
  const lb_lattice bad_lattices[] = {
      {5, 48, LB_FP64, LB_Y_WALLS, LB_LAYOUT_COLUMN, 0},
      {64, 3, LB_FP64, LB_Y_WALLS, LB_LAYOUT_COLUMN, 0},
      {(1 << 22) + 1, 48, LB_FP64, LB_Y_WALLS, LB_LAYOUT_COLUMN, 0},
      {1 << 16, (1 << 14) + 1, LB_FP64, LB_Y_WALLS, LB_LAYOUT_COLUMN, 0},
      {64, 48, 7, LB_Y_WALLS, LB_LAYOUT_COLUMN, 0},
      {64, 48, LB_FP64, 2, LB_LAYOUT_COLUMN, 0},
      {64, 48, LB_FP64, LB_Y_WALLS, 9, 0},
      {64, 48, LB_FP64, LB_Y_WALLS, LB_LAYOUT_COLUMN, 1}};
  for (const lb_lattice& b : bad_lattices) EXPECT(lb_workspace_bytes(&b, &par, &need) == LB_E_ARG);
  lb_params bad = par;
  bad.tau = NAN;
  EXPECT(lb_workspace_bytes(&lat, &bad, &need) == LB_E_ARG);
  bad = par;
  bad.t_top = 0.0;
  EXPECT(lb_workspace_bytes(&lat, &bad, &need) == LB_E_ARG);
  bad = par;
  bad.gy = INFINITY;
  EXPECT(lb_workspace_bytes(&lat, &bad, &need) == LB_E_ARG);
  bad = par;
  bad.check_finite = -2;
  EXPECT(lb_workspace_bytes(&lat, &bad, &need) == LB_E_ARG);
  bad = par;
  bad.reserved = 3;
  EXPECT(lb_workspace_bytes(&lat, &bad, &need) == LB_E_ARG);
  lb_lattice big = {1 << 16, 1 << 14, LB_FP64, LB_Y_WALLS, LB_LAYOUT_COLUMN, 0};
  EXPECT(lb_workspace_bytes(&big, &par, &need) == LB_OK);

  {  // lb_adjoint_run_static rejects lattices beyond its 64 MiB scratch before any launch
    lb_lattice bl = {400, 300, LB_FP64, LB_Y_WALLS, LB_LAYOUT_COLUMN, 0};
    lb_params bp = {0.7, 0.0, -1e-4, 1.5, 0.5, 1.0, 1, LB_KERNEL_FUSED, 0, 0};
    size_t bneed = 0;
    EXPECT(lb_workspace_bytes(&bl, &bp, &bneed) == LB_OK);
    void* bws = std::aligned_alloc(256, round256(bneed));
    const size_t BS = size_t(400) * 300;
    std::vector<double> bf(4 * BS, 1.0), blam(37 * BS), btape(4 * BS);
    lb_ctx* bctx = nullptr;
    EXPECT(lb_init(&bl, &bp, bws, round256(bneed), nullptr, bf.data(), bf.data() + BS,
                   bf.data() + 2 * BS, bf.data() + 3 * BS, &bctx) == LB_OK);
    EXPECT(lb_adjoint_run_static(bctx, 1, btape.data(), blam.data()) == LB_E_WORKSPACE);
    EXPECT(std::string(lb_last_error()).find("64 MiB") != std::string::npos);
    EXPECT(lb_adjoint_run_static(nullptr, 1, btape.data(), blam.data()) == LB_E_ARG);
    lb_free(bctx);
    std::free(bws);
  }

  for (int prec : {LB_FP64, LB_FP32_SHIFTED, LB_FP32_SHIFTED_F32SUM, LB_FP32_COLLIDE,
                   LB_FP32_LOCAL})
    for (int layout : {LB_LAYOUT_SOA, LB_LAYOUT_COLUMN})
      for (int kernel : {LB_KERNEL_FUSED, LB_KERNEL_SPLIT, LB_KERNEL_SPLIT_LDS,
                         LB_KERNEL_SPLIT_WIDE, LB_KERNEL_SPLIT_MFMA})
        for (int ybc : {LB_Y_WALLS, LB_Y_PERIODIC}) check_context(prec, layout, kernel, ybc);

  EXPECT(lb_step(nullptr, 1) == LB_E_ARG);
  EXPECT(lb_free(nullptr) == LB_OK);
  const std::string here = lb_last_error();
  std::string there = "unset";
  std::thread th([&] { there = lb_last_error(); });
  th.join();
  EXPECT(!here.empty() && there.empty());

  std::printf("host_abi_check: %d failure(s)\n", failures);
  return failures ? 1 : 0;
}
