// C ABI of the D2Q37 step (declared in include/lb.h): argument checks,
// workspace carving, the per-step launch sequence and error reporting.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "d2q37_launch.h"
#include "lb.h"

using d2q37::Geom;
using d2q37::Phys;

struct lb_ctx {
  int device;  // the HIP device current at lb_init: every launch goes there
  lb_lattice lat;
  lb_params par;
  Geom g;
  Phys p;
  int prec;
  hipStream_t stream;
  char* A;  // state buffer (post-collision populations)
  char* B;  // scratch buffer (propagated populations, next state)
  double* partials;
  double* obs;  // observable scratch (chunk partials | profiles | scalars)
  unsigned int* flag;
  bool halos_valid;
  long long steps_since_check;
};

namespace {

thread_local std::string g_error;

int fail(int code, const char* fmt, const char* what = "") {
  char buf[512];
  std::snprintf(buf, sizeof(buf), fmt, what);
  g_error = buf;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  char buf[512];
  std::snprintf(buf, sizeof(buf), "%s: HIP error %d (%s)", where, int(e), hipGetErrorString(e));
  g_error = buf;
  return LB_E_HIP;
}

// The static scratch of lb_adjoint_run_static (csrc/lb_scratch.hip).
int scratch_address(void** out) {
  const hipError_t e = d2q37::static_scratch(out);
  if (e != hipSuccess) return hip_fail(e, "lb_adjoint_run_static: scratch address");
  return LB_OK;
}

#define LB_HIP(call, where)                   \
  do {                                        \
    hipError_t e_ = (call);                   \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

constexpr size_t kAlign = 256;

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int elem_bytes(int prec) { return prec == LB_FP64 ? 8 : 4; }

// FP32 storage relative to the local rest Maxwellian (38 planes)
bool is_local_form(int prec) { return prec == LB_FP32_COLLIDE || prec == LB_FP32_LOCAL; }

int check_lattice(const lb_lattice* lat) {
  if (!lat) return fail(LB_E_ARG, "lattice is NULL%s");
  if (lat->lx < 6 || lat->ly < 6) return fail(LB_E_ARG, "lx and ly must be >= 6%s");
  // bounds that keep every launch below 2^32 work-items (tile grids cover at
  // most lx*ly + 256*lx + 4*ly + 256 sites) and all 32-bit site indices exact
  if (lat->lx > (1 << 22) || lat->ly > (1 << 24) ||
      (long long)lat->lx * lat->ly > (1LL << 30))
    return fail(LB_E_ARG, "lattice too large (lx <= 2^22, ly <= 2^24, lx*ly <= 2^30)%s");
  if (lat->precision != LB_FP64 && lat->precision != LB_FP32_SHIFTED &&
      lat->precision != LB_FP32_SHIFTED_F32SUM && lat->precision != LB_FP32_COLLIDE &&
      lat->precision != LB_FP32_LOCAL)
    return fail(LB_E_ARG, "unknown precision%s");
  if (lat->ybc != LB_Y_WALLS && lat->ybc != LB_Y_PERIODIC) return fail(LB_E_ARG, "unknown ybc%s");
  if (lat->layout != LB_LAYOUT_SOA && lat->layout != LB_LAYOUT_COLUMN)
    return fail(LB_E_ARG, "unknown layout%s");
  if (lat->reserved != 0) return fail(LB_E_ARG, "lattice.reserved must be 0%s");
  return LB_OK;
}

int check_params(const lb_params* par) {
  if (!par) return fail(LB_E_ARG, "params is NULL%s");
  if (!(par->tau > 0.5) || !std::isfinite(par->tau)) return fail(LB_E_ARG, "tau must be > 0.5%s");
  if (!std::isfinite(par->gx) || !std::isfinite(par->gy)) return fail(LB_E_ARG, "g not finite%s");
  if (!(par->t_bottom > 0) || !(par->t_top > 0) || !std::isfinite(par->t_bottom) ||
      !std::isfinite(par->t_top))
    return fail(LB_E_ARG, "wall temperatures must be finite and > 0%s");
  if (!std::isfinite(par->rho_ref)) return fail(LB_E_ARG, "rho_ref not finite%s");
  if (par->regularize != 0 && par->regularize != 1) return fail(LB_E_ARG, "regularize must be 0 or 1%s");
  if (par->kernel < LB_KERNEL_FUSED || par->kernel > LB_KERNEL_SPLIT_MFMA)
    return fail(LB_E_ARG, "unknown kernel%s");
  if (par->check_finite < 0) return fail(LB_E_ARG, "check_finite must be >= 0%s");
  if (par->reserved != 0) return fail(LB_E_ARG, "params.reserved must be 0%s");
  return LB_OK;
}

Geom make_geom(const lb_lattice& lat) {
  Geom g;
  const int eb = elem_bytes(lat.precision);
  const int per_line = int(kAlign) / eb;  // elements in 256 bytes
  g.lx = lat.lx;
  g.ly = lat.ly;
  g.nx = lat.lx + 2 * d2q37::HX;
  g.hy = per_line;  // physical row 0 starts 256-byte aligned
  g.ny = int(round_up(size_t(lat.ly) + 2 * size_t(g.hy), size_t(per_line)));
  g.walls = lat.ybc == LB_Y_WALLS;
  g.np = is_local_form(lat.precision) ? d2q37::kLocalPlanes : d2q37::Q;
  if (lat.layout == LB_LAYOUT_SOA) {
    g.ps = (long long)g.nx * g.ny;
    g.cs = g.ny;
  } else {
    g.ps = g.ny;
    g.cs = (long long)g.np * g.ny;
  }
  return g;
}

Phys make_phys(const lb_params& par, int prec) {
  Phys p;
  p.omega = 1.0 / par.tau;
  p.tau_gx = par.tau * par.gx;
  p.tau_gy = par.tau * par.gy;
  p.dtheta = par.tau * (1.0 - par.tau) * (par.gx * par.gx + par.gy * par.gy) / 2.0;
  p.th_bottom = par.t_bottom - 1.0;
  p.th_top = par.t_top - 1.0;
  p.rho_ref = (prec == LB_FP64 || is_local_form(prec)) ? 0.0 : par.rho_ref;
  return p;
}

size_t buffer_bytes(const Geom& g, int prec) {
  return round_up(size_t(g.np) * size_t(g.nx) * size_t(g.ny) * elem_bytes(prec), kAlign);
}

// The local-reference forms rebuild a population from the reference of the
// site it comes from, which only the fused step has at hand: no split path.
int check_kernel(int prec, const lb_params& par) {
  if (is_local_form(prec) && par.kernel != LB_KERNEL_FUSED)
    return fail(LB_E_ARG, "LB_FP32_COLLIDE and LB_FP32_LOCAL run the fused kernel only%s");
  if (par.kernel == LB_KERNEL_SPLIT_MFMA && prec != LB_FP64)
    return fail(LB_E_ARG, "LB_KERNEL_SPLIT_MFMA needs LB_FP64%s");
  return LB_OK;
}

// The split stages, with the alternative kernel the context's kernel value
// names (same results as the main ones).
hipError_t propagate_stage(lb_ctx* c) {
  if (c->par.kernel == LB_KERNEL_SPLIT_LDS)
    return d2q37::launch_propagate_variant(c->A, c->B, c->g, c->prec, d2q37::kPropagateLds,
                                           c->stream);
  if (c->par.kernel == LB_KERNEL_SPLIT_WIDE)
    return d2q37::launch_propagate_variant(c->A, c->B, c->g, c->prec, d2q37::kPropagateWide,
                                           c->stream);
  return d2q37::launch_propagate(c->A, c->B, c->g, c->prec, c->stream);
}

hipError_t collide_stage(lb_ctx* c) {
  if (c->par.kernel == LB_KERNEL_SPLIT_MFMA)
    return d2q37::launch_collide_mfma(c->B, c->A, c->g, c->p, c->par.regularize, c->stream);
  return d2q37::launch_collide(c->B, c->A, c->g, c->p, c->prec, c->par.regularize, c->stream);
}

int no_split_stage(lb_ctx* ctx, const char* what) {
  if (is_local_form(ctx->prec))
    return fail(LB_E_STATE, "%s is not available for the local-reference forms (fused only)",
                what);
  return LB_OK;
}

size_t partial_bytes(const Geom& g) {
  return round_up(size_t(d2q37::loss_ke_blocks(g)) * sizeof(double), kAlign);
}

// observable scratch: chunk partials, then the profiles and the scalars
size_t observable_bytes(const Geom& g) {
  const size_t prof = size_t(d2q37::kObservables) * size_t(g.ly);
  return round_up((size_t(d2q37::observable_chunks(g)) * prof + prof +
                   size_t(d2q37::kObservableScalars)) * sizeof(double), kAlign);
}

// A context's buffers and stream live on the device that was current at
// lb_init, and kernels launch on the current device: refuse a call made with
// another device current instead of launching there.
int check_ctx(lb_ctx* ctx) {
  if (!ctx) return fail(LB_E_ARG, "context is NULL%s");
  int dev = -1;
  const hipError_t e = d2q37::current_device(&dev);
  if (e != hipSuccess) return hip_fail(e, "current device");
  if (dev != ctx->device) {
    char buf[160];
    std::snprintf(buf, sizeof(buf),
                  "the context belongs to device %d but device %d is current", ctx->device, dev);
    g_error = buf;
    return LB_E_STATE;
  }
  return LB_OK;
}

int need_fp64(lb_ctx* ctx, const char* what) {
  if (ctx->prec != LB_FP64) return fail(LB_E_STATE, "%s needs an LB_FP64 context", what);
  return LB_OK;
}

int do_halo(lb_ctx* c) {
  LB_HIP(d2q37::launch_halo(c->A, c->g, c->prec, c->stream), "halo");
  c->halos_valid = true;
  return LB_OK;
}

int check_finite_now(lb_ctx* c) {
  LB_HIP(d2q37::launch_zero(c->flag, kAlign, c->stream), "check_finite zero");
  LB_HIP(d2q37::launch_check(c->A, c->flag, c->g, c->p, c->prec, c->stream), "check_finite");
  unsigned int bad = 0;
  LB_HIP(hipMemcpyAsync(&bad, c->flag, sizeof(bad), hipMemcpyDeviceToHost, c->stream),
         "check_finite copy");
  LB_HIP(hipStreamSynchronize(c->stream), "check_finite sync");
  if (bad) {
    char buf[128];
    std::snprintf(buf, sizeof(buf), "%u sites with rho<=0, T<=0 or a non-finite population", bad);
    g_error = buf;
    return LB_E_NONFINITE;
  }
  return LB_OK;
}

int one_step(lb_ctx* c, double* tape) {
  if (c->par.kernel == LB_KERNEL_FUSED || tape) {
    if (!c->halos_valid || !c->g.walls) {
      int rc = do_halo(c);
      if (rc) return rc;
    }
    LB_HIP(d2q37::launch_fused(c->A, c->B, c->g, c->p, c->prec, c->par.regularize, tape,
                               c->stream),
           "fused step");
    std::swap(c->A, c->B);
    // the fused kernel writes the x halos of its output; y halos (periodic
    // y) are refreshed before the next step
    c->halos_valid = c->g.walls;
  } else {
    int rc = do_halo(c);
    if (rc) return rc;
    LB_HIP(propagate_stage(c), "propagate");
    LB_HIP(d2q37::launch_bc(c->B, c->g, c->p, c->prec, c->stream), "bc");
    LB_HIP(collide_stage(c), "collide");
    c->halos_valid = false;
  }
  if (c->par.check_finite > 0 && ++c->steps_since_check >= c->par.check_finite) {
    c->steps_since_check = 0;
    return check_finite_now(c);
  }
  return LB_OK;
}

// n transposed steps, lambda^n -> lambda^0 in place, with the two padded FP64
// buffers at ws (2 * buffer_bytes(g, LB_FP64) bytes, 256-byte aligned).
int adjoint_run(lb_ctx* ctx, int n, const double* tape, double* lambda, char* ws) {
  const size_t nb = buffer_bytes(ctx->g, LB_FP64);
  double* m0 = reinterpret_cast<double*>(ws);
  double* m1 = reinterpret_cast<double*>(ws + nb);
  const Geom& g = ctx->g;
  const bool walls = g.walls != 0;
  const long long per = 4LL * g.lx * g.ly;
  const int reg = ctx->par.regularize;
  // Where the two compact lambda arrays fit in the 256 MB Infinity Cache the
  // scatter form's partial-sector stores cost nothing and it is the faster
  // one (measured 25 vs 33 us at 512 x 512; the gather form wins from
  // 768 x 768 up and on lattices too small to fill the GPU); same result.
  const long long sites = (long long)g.lx * g.ly;
  const bool scatter = sites >= (1LL << 17) && 2 * 37 * 8 * sites <= (256LL << 20);
  if (scatter) {
    double* in = lambda;
    double* out = m0;  // a compact array fits in one padded buffer
    for (int j = n - 1; j >= 0; --j) {
      LB_HIP(d2q37::launch_adjoint_step(tape + per * j, in, out, g, ctx->p, reg, ctx->stream),
             "adjoint_run step");
      std::swap(in, out);
    }
    if (in != lambda)
      LB_HIP(hipMemcpyAsync(lambda, in, size_t(37) * size_t(sites) * sizeof(double),
                            hipMemcpyDeviceToDevice, ctx->stream),
             "adjoint_run copy");
    return LB_OK;
  }
  if (walls) {  // the gather reads zero beyond the walls
    LB_HIP(d2q37::launch_zero_pad_rows(m0, g, LB_FP64, ctx->stream), "adjoint_run pad rows");
    LB_HIP(d2q37::launch_zero_pad_rows(m1, g, LB_FP64, ctx->stream), "adjoint_run pad rows");
  }
  LB_HIP(d2q37::launch_adjoint_mu(tape + per * (n - 1), lambda, true, m0, g, ctx->p, reg,
                                  ctx->stream),
         "adjoint_run first step");
  for (int j = n - 2; j >= 0; --j) {
    if (!walls) LB_HIP(d2q37::launch_halo(m0, g, LB_FP64, ctx->stream), "adjoint_run halo");
    LB_HIP(d2q37::launch_adjoint_mu(tape + per * j, m0, false, m1, g, ctx->p, reg, ctx->stream),
           "adjoint_run step");
    std::swap(m0, m1);
  }
  if (!walls) LB_HIP(d2q37::launch_halo(m0, g, LB_FP64, ctx->stream), "adjoint_run halo");
  LB_HIP(d2q37::launch_adjoint_gather(m0, lambda, g, ctx->stream), "adjoint_run gather");
  return LB_OK;
}

}  // namespace

extern "C" {

const char* lb_last_error(void) { return g_error.c_str(); }

int lb_version(void) { return 5; }

int lb_workspace_bytes(const lb_lattice* lat, const lb_params* par, size_t* bytes) {
  int rc = check_lattice(lat);
  if (rc) return rc;
  rc = check_params(par);
  if (rc) return rc;
  rc = check_kernel(lat->precision, *par);
  if (rc) return rc;
  if (!bytes) return fail(LB_E_ARG, "bytes is NULL%s");
  const Geom g = make_geom(*lat);
  *bytes = 2 * buffer_bytes(g, lat->precision) + partial_bytes(g) + observable_bytes(g) + kAlign;
  return LB_OK;
}

int lb_init(const lb_lattice* lat, const lb_params* par, void* workspace, size_t workspace_bytes,
            void* stream, const double* rho0, const double* ux0, const double* uy0,
            const double* T0, lb_ctx** out) {
  if (!out) return fail(LB_E_ARG, "out is NULL%s");
  *out = nullptr;
  size_t need = 0;
  int rc = lb_workspace_bytes(lat, par, &need);
  if (rc) return rc;
  if (!workspace) return fail(LB_E_ARG, "workspace is NULL%s");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
    return fail(LB_E_WORKSPACE, "workspace must be 256-byte aligned%s");
  if (workspace_bytes < need) return fail(LB_E_WORKSPACE, "workspace too small%s");
  if (!rho0 || !ux0 || !uy0 || !T0) return fail(LB_E_ARG, "initial fields must not be NULL%s");
  if (lat->precision != LB_FP64 && !(par->rho_ref >= 0))
    return fail(LB_E_ARG, "rho_ref must be >= 0%s");
  int dev = -1;
  LB_HIP(d2q37::current_device(&dev), "current device");
  lb_ctx* c = new (std::nothrow) lb_ctx;
  if (!c) return fail(LB_E_ARG, "out of host memory%s");
  c->device = dev;
  c->lat = *lat;
  c->par = *par;
  c->prec = lat->precision;
  c->g = make_geom(*lat);
  c->p = make_phys(*par, c->prec);
  c->stream = static_cast<hipStream_t>(stream);
  const size_t nb = buffer_bytes(c->g, c->prec);
  char* ws = static_cast<char*>(workspace);
  c->A = ws;
  c->B = ws + nb;
  c->partials = reinterpret_cast<double*>(ws + 2 * nb);
  c->obs = reinterpret_cast<double*>(ws + 2 * nb + partial_bytes(c->g));
  c->flag = reinterpret_cast<unsigned int*>(ws + 2 * nb + partial_bytes(c->g) +
                                            observable_bytes(c->g));
  c->halos_valid = false;
  c->steps_since_check = 0;
  // Rows beyond the walls are never written by a step; the wall rows' gather
  // reads them before bc replaces those populations.  Give them finite values
  // (zero); every other element is written before it is read.
  hipError_t e = d2q37::launch_zero_pad_rows(c->A, c->g, c->prec, c->stream);
  if (e == hipSuccess) e = d2q37::launch_zero_pad_rows(c->B, c->g, c->prec, c->stream);
  if (e == hipSuccess)
    e = d2q37::launch_init_feq(c->A, rho0, ux0, uy0, T0, c->g, c->p, c->prec, c->stream);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "lb_init");
  }
  rc = do_halo(c);
  if (rc) {
    delete c;
    return rc;
  }
  *out = c;
  return LB_OK;
}

int lb_free(lb_ctx* ctx) {
  delete ctx;
  return LB_OK;
}

int lb_set_stream(lb_ctx* ctx, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  ctx->stream = static_cast<hipStream_t>(stream);
  return LB_OK;
}

int lb_set_params(lb_ctx* ctx, const lb_params* par) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  rc = check_params(par);
  if (rc) return rc;
  rc = check_kernel(ctx->prec, *par);
  if (rc) return rc;
  if (ctx->prec != LB_FP64 && par->rho_ref != ctx->par.rho_ref)
    return fail(LB_E_ARG, "rho_ref cannot change after lb_init%s");
  ctx->par = *par;
  ctx->p = make_phys(*par, ctx->prec);
  return LB_OK;
}

int lb_step(lb_ctx* ctx, int n) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (n < 0) return fail(LB_E_ARG, "n must be >= 0%s");
  for (int i = 0; i < n; ++i) {
    rc = one_step(ctx, nullptr);
    if (rc) return rc;
  }
  return LB_OK;
}

int lb_moments(lb_ctx* ctx, double* rho, double* ux, double* uy, double* T) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  LB_HIP(d2q37::launch_moments(ctx->A, rho, ux, uy, T, ctx->g, ctx->p, ctx->prec, ctx->stream),
         "moments");
  return LB_OK;
}

int lb_get_state(lb_ctx* ctx, void* f) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!f) return fail(LB_E_ARG, "f is NULL%s");
  LB_HIP(d2q37::launch_pack(ctx->A, f, ctx->g, ctx->prec, ctx->stream), "get_state");
  return LB_OK;
}

int lb_set_state(lb_ctx* ctx, const void* f) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!f) return fail(LB_E_ARG, "f is NULL%s");
  LB_HIP(d2q37::launch_unpack(f, ctx->A, ctx->g, ctx->prec, ctx->stream), "set_state");
  return do_halo(ctx);
}

int lb_get_populations(lb_ctx* ctx, double* f) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!f) return fail(LB_E_ARG, "f is NULL%s");
  LB_HIP(d2q37::launch_populations_f64(ctx->A, f, ctx->g, ctx->p, ctx->prec, ctx->stream),
         "get_populations");
  return LB_OK;
}

int lb_halo(lb_ctx* ctx) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  return do_halo(ctx);
}

int lb_propagate(lb_ctx* ctx) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  rc = no_split_stage(ctx, "lb_propagate");
  if (rc) return rc;
  LB_HIP(propagate_stage(ctx), "propagate");
  return LB_OK;
}

int lb_bc(lb_ctx* ctx) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  rc = no_split_stage(ctx, "lb_bc");
  if (rc) return rc;
  LB_HIP(d2q37::launch_bc(ctx->B, ctx->g, ctx->p, ctx->prec, ctx->stream), "bc");
  return LB_OK;
}

int lb_collide(lb_ctx* ctx) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  rc = no_split_stage(ctx, "lb_collide");
  if (rc) return rc;
  LB_HIP(collide_stage(ctx), "collide");
  ctx->halos_valid = false;
  return LB_OK;
}

int lb_get_scratch(lb_ctx* ctx, void* f) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  rc = no_split_stage(ctx, "lb_get_scratch");
  if (rc) return rc;
  if (!f) return fail(LB_E_ARG, "f is NULL%s");
  LB_HIP(d2q37::launch_pack(ctx->B, f, ctx->g, ctx->prec, ctx->stream), "get_scratch");
  return LB_OK;
}

int lb_set_scratch(lb_ctx* ctx, const void* f) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  rc = no_split_stage(ctx, "lb_set_scratch");
  if (rc) return rc;
  if (!f) return fail(LB_E_ARG, "f is NULL%s");
  LB_HIP(d2q37::launch_unpack(f, ctx->B, ctx->g, ctx->prec, ctx->stream), "set_scratch");
  return LB_OK;
}

int lb_observables(lb_ctx* ctx, double* profiles, double* scalars) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  const size_t prof = size_t(d2q37::kObservables) * size_t(ctx->g.ly);
  double* partial = ctx->obs;
  double* own_prof = ctx->obs + size_t(d2q37::observable_chunks(ctx->g)) * prof;
  LB_HIP(d2q37::launch_observables(ctx->A, partial, profiles ? profiles : own_prof, scalars,
                                   ctx->g, ctx->p, ctx->prec, ctx->par.t_bottom, ctx->par.t_top,
                                   ctx->stream),
         "observables");
  return LB_OK;
}

int lb_run_observed(lb_ctx* ctx, int n, int every, double* series) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (n < 0 || every <= 0) return fail(LB_E_ARG, "need n >= 0 and every > 0%s");
  if (n >= every && !series) return fail(LB_E_ARG, "series is NULL%s");
  for (int i = 1; i <= n; ++i) {
    rc = one_step(ctx, nullptr);
    if (rc) return rc;
    if (i % every == 0) {
      rc = lb_observables(ctx, nullptr,
                          series + size_t(i / every - 1) * d2q37::kObservableScalars);
      if (rc) return rc;
    }
  }
  return LB_OK;
}

int lb_step_record(lb_ctx* ctx, int n, double* tape) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  rc = need_fp64(ctx, "lb_step_record");
  if (rc) return rc;
  if (n < 0) return fail(LB_E_ARG, "n must be >= 0%s");
  if (n > 0 && !tape) return fail(LB_E_ARG, "tape is NULL%s");
  const long long per = 4LL * ctx->g.lx * ctx->g.ly;
  for (int i = 0; i < n; ++i) {
    rc = one_step(ctx, tape + per * i);
    if (rc) return rc;
  }
  return LB_OK;
}

int lb_loss_ke(lb_ctx* ctx, double* ke_dev, double* lambda) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  rc = need_fp64(ctx, "lb_loss_ke");
  if (rc) return rc;
  if (!ke_dev) return fail(LB_E_ARG, "ke_dev is NULL%s");
  LB_HIP(d2q37::launch_loss_ke(ctx->A, ke_dev, lambda, ctx->partials, ctx->g, ctx->stream),
         "loss_ke");
  return LB_OK;
}

int lb_adjoint_step(lb_ctx* ctx, const double* tape_j, const double* lambda_in,
                    double* lambda_out) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  rc = need_fp64(ctx, "lb_adjoint_step");
  if (rc) return rc;
  if (!tape_j || !lambda_in || !lambda_out) return fail(LB_E_ARG, "NULL argument%s");
  if (lambda_in == lambda_out) return fail(LB_E_ARG, "lambda_in and lambda_out must differ%s");
  LB_HIP(d2q37::launch_adjoint_step(tape_j, lambda_in, lambda_out, ctx->g, ctx->p,
                                    ctx->par.regularize, ctx->stream),
         "adjoint_step");
  return LB_OK;
}

int lb_adjoint_workspace_bytes(lb_ctx* ctx, size_t* bytes) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  rc = need_fp64(ctx, "lb_adjoint_workspace_bytes");
  if (rc) return rc;
  if (!bytes) return fail(LB_E_ARG, "bytes is NULL%s");
  *bytes = 2 * buffer_bytes(ctx->g, LB_FP64);
  return LB_OK;
}

int lb_adjoint_run(lb_ctx* ctx, int n, const double* tape, double* lambda, void* workspace,
                   size_t workspace_bytes) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  rc = need_fp64(ctx, "lb_adjoint_run");
  if (rc) return rc;
  if (n < 0) return fail(LB_E_ARG, "n must be >= 0%s");
  if (n == 0) return LB_OK;
  if (!tape || !lambda || !workspace) return fail(LB_E_ARG, "NULL argument%s");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
    return fail(LB_E_WORKSPACE, "adjoint workspace must be 256-byte aligned%s");
  const size_t nb = buffer_bytes(ctx->g, LB_FP64);
  if (workspace_bytes < 2 * nb) return fail(LB_E_WORKSPACE, "adjoint workspace too small%s");
  return adjoint_run(ctx, n, tape, lambda, static_cast<char*>(workspace));
}

int lb_adjoint_run_static(lb_ctx* ctx, int n, const double* tape, double* lambda) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  rc = need_fp64(ctx, "lb_adjoint_run_static");
  if (rc) return rc;
  if (n < 0) return fail(LB_E_ARG, "n must be >= 0%s");
  if (2 * buffer_bytes(ctx->g, LB_FP64) > d2q37::kStaticScratchBytes)
    return fail(LB_E_WORKSPACE,
                "lattice too large for the 64 MiB static adjoint scratch "
                "(2 padded FP64 buffers; use lb_adjoint_run with a workspace)%s");
  if (n == 0) return LB_OK;
  if (!tape || !lambda) return fail(LB_E_ARG, "NULL argument%s");
  void* ws = nullptr;
  rc = scratch_address(&ws);
  if (rc) return rc;
  return adjoint_run(ctx, n, tape, lambda, static_cast<char*>(ws));
}

int lb_init_adjoint(lb_ctx* ctx, const double* rho0, const double* ux0, const double* uy0,
                    const double* T0, const double* lambda0, double* drho0, double* dux0,
                    double* duy0, double* dT0) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  rc = need_fp64(ctx, "lb_init_adjoint");
  if (rc) return rc;
  if (!rho0 || !ux0 || !uy0 || !T0 || !lambda0) return fail(LB_E_ARG, "NULL argument%s");
  LB_HIP(d2q37::launch_init_adjoint(lambda0, rho0, ux0, uy0, T0, drho0, dux0, duy0, dT0, ctx->g,
                                    ctx->stream),
         "init_adjoint");
  return LB_OK;
}

}  // extern "C"
