// Host-side launchers of the D2Q37 kernels (implemented in d2q37_kernels.hip).
// Every launcher enqueues on the given stream and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "d2q37_device.h"

namespace d2q37 {

// Precision modes (values of lb_lattice.precision): storage / collision.
enum Precision {
  kF64 = 0,
  kF32Shifted = 1,
  kF32ShiftedF32Sum = 2,
  kF32Collide = 3,
  kF32Local = 4
};

// The current HIP device (hipGetDevice).
hipError_t current_device(int* dev);

// Fill `bytes` (multiple of 4) of device memory with zero.
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);

// Periodic refresh of halo columns (and, for periodic y, halo rows) of a
// padded population buffer.
hipError_t launch_halo(void* buf, const Geom& g, int prec, hipStream_t s);

// One fused step: dst = collide(bc(propagate(src))), with the periodic x
// halos of dst written too.  tape (optional, FP64 only): [4][lx][ly].
hipError_t launch_fused(const void* src, void* dst, const Geom& g, const Phys& p, int prec,
                        int regularize, double* tape, hipStream_t s);

// Split path.
hipError_t launch_propagate(const void* src, void* dst, const Geom& g, int prec, hipStream_t s);
hipError_t launch_bc(void* buf, const Geom& g, const Phys& p, int prec, hipStream_t s);
hipError_t launch_collide(const void* src, void* dst, const Geom& g, const Phys& p, int prec,
                          int regularize, hipStream_t s);

// Alternative split-stage kernels (d2q37_variants.hip), same results:
// propagate staged through LDS or with 16-byte accesses (FP64 and the
// shifted FP32 forms), and the FP64 collide on the matrix cores.
enum PropagateVariant { kPropagateLds = 1, kPropagateWide = 2 };
hipError_t launch_propagate_variant(const void* src, void* dst, const Geom& g, int prec,
                                    int variant, hipStream_t s);
hipError_t launch_collide_mfma(const void* src, void* dst, const Geom& g, const Phys& p,
                               int regularize, hipStream_t s);

// dst = f^eq(rho0, u0, T0) (shifted by w rho_ref for FP32), physical region.
hipError_t launch_init_feq(void* dst, const double* rho, const double* ux, const double* uy,
                           const double* T, const Geom& g, const Phys& p, int prec,
                           hipStream_t s);

// Eq. (2) moments of a padded buffer in FP64; outputs may be null.
hipError_t launch_moments(const void* src, double* rho, double* ux, double* uy, double* T,
                          const Geom& g, const Phys& p, int prec, hipStream_t s);

// Copies between a padded buffer and the compact [37][lx][ly] form.
hipError_t launch_pack(const void* padded, void* compact, const Geom& g, int prec,
                       hipStream_t s);
hipError_t launch_unpack(const void* compact, void* padded, const Geom& g, int prec,
                         hipStream_t s);
// Unshifted FP64 populations of a padded buffer, compact form.
hipError_t launch_populations_f64(const void* padded, double* out, const Geom& g,
                                  const Phys& p, int prec, hipStream_t s);

// Counts sites with rho <= 0, T <= 0 or a non-finite value into *flag
// (which the caller zeroes first).
hipError_t launch_check(const void* src, unsigned int* flag, const Geom& g, const Phys& p,
                        int prec, hipStream_t s);

// In-situ observables.  profiles: [kObservables][ly] row averages over x of
// rho, u_x, u_y, T, rho |u|^2 / 2, rho T; scalars (optional): total mass,
// kinetic energy, sum of rho T, mixing-layer width.  partial: scratch of
// observable_chunks(g) * kObservables * ly doubles.
constexpr int kObservables = 6;
constexpr int kObservableScalars = 4;
int observable_chunks(const Geom& g);
hipError_t launch_observables(const void* src, double* partial, double* profiles,
                              double* scalars, const Geom& g, const Phys& p, int prec,
                              double t_bottom, double t_top, hipStream_t s);

// Adjoint (FP64 buffers).
// KE of the padded state: per-block partial sums into `partials` (size
// returned by loss_ke_blocks), then reduced into *ke; lambda (optional)
// compact, in the lattice's layout ([lx][37][ly] column, [37][lx][ly] SoA),
// as are the adjoint arrays below.
int loss_ke_blocks(const Geom& g);
hipError_t launch_loss_ke(const void* src, double* ke, double* lambda, double* partials,
                          const Geom& g, hipStream_t s);
hipError_t launch_adjoint_step(const double* tape, const double* lam_in, double* lam_out,
                               const Geom& g, const Phys& p, int regularize, hipStream_t s);
// Gather form of a run of adjoint steps over padded FP64 buffers laid out
// like the state: mu_out = B^T C(tape)^T lambda at the arriving populations,
// lambda read from a compact array (from_compact) or gathered from a padded
// mu buffer (lambda_l(z) = mu_l(z + e_l)); the last step gathers into a
// compact array.  Rows beyond the walls of a mu buffer must be zero
// (launch_zero_pad_rows: the padded rows outside [0, ly) of a padded buffer
// of the given precision) or, for periodic y, refreshed halos.
hipError_t launch_adjoint_mu(const double* tape, const double* in, bool from_compact, double* mu_out,
                             const Geom& g, const Phys& p, int regularize, hipStream_t s);
hipError_t launch_adjoint_gather(const double* mu, double* lam, const Geom& g, hipStream_t s);
hipError_t launch_zero_pad_rows(void* buf, const Geom& g, int prec, hipStream_t s);
hipError_t launch_init_adjoint(const double* lam0, const double* rho, const double* ux,
                               const double* uy, const double* T, double* drho, double* dux,
                               double* duy, double* dT, const Geom& g, hipStream_t s);

// The library's per-GPU static scratch (lb_adjoint_run_static): its size,
// and its device address on the current device (looked up on the first call
// for each device, then kept).
constexpr size_t kStaticScratchBytes = size_t(64) << 20;  // 64 MiB
hipError_t static_scratch(void** out);

}  // namespace d2q37
