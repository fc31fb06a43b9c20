// Stand-ins for the kernel launchers (csrc/d2q37_kernels.hip) that enqueue
// nothing and touch no memory, so that the C ABI's host logic (argument
// checks, workspace carving, call sequencing, error reporting) can be built
// with AddressSanitizer and run on a machine without a GPU.  Test-only.
#include "d2q37_launch.h"

namespace d2q37 {

int g_stub_device = 0;  // the "current device" the stubbed runtime reports
hipError_t current_device(int* dev) {
  *dev = g_stub_device;
  return hipSuccess;
}
hipError_t launch_zero(void*, size_t, hipStream_t) { return hipSuccess; }
hipError_t launch_halo(void*, const Geom&, int, hipStream_t) { return hipSuccess; }
hipError_t launch_fused(const void*, void*, const Geom&, const Phys&, int, int, double*,
                        hipStream_t) {
  return hipSuccess;
}
hipError_t launch_propagate(const void*, void*, const Geom&, int, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_bc(void*, const Geom&, const Phys&, int, hipStream_t) { return hipSuccess; }
hipError_t launch_propagate_variant(const void*, void*, const Geom&, int, int, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_collide_mfma(const void*, void*, const Geom&, const Phys&, int, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_collide(const void*, void*, const Geom&, const Phys&, int, int, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_init_feq(void*, const double*, const double*, const double*, const double*,
                           const Geom&, const Phys&, int, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_moments(const void*, double*, double*, double*, double*, const Geom&,
                          const Phys&, int, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_pack(const void*, void*, const Geom&, int, hipStream_t) { return hipSuccess; }
hipError_t launch_unpack(const void*, void*, const Geom&, int, hipStream_t) { return hipSuccess; }
hipError_t launch_populations_f64(const void*, double*, const Geom&, const Phys&, int,
                                  hipStream_t) {
  return hipSuccess;
}
hipError_t launch_check(const void*, unsigned int*, const Geom&, const Phys&, int, hipStream_t) {
  return hipSuccess;
}
int observable_chunks(const Geom& g) { return g.lx < 64 ? g.lx : 64; }
hipError_t launch_observables(const void*, double*, double*, double*, const Geom&, const Phys&,
                              int, double, double, hipStream_t) {
  return hipSuccess;
}
int loss_ke_blocks(const Geom& g) { return (g.lx + 1) * ((g.ly + 63) / 64); }
hipError_t launch_loss_ke(const void*, double*, double*, double*, const Geom&, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_adjoint_step(const double*, const double*, double*, const Geom&, const Phys&,
                               int, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_adjoint_mu(const double*, const double*, bool, double*, const Geom&, const Phys&,
                             int, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_adjoint_gather(const double*, double*, const Geom&, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_zero_pad_rows(void*, const Geom&, int, hipStream_t) { return hipSuccess; }
hipError_t launch_init_adjoint(const double*, const double*, const double*, const double*,
                               const double*, double*, double*, double*, double*, const Geom&,
                               hipStream_t) {
  return hipSuccess;
}

// No device memory on the host-only build: the static scratch is unavailable.
hipError_t static_scratch(void**) { return hipErrorNoDevice; }

}  // namespace d2q37
