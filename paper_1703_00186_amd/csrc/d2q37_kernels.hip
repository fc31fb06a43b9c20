// D2Q37 kernels for gfx950 (MI355X) and their host launchers.
//
// Site kernels map one thread to one lattice site.  A workgroup is a tile of
// BY consecutive rows (y, the contiguous direction) by BX columns, BY*BX = 256
// (four wave64s).  Tiles are numbered column-major (all row tiles of a column
// first), and the flat workgroup index is remapped so that consecutive tiles
// land on the same XCD: workgroups are handed to the 8 XCDs round-robin, and
// a population's misaligned row segment shares its end cache lines with the
// neighbouring row tile of the same column, which then hits that XCD's L2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "d2q37_launch.h"

namespace d2q37 {

namespace {

constexpr int kThreads = 256;
constexpr int kXcds = 8;

struct Tiling {
  int by, bx;    // tile shape (rows, columns)
  int nty, ntx;  // tiles along y and x
  unsigned nb;   // total tiles
};

Tiling make_tiling(int lx, int ly) {
  Tiling t;
  t.by = ly > 128 ? 256 : (ly > 64 ? 128 : 64);
  t.bx = kThreads / t.by;
  t.nty = (ly + t.by - 1) / t.by;
  t.ntx = (lx + t.bx - 1) / t.bx;
  t.nb = unsigned(t.nty) * unsigned(t.ntx);
  return t;
}

// Tile of this workgroup after the XCD-aware remap (a bijection of [0, nb)).
__device__ __forceinline__ unsigned tile_index(unsigned nb) {
  const unsigned b = blockIdx.x;
  const unsigned q = nb / kXcds, rem = nb % kXcds;
  const unsigned xcd = b % kXcds, j = b / kXcds;
  return xcd * q + (xcd < rem ? xcd : rem) + j;
}

// Physical (x, y) of this thread; false if it falls outside the lattice.
__device__ __forceinline__ bool site_of(const Geom& g, int by, int bx, int nty, unsigned nb,
                                        int& x, int& y) {
  const unsigned t = tile_index(nb);
  const int ty = int(t % unsigned(nty)), tx = int(t / unsigned(nty));
  const int lin = threadIdx.x;
  y = ty * by + (lin % by);
  x = tx * bx + (lin / by);
  return x < g.lx && y < g.ly;
}

template <class S>
__device__ __forceinline__ long long padded(const Geom& g, int X, int Y) {
  return (long long)X * g.cs + Y;
}

// Gather of propagate: f_l = src(l, x - e_lx, y - e_ly) (Eq. (1), Fig. 4).
template <class S, class A>
__device__ __forceinline__ void gather(const S* __restrict__ src, const Geom& g, long long site,
                                       A (&f)[Q]) {
#pragma unroll
  for (int l = 0; l < Q; ++l) f[l] = A(src[l * g.ps + site - EX[l] * g.cs - EY[l]]);
}

template <class S, class A>
__device__ __forceinline__ void load_site(const S* __restrict__ src, const Geom& g,
                                          long long site, A (&f)[Q]) {
#pragma unroll
  for (int l = 0; l < Q; ++l) f[l] = A(src[l * g.ps + site]);
}

// Stores of a step's output are streamed past the caches (non-temporal):
// the next step reads them only after the whole lattice, far more than the
// caches hold, has been written.
template <class S, class A>
__device__ __forceinline__ void store_site(S* __restrict__ dst, const Geom& g, long long site,
                                           const A (&f)[Q]) {
#pragma unroll
  for (int l = 0; l < Q; ++l) __builtin_nontemporal_store(S(f[l]), &dst[l * g.ps + site]);
}

// Accumulation-type tags of the local-reference FP32 forms (populations
// stored as FP32 deviations from the rest Maxwellian of their writer site,
// plus that site's packed reference in plane Q), with the FP32 or the FP64
// collision.
template <bool kF64Collide>
struct LocalRefT {
  static constexpr bool f64_collide = kF64Collide;
};
using LocalRef = LocalRefT<false>;    // FP32 collision (collide_site_local)
using LocalRef64 = LocalRefT<true>;   // FP64 collision (collide_site_local64)
template <class A>
constexpr bool is_local = std::is_same<A, LocalRef>::value || std::is_same<A, LocalRef64>::value;

// The packed reference word of padded site `site` (plane Q).
__device__ __forceinline__ unsigned ref_at(const float* __restrict__ buf, const Geom& g,
                                           long long site) {
  return reinterpret_cast<const unsigned*>(buf)[Q * g.ps + site];
}

// FP64 populations of one padded site in the local-reference form: all 37
// deviations are relative to the site's own reference.
__device__ __forceinline__ void load_local(const float* __restrict__ src, const Geom& g,
                                           long long site, double (&f)[Q]) {
  double rho, th;
  unpack_ref(ref_at(src, g, site), rho, th);
#pragma unroll
  for (int l = 0; l < Q; ++l) f[l] = rest_maxwellian(l, rho, th) + double(src[l * g.ps + site]);
}

__device__ __forceinline__ void store_local(float* __restrict__ dst, const Geom& g, long long site,
                                            const float (&v)[Q], unsigned ref) {
#pragma unroll
  for (int l = 0; l < Q; ++l) __builtin_nontemporal_store(v[l], &dst[l * g.ps + site]);
  __builtin_nontemporal_store(ref, &reinterpret_cast<unsigned*>(dst)[Q * g.ps + site]);
}

// Adjoint arrays are compact (no halos) in the lattice's layout: [lx][37][ly]
// for the column layout (population stride below column stride), [37][lx][ly]
// for SoA.
struct LamStrides {
  long long ps, cs;
};

__device__ __forceinline__ LamStrides lam_strides(const Geom& g) {
  const long long s2 = (long long)g.lx * g.ly;
  return g.ps < g.cs ? LamStrides{g.ly, (long long)Q * g.ly} : LamStrides{s2, g.ly};
}

__device__ __forceinline__ bool on_wall_rows(const Geom& g, int y) {
  return g.walls && (y < 3 || y >= g.ly - 3);
}

// ---------------------------------------------------------------------------
// Fused step: propagate (gather), bc on wall rows, collide, store; the three
// edge columns are also written into the opposite halo so the next step needs
// no separate halo refresh.
// ---------------------------------------------------------------------------
template <class S, class A, bool kReg, bool kTape>
__global__ __launch_bounds__(kThreads) void k_fused(const S* __restrict__ src,
                                                    S* __restrict__ dst, Geom g, Phys P,
                                                    double* __restrict__ tape, int by, int bx,
                                                    int nty, unsigned nb) {
  int x, y;
  if (!site_of(g, by, bx, nty, nb, x, y)) return;
  const long long site = padded<S>(g, x + HX, y + g.hy);
  A f[Q];
  gather<S, A>(src, g, site, f);
  if (on_wall_rows(g, y)) wall_site<A>(f, y, g.ly, P.th_bottom, P.th_top, P.rho_ref);
  const Tape4 m = collide<A, kReg>(f, P);
  if (kTape) {
    const long long S2 = (long long)g.lx * g.ly, s = (long long)x * g.ly + y;
    tape[s] = m.rho;
    tape[S2 + s] = m.jx;
    tape[2 * S2 + s] = m.jy;
    tape[3 * S2 + s] = m.e;
  }
  store_site<S, A>(dst, g, site, f);
  if (x < HX) store_site<S, A>(dst, g, site + (long long)g.lx * g.cs, f);
  if (x >= g.lx - HX) store_site<S, A>(dst, g, site - (long long)g.lx * g.cs, f);
}

// Fused step of the local-reference FP32 form: each population is rebuilt in
// FP64 from its deviation and the reference of the site it comes from
// (f_l = M_l(rho_s, th_s of x - e_l) + g_l), then bc, the FP32 collision and
// the store of the new deviations and reference.  Rows beyond the walls hold
// zeros (reference 0: M = 0), which bc replaces.
template <bool kReg, bool kF64Collide>
__global__ __launch_bounds__(kThreads) void k_fused_local(const float* __restrict__ src,
                                                          float* __restrict__ dst, Geom g, Phys P,
                                                          int by, int bx, int nty, unsigned nb) {
  int x, y;
  if (!site_of(g, by, bx, nty, nb, x, y)) return;
  const long long site = padded<float>(g, x + HX, y + g.hy);
  float gv[Q];
  unsigned rv[Q];
#pragma unroll
  for (int l = 0; l < Q; ++l) gv[l] = src[l * g.ps + site - EX[l] * g.cs - EY[l]];
#pragma unroll
  for (int l = 0; l < Q; ++l) rv[l] = ref_at(src, g, site - EX[l] * g.cs - EY[l]);
  __builtin_amdgcn_sched_barrier(0);
  double f[Q];
#pragma unroll
  for (int l = 0; l < Q; ++l) {
    double rho, th;
    unpack_ref(rv[l], rho, th);
    f[l] = rest_maxwellian(l, rho, th) + double(gv[l]);
  }
  if (on_wall_rows(g, y)) wall_site<double>(f, y, g.ly, P.th_bottom, P.th_top, 0.0);
  float v[Q];
  const unsigned ref =
      kF64Collide ? collide_site_local64<kReg>(f, v, P) : collide_site_local<kReg>(f, v, P);
  store_local(dst, g, site, v, ref);
  if (x < HX) store_local(dst, g, site + (long long)g.lx * g.cs, v, ref);
  if (x >= g.lx - HX) store_local(dst, g, site - (long long)g.lx * g.cs, v, ref);
}

// The same step for the column layout, with the loads and stores of the
// tile's own columns addressed through buffer resources: one resource spans
// the padded columns x0 .. x0 + bx + 5 that the tile's gathers read (its
// first column is the tile's first source column), so every load is the
// lane's 32-bit offset (shared by all populations) plus a per-population
// scalar offset and an immediate row shift; no per-lane 64-bit address
// arithmetic.  The lattice-wide halo double-writes keep global stores.
constexpr int kBufferWord3 = 0x00020000;  // raw 32-bit buffer, gfx9 family
constexpr int kNonTemporal = 2;           // cache policy bits of a streaming store

template <bool kReg, bool kF64Collide>
__global__ __launch_bounds__(kThreads) void k_fused_local_col(const float* __restrict__ src,
                                                              float* __restrict__ dst, Geom g,
                                                              Phys P, int by, int bx, int nty,
                                                              unsigned nb) {
  const unsigned t = tile_index(nb);
  const int ty = int(t % unsigned(nty)), tx = int(t / unsigned(nty));
  const int x0 = tx * bx;  // the tile's first column (workgroup-uniform)
  const int lin = threadIdx.x;
  const int y = ty * by + (lin % by), x = x0 + (lin / by);
  if (x >= g.lx || y >= g.ly) return;
  const unsigned cs = unsigned(g.cs), ps = unsigned(g.ps);
  const long long first = (long long)x0 * g.cs;  // padded column x0 = source column x0 - 3
  const unsigned span = unsigned(min((long long)(bx + 2 * HX) * g.cs,
                                     (long long)g.nx * g.cs - first) * 4);
  const __amdgpu_buffer_rsrc_t in =
      __builtin_amdgcn_make_buffer_rsrc((void*)(src + first), (short)0, span, kBufferWord3);
  const unsigned Y = unsigned(y + g.hy);
  const unsigned lane = (unsigned(x - x0) * cs + Y - 3u) * 4u;
  // all 74 loads first (the scheduling barrier keeps the decode from being
  // interleaved with them, which would cap the loads in flight)
  unsigned gv[Q], rv[Q];
#pragma unroll
  for (int l = 0; l < Q; ++l)
    gv[l] = __builtin_amdgcn_raw_buffer_load_b32(
        in, lane + unsigned(3 - EY[l]) * 4u, (unsigned(HX - EX[l]) * cs + unsigned(l) * ps) * 4u, 0);
#pragma unroll
  for (int l = 0; l < Q; ++l)
    rv[l] = __builtin_amdgcn_raw_buffer_load_b32(
        in, lane + unsigned(3 - EY[l]) * 4u, (unsigned(HX - EX[l]) * cs + Q * ps) * 4u, 0);
  __builtin_amdgcn_sched_barrier(0);
  double f[Q];
#pragma unroll
  for (int l = 0; l < Q; ++l) {
    double rho, th;
    unpack_ref(rv[l], rho, th);
    f[l] = rest_maxwellian(l, rho, th) + double(__builtin_bit_cast(float, gv[l]));
  }
  if (on_wall_rows(g, y)) wall_site<double>(f, y, g.ly, P.th_bottom, P.th_top, 0.0);
  float v[Q];
  const unsigned ref =
      kF64Collide ? collide_site_local64<kReg>(f, v, P) : collide_site_local<kReg>(f, v, P);
  const long long own = (long long)(x0 + HX) * g.cs;
  const __amdgpu_buffer_rsrc_t out = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(dst + own), (short)0, unsigned(min((long long)bx * g.cs, (long long)g.nx * g.cs - own) * 4),
      kBufferWord3);
  const unsigned lane_out = (unsigned(x - x0) * cs + Y) * 4u;
#pragma unroll
  for (int l = 0; l < Q; ++l)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v[l]), out, lane_out,
                                          unsigned(l) * ps * 4u, kNonTemporal);
  __builtin_amdgcn_raw_buffer_store_b32(ref, out, lane_out, Q * ps * 4u, kNonTemporal);
  const long long site = padded<float>(g, x + HX, y + g.hy);
  if (x < HX) store_local(dst, g, site + (long long)g.lx * g.cs, v, ref);
  if (x >= g.lx - HX) store_local(dst, g, site - (long long)g.lx * g.cs, v, ref);
}

template <class S>
__global__ __launch_bounds__(kThreads) void k_propagate(const S* __restrict__ src,
                                                        S* __restrict__ dst, Geom g, int by,
                                                        int bx, int nty, unsigned nb) {
  int x, y;
  if (!site_of(g, by, bx, nty, nb, x, y)) return;
  const long long site = padded<S>(g, x + HX, y + g.hy);
#pragma unroll
  for (int l = 0; l < Q; ++l)
    __builtin_nontemporal_store(src[l * g.ps + site - EX[l] * g.cs - EY[l]], &dst[l * g.ps + site]);
}

template <class S, class A, bool kReg>
__global__ __launch_bounds__(kThreads) void k_collide(const S* __restrict__ src,
                                                      S* __restrict__ dst, Geom g, Phys P,
                                                      int by, int bx, int nty, unsigned nb) {
  int x, y;
  if (!site_of(g, by, bx, nty, nb, x, y)) return;
  const long long site = padded<S>(g, x + HX, y + g.hy);
  A f[Q];
  load_site<S, A>(src, g, site, f);
  collide<A, kReg>(f, P);
  store_site<S, A>(dst, g, site, f);
}

// bc on the six wall rows, in place; one thread per (x, wall row).
template <class S>
__global__ __launch_bounds__(kThreads) void k_bc(S* __restrict__ buf, Geom g, Phys P) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= g.lx * 6) return;
  const int x = i / 6, r = i % 6;
  const int y = r < 3 ? r : g.ly - 6 + r;
  const long long site = padded<S>(g, x + HX, y + g.hy);
  double f[Q];
  load_site<S, double>(buf, g, site, f);
  wall_site<double>(f, y, g.ly, P.th_bottom, P.th_top, P.rho_ref);
#pragma unroll
  for (int l = 0; l < Q; ++l) {
    const int ys = y - EY[l];
    if (ys < 0 || ys >= g.ly) buf[l * g.ps + site] = S(f[l]);
  }
}

// Halo columns: X in [0, 3) <- X + lx, X in [lx + 3, lx + 6) <- X - lx, all rows.
template <class S>
__global__ __launch_bounds__(kThreads) void k_halo_x(S* __restrict__ buf, Geom g) {
  const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
  const long long per_l = 6LL * g.ny;
  if (i >= per_l * g.np) return;
  const int l = int(i / per_l);
  const int c = int((i % per_l) / g.ny), Y = int(i % g.ny);
  const int Xd = c < 3 ? c : g.lx + c;
  const int Xs = c < 3 ? g.lx + c : c;
  buf[l * g.ps + (long long)Xd * g.cs + Y] = buf[l * g.ps + (long long)Xs * g.cs + Y];
}

// Halo rows (periodic y only): three rows below and above, all padded columns.
template <class S>
__global__ __launch_bounds__(kThreads) void k_halo_y(S* __restrict__ buf, Geom g) {
  const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
  const long long per_l = 6LL * g.nx;
  if (i >= per_l * g.np) return;
  const int l = int(i / per_l);
  const int X = int((i % per_l) / 6), r = int(i % 6);
  const int Yd = r < 3 ? g.hy - 3 + r : g.hy + g.ly + (r - 3);
  const int Ys = r < 3 ? g.hy + g.ly - 3 + r : g.hy + (r - 3);
  const long long col = l * g.ps + (long long)X * g.cs;
  buf[col + Yd] = buf[col + Ys];
}

// f = f^eq(rho0, u0, T0) - w rho_ref, reconstructed from the Hermite
// coefficients of the Gaussian (no forcing shift at t = 0).
template <class S, class A>
__global__ __launch_bounds__(kThreads) void k_init_feq(S* __restrict__ dst,
                                                       const double* __restrict__ rho,
                                                       const double* __restrict__ ux,
                                                       const double* __restrict__ uy,
                                                       const double* __restrict__ T, Geom g,
                                                       Phys P, int by, int bx, int nty,
                                                       unsigned nb) {
  int x, y;
  if (!site_of(g, by, bx, nty, nb, x, y)) return;
  const long long s = (long long)x * g.ly + y;
  double aeq[5][5];
  equilibrium_coeffs(rho[s], ux[s], uy[s], T[s] - 1.0, aeq);
  aeq[0][0] = rho[s] - P.rho_ref;
  A b[5][5];
#pragma unroll
  for (int p = 0; p < 5; ++p)
#pragma unroll
    for (int q = 0; q + p < 5; ++q) b[p][q] = A(aeq[p][q]);
  A f[Q];
  reconstruct<A>(b, f);
  store_site<S, A>(dst, g, padded<S>(g, x + HX, y + g.hy), f);
}

// f = f^eq(rho0, u0, T0) in the local-reference form.
__global__ __launch_bounds__(kThreads) void k_init_local(float* __restrict__ dst,
                                                        const double* __restrict__ rho,
                                                        const double* __restrict__ ux,
                                                        const double* __restrict__ uy,
                                                        const double* __restrict__ T, Geom g,
                                                        int by, int bx, int nty, unsigned nb) {
  int x, y;
  if (!site_of(g, by, bx, nty, nb, x, y)) return;
  const long long s = (long long)x * g.ly + y;
  double aeq[5][5];
  equilibrium_coeffs(rho[s], ux[s], uy[s], T[s] - 1.0, aeq);
  double f[Q];
  reconstruct<double>(aeq, f);
  float v[Q];
  const unsigned ref = encode_site(f, v);
  store_local(dst, g, padded<float>(g, x + HX, y + g.hy), v, ref);
}

// Eq. (2) in FP64 from the stored populations (FP64, shifted FP32 or the
// local-reference form).
template <class S, class A>
__device__ __forceinline__ Macro site_macro(const S* __restrict__ src, const Geom& g,
                                            long long site, double rho_ref) {
  double f[Q];
  if constexpr (is_local<A>) {
    load_local(src, g, site, f);
    rho_ref = 0.0;
  } else {
    load_site<S, double>(src, g, site, f);
  }
  double a[5][5];
  project<double>(f, a);
  return macro_from(rho_ref + a[0][0], a[1][0], a[0][1], a[2][0], a[0][2]);
}

template <class S, class A>
__global__ __launch_bounds__(kThreads) void k_moments(const S* __restrict__ src,
                                                      double* __restrict__ rho,
                                                      double* __restrict__ ux,
                                                      double* __restrict__ uy,
                                                      double* __restrict__ T, Geom g, Phys P,
                                                      int by, int bx, int nty, unsigned nb) {
  int x, y;
  if (!site_of(g, by, bx, nty, nb, x, y)) return;
  const Macro m = site_macro<S, A>(src, g, padded<S>(g, x + HX, y + g.hy), P.rho_ref);
  const long long s = (long long)x * g.ly + y;
  if (rho) rho[s] = m.rho;
  if (ux) ux[s] = m.ux;
  if (uy) uy[s] = m.uy;
  if (T) T[s] = 1.0 + m.th;
}

template <class S, class A>
__global__ __launch_bounds__(kThreads) void k_check(const S* __restrict__ src,
                                                    unsigned int* __restrict__ flag, Geom g,
                                                    Phys P, int by, int bx, int nty,
                                                    unsigned nb) {
  int x, y;
  if (!site_of(g, by, bx, nty, nb, x, y)) return;
  const long long site = padded<S>(g, x + HX, y + g.hy);
  bool bad = false;
  if constexpr (is_local<A>) {
    double f[Q];
    load_local(src, g, site, f);
#pragma unroll
    for (int l = 0; l < Q; ++l) bad |= !isfinite(f[l]);
  } else {
#pragma unroll
    for (int l = 0; l < Q; ++l) bad |= !isfinite(double(src[l * g.ps + site]));
  }
  const Macro m = site_macro<S, A>(src, g, site, P.rho_ref);
  bad |= !(m.rho > 0.0) || !(1.0 + m.th > 0.0);
  if (bad) atomicAdd(flag, 1u);
}

// compact [37][lx][ly] <-> padded.  One workgroup copies up to kThreads
// consecutive y of one (population, column) row: population blockIdx.y,
// column and y block from blockIdx.x with scalar arithmetic (no per-lane
// 64-bit division).
struct CompactSite {
  long long compact, padded;
  bool in;
  int l;
};

__device__ __forceinline__ CompactSite compact_site(const Geom& g, unsigned nyb) {
  const unsigned x = blockIdx.x / nyb, yb = blockIdx.x - x * nyb;
  const int l = int(blockIdx.y);
  const int y = int(yb) * kThreads + int(threadIdx.x);
  CompactSite c;
  c.in = y < g.ly;
  c.l = l;
  c.compact = ((long long)l * g.lx + x) * g.ly + y;
  c.padded = l * g.ps + (long long)(x + HX) * g.cs + (y + g.hy);
  return c;
}

template <class S>
__global__ __launch_bounds__(kThreads) void k_pack(const S* __restrict__ padded_buf,
                                                   S* __restrict__ compact, Geom g,
                                                   unsigned nyb) {
  const CompactSite c = compact_site(g, nyb);
  if (c.in) __builtin_nontemporal_store(padded_buf[c.padded], &compact[c.compact]);
}

template <class S>
__global__ __launch_bounds__(kThreads) void k_unpack(const S* __restrict__ compact,
                                                     S* __restrict__ padded_buf, Geom g,
                                                     unsigned nyb) {
  const CompactSite c = compact_site(g, nyb);
  if (c.in) __builtin_nontemporal_store(compact[c.compact], &padded_buf[c.padded]);
}

template <class S, class A>
__global__ __launch_bounds__(kThreads) void k_populations_f64(const S* __restrict__ padded_buf,
                                                              double* __restrict__ out, Geom g,
                                                              double rho_ref, unsigned nyb) {
  const CompactSite c = compact_site(g, nyb);
  if (!c.in) return;
  if constexpr (is_local<A>) {
    double rho, th, m = 0.0;
    unpack_ref(ref_at(padded_buf, g, c.padded - c.l * g.ps), rho, th);
#pragma unroll
    for (int k = 0; k < Q; ++k)
      if (k == c.l) m = rest_maxwellian(k, rho, th);
    out[c.compact] = m + double(padded_buf[c.padded]);
  } else {
    double w = 0.0;
#pragma unroll
    for (int k = 0; k < Q; ++k)
      if (k == c.l) w = W[k];
    out[c.compact] = double(padded_buf[c.padded]) + rho_ref * w;
  }
}

__global__ __launch_bounds__(kThreads) void k_zero(unsigned int* __restrict__ p, long long n) {
  const long long stride = (long long)gridDim.x * kThreads;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) p[i] = 0u;
}

// ---------------------------------------------------------------------------
// Adjoint.
// ---------------------------------------------------------------------------

// Block-wide sum of one double per thread; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[kThreads];
  red[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  return red[0];
}

// KE = (1/2) sum rho |u|^2; dKE/df_l = c_l . u - |u|^2 / 2.
__global__ __launch_bounds__(kThreads) void k_loss_ke(const double* __restrict__ src,
                                                      double* __restrict__ lambda,
                                                      double* __restrict__ partials, Geom g,
                                                      int by, int bx, int nty, unsigned nb) {
  int x, y;
  const bool in = site_of(g, by, bx, nty, nb, x, y);
  double ke = 0.0;
  if (in) {
    const Macro m = site_macro<double, double>(src, g, padded<double>(g, x + HX, y + g.hy), 0.0);
    const double u2 = m.ux * m.ux + m.uy * m.uy;
    ke = 0.5 * m.rho * u2;
    if (lambda) {
      const LamStrides ls = lam_strides(g);
      const long long s = (long long)x * ls.cs + y;
#pragma unroll
      for (int l = 0; l < Q; ++l)
        lambda[l * ls.ps + s] = R * (EX[l] * m.ux + EY[l] * m.uy) - 0.5 * u2;
    }
  }
  const double tot = block_sum(ke);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kThreads) void k_sum(const double* __restrict__ partials, int n,
                                                  double* __restrict__ out) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) v += partials[i];
  const double tot = block_sum(v);
  if (threadIdx.x == 0) *out = tot;
}

// Gradient of a^eq_pq = rho h_p(Ux) h_q(Uy) contracted with L_pq:
// returns (dRho, dUx, dUy, dTh).
struct EqGrad {
  double rho, ux, uy, th;
};

__device__ __forceinline__ EqGrad equilibrium_grad(const double (&L)[5][5], double rho,
                                                   double Ux, double Uy, double th) {
  double hx[5], hy[5], dxU[5], dxT[5], dyU[5], dyT[5];
  gauss_hermite(Ux, th, hx);
  gauss_hermite(Uy, th, hy);
  gauss_hermite_d(Ux, th, dxU, dxT);
  gauss_hermite_d(Uy, th, dyU, dyT);
  EqGrad e{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int p = 0; p < 5; ++p)
#pragma unroll
    for (int q = 0; q + p < 5; ++q) {
      e.rho += L[p][q] * hx[p] * hy[q];
      e.ux += L[p][q] * dxU[p] * hy[q];
      e.uy += L[p][q] * hx[p] * dyU[q];
      e.th += L[p][q] * (dxT[p] * hy[q] + hx[p] * dyT[q]);
    }
  e.ux *= rho;
  e.uy *= rho;
  e.th *= rho;
  return e;
}

// L_pq = sum_l lambda_l w_l H_pq(c_l) / (p! q!)
__device__ __forceinline__ void adjoint_project(const double (&lam)[Q], double (&L)[5][5]) {
  double lw[Q];
#pragma unroll
  for (int l = 0; l < Q; ++l) lw[l] = lam[l] * W[l];
  project<double>(lw, L);
#pragma unroll
  for (int p = 0; p < 5; ++p)
#pragma unroll
    for (int q = 0; q + p < 5; ++q) L[p][q] *= INVFAC[p] * INVFAC[q];
}

// lambda_out = P^T B^T C^T lambda_in for one step (scatter form).
// B^T C(m)^T of one site: lam holds lambda^{j+1} at the site's arriving
// populations, m = (rho, j_x, j_y, sum |c|^2 f) the pre-collision moments of
// step j; on return mu holds the adjoint of the propagated populations
// (zero for those a wall supplied).
template <bool kReg>
__device__ __forceinline__ void adjoint_site(const double (&lam)[Q], double rho, double jx,
                                             double jy, double e, const Geom& g, const Phys& P,
                                             int y, double (&mu)[Q]) {
  const double inv = 1.0 / rho;
  const double ux = jx * inv, uy = jy * inv;
  const double u2 = ux * ux + uy * uy;
  const double th = 0.5 * e * inv - 1.0 - 0.5 * u2;
  // C^T: the collision as a function of the pre-collision populations.
  double L[5][5];
  adjoint_project(lam, L);
  double Lw[5][5];
#pragma unroll
  for (int p = 0; p < 5; ++p)
#pragma unroll
    for (int q = 0; q + p < 5; ++q) Lw[p][q] = P.omega * L[p][q];
  const EqGrad G =
      equilibrium_grad(Lw, rho, ux + P.tau_gx, uy + P.tau_gy, th + P.dtheta);
  const double g00 = G.rho - (ux * G.ux + uy * G.uy) * inv + G.th * (0.5 * u2 - th) * inv;
  const double g10 = (G.ux - ux * G.th) * inv;
  const double g01 = (G.uy - uy * G.th) * inv;
  const double ge2 = 0.5 * G.th * inv;
  double B[5][5];
  const double keep = 1.0 - P.omega;
#pragma unroll
  for (int p = 0; p < 5; ++p)
#pragma unroll
    for (int q = 0; q + p < 5; ++q) B[p][q] = kReg ? keep * L[p][q] : 0.0;
  B[0][0] += g00;
  B[1][0] += g10;
  B[0][1] += g01;
  B[2][0] += ge2;
  B[0][2] += ge2;
  expand<double>(B, mu);
  if (!kReg) {
#pragma unroll
    for (int l = 0; l < Q; ++l) mu[l] += keep * lam[l];
  }
  // B^T: on wall rows the unknown populations were rho_w v_l with
  // rho_w = sum_K f / sum_K v.
  if (on_wall_rows(g, y)) {
    const double thw = y < 3 ? P.th_bottom : P.th_top;
    double vk = 0.0, su = 0.0;
#pragma unroll
    for (int l = 0; l < Q; ++l) {
      const int ys = y - EY[l];
      const bool unknown = ys < 0 || ys >= g.ly;
      const double v = wall_feq(l, thw);
      if (unknown)
        su += mu[l] * v;
      else
        vk += v;
    }
    const double add = su / vk;
#pragma unroll
    for (int l = 0; l < Q; ++l) {
      const int ys = y - EY[l];
      const bool unknown = ys < 0 || ys >= g.ly;
      mu[l] = unknown ? 0.0 : mu[l] + add;
    }
  }
}

template <bool kReg>
__global__ __launch_bounds__(kThreads) void k_adjoint(const double* __restrict__ tape,
                                                      const double* __restrict__ lam_in,
                                                      double* __restrict__ lam_out, Geom g,
                                                      Phys P, int by, int bx, int nty,
                                                      unsigned nb) {
  int x, y;
  if (!site_of(g, by, bx, nty, nb, x, y)) return;
  // tape: [4][lx][ly]; lambda: compact, in the lattice's layout
  const long long S2 = (long long)g.lx * g.ly, s = (long long)x * g.ly + y;
  const LamStrides ls = lam_strides(g);
  const long long sl = (long long)x * ls.cs + y;
  double lam[Q];
#pragma unroll
  for (int l = 0; l < Q; ++l) lam[l] = lam_in[l * ls.ps + sl];
  double mu[Q];
  adjoint_site<kReg>(lam, tape[s], tape[S2 + s], tape[2 * S2 + s], tape[3 * S2 + s], g, P, y,
                     mu);
  // P^T: the population that arrived here came from (x - e_lx, y - e_ly).
#pragma unroll
  for (int l = 0; l < Q; ++l) {
    const int ys = y - EY[l];
    if (g.walls && (ys < 0 || ys >= g.ly)) continue;
    int xs = x - EX[l];
    xs += xs < 0 ? g.lx : (xs >= g.lx ? -g.lx : 0);
    int yd = ys;
    if (!g.walls) yd += yd < 0 ? g.ly : (yd >= g.ly ? -g.ly : 0);
    lam_out[l * ls.ps + (long long)xs * ls.cs + yd] = mu[l];
  }
  // Populations leaving through a wall from this site reach no site: zero.
  if (on_wall_rows(g, y)) {
#pragma unroll
    for (int l = 0; l < Q; ++l) {
      const int yd = y + EY[l];
      if (yd < 0 || yd >= g.ly) lam_out[l * ls.ps + sl] = 0.0;
    }
  }
}

// Gather form of a run of adjoint steps.  mu^j = B^T C(m_j)^T lambda^{j+1}
// is kept where the populations arrived, in a padded buffer laid out like the
// state (x halos written by the edge columns, rows beyond the walls zero), and
// P^T is applied when the next kernel reads it:
// lambda^j_l(z) = mu^j_l(z + e_l).  So every load is a shifted coalesced read
// and every store is aligned, as in the forward step.  kFromCompact: the
// first kernel of a run reads lambda^{j+1} itself from a compact array.
template <bool kReg, bool kFromCompact>
__global__ __launch_bounds__(kThreads) void k_adjoint_mu(const double* __restrict__ tape,
                                                         const double* __restrict__ in,
                                                         double* __restrict__ mu_out, Geom g,
                                                         Phys P, int by, int bx, int nty,
                                                         unsigned nb) {
  int x, y;
  if (!site_of(g, by, bx, nty, nb, x, y)) return;
  const long long S2 = (long long)g.lx * g.ly, s = (long long)x * g.ly + y;
  const long long site = padded<double>(g, x + HX, y + g.hy);
  double lam[Q];
  if (kFromCompact) {
    const LamStrides ls = lam_strides(g);
    const long long sl = (long long)x * ls.cs + y;
#pragma unroll
    for (int l = 0; l < Q; ++l) lam[l] = in[l * ls.ps + sl];
  } else {
#pragma unroll
    for (int l = 0; l < Q; ++l) lam[l] = in[l * g.ps + site + EX[l] * g.cs + EY[l]];
  }
  double mu[Q];
  adjoint_site<kReg>(lam, tape[s], tape[S2 + s], tape[2 * S2 + s], tape[3 * S2 + s], g, P, y,
                     mu);
  store_site<double, double>(mu_out, g, site, mu);
  if (x < HX) store_site<double, double>(mu_out, g, site + (long long)g.lx * g.cs, mu);
  if (x >= g.lx - HX) store_site<double, double>(mu_out, g, site - (long long)g.lx * g.cs, mu);
}

// Last kernel of a run: lambda^j_l(z) = mu^j_l(z + e_l) into a compact array.
__global__ __launch_bounds__(kThreads) void k_adjoint_gather(const double* __restrict__ mu,
                                                             double* __restrict__ lam, Geom g,
                                                             int by, int bx, int nty,
                                                             unsigned nb) {
  int x, y;
  if (!site_of(g, by, bx, nty, nb, x, y)) return;
  const long long site = padded<double>(g, x + HX, y + g.hy);
  const LamStrides ls = lam_strides(g);
  const long long sl = (long long)x * ls.cs + y;
#pragma unroll
  for (int l = 0; l < Q; ++l)
    __builtin_nontemporal_store(mu[l * g.ps + site + EX[l] * g.cs + EY[l]], &lam[l * ls.ps + sl]);
}

// Zero the rows beyond the walls (padded rows outside [0, ly)) of every
// padded column: there the gather of the adjoint reads the zero that a
// population leaving the lattice contributes, and the state buffers get
// finite values in the rows that no step writes.
template <class S>
__global__ __launch_bounds__(kThreads) void k_zero_pad_rows(S* __restrict__ buf, Geom g) {
  const int pad = g.ny - g.ly;  // hy rows below, ny - ly - hy above
  const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
  const long long n = (long long)g.np * g.nx * pad;
  if (i >= n) return;
  const int r = int(i % pad);
  const long long lx_ = i / pad;
  const int l = int(lx_ / g.nx), X = int(lx_ % g.nx);
  const int Y = r < g.hy ? r : g.ly + r;
  buf[l * g.ps + (long long)X * g.cs + Y] = S(0);
}

__global__ __launch_bounds__(kThreads) void k_init_adjoint(
    const double* __restrict__ lam0, const double* __restrict__ rho,
    const double* __restrict__ ux, const double* __restrict__ uy, const double* __restrict__ T,
    double* __restrict__ drho, double* __restrict__ dux, double* __restrict__ duy,
    double* __restrict__ dT, Geom g, int by, int bx, int nty, unsigned nb) {
  int x, y;
  if (!site_of(g, by, bx, nty, nb, x, y)) return;
  const LamStrides ls = lam_strides(g);
  const long long s = (long long)x * g.ly + y, sl = (long long)x * ls.cs + y;
  double lam[Q];
#pragma unroll
  for (int l = 0; l < Q; ++l) lam[l] = lam0[l * ls.ps + sl];
  double L[5][5];
  adjoint_project(lam, L);
  const EqGrad G = equilibrium_grad(L, rho[s], ux[s], uy[s], T[s] - 1.0);
  if (drho) drho[s] = G.rho;
  if (dux) dux[s] = G.ux;
  if (duy) duy[s] = G.uy;
  if (dT) dT[s] = G.th;
}

// ---------------------------------------------------------------------------
// In-situ observables: row averages over x and lattice totals.
// ---------------------------------------------------------------------------

// partial[c][k][y] = sum over the columns of chunk c of the k-th per-site
// observable at row y: rho, u_x, u_y, T, rho |u|^2 / 2, rho T.
template <class S, class A>
__global__ __launch_bounds__(kThreads) void k_obs_rows(const S* __restrict__ src,
                                                       double* __restrict__ partial, Geom g,
                                                       Phys P, int nchunks) {
  const int y = blockIdx.x * kThreads + threadIdx.x;
  const int c = blockIdx.y;
  if (y >= g.ly) return;
  const int x0 = int((long long)g.lx * c / nchunks), x1 = int((long long)g.lx * (c + 1) / nchunks);
  double acc[kObservables] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int x = x0; x < x1; ++x) {
    const Macro m = site_macro<S, A>(src, g, (long long)(x + HX) * g.cs + (y + g.hy), P.rho_ref);
    const double T = 1.0 + m.th;
    acc[0] += m.rho;
    acc[1] += m.ux;
    acc[2] += m.uy;
    acc[3] += T;
    acc[4] += 0.5 * m.rho * (m.ux * m.ux + m.uy * m.uy);
    acc[5] += m.rho * T;
  }
#pragma unroll
  for (int k = 0; k < kObservables; ++k)
    partial[((long long)c * kObservables + k) * g.ly + y] = acc[k];
}

// profiles[k][y] = (sum over chunks of partial[c][k][y]) / lx, in chunk order.
__global__ __launch_bounds__(kThreads) void k_obs_reduce(const double* __restrict__ partial,
                                                         double* __restrict__ profiles, int lx,
                                                         int ly, int nchunks) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= kObservables * ly) return;
  double s = 0.0;
  for (int c = 0; c < nchunks; ++c) s += partial[(long long)c * kObservables * ly + i];
  profiles[i] = s / lx;
}

// scalars: mass, kinetic energy, sum rho T, mixing-layer width
// 6 sum_y phi (1 - phi), phi = (Tbar(y) - T_top) / (T_bottom - T_top) in [0, 1].
__global__ __launch_bounds__(kThreads) void k_obs_scalars(const double* __restrict__ profiles,
                                                          double* __restrict__ scalars, int lx,
                                                          int ly, double t_bottom, double t_top) {
  double m = 0.0, ke = 0.0, e = 0.0, w = 0.0;
  const double dT = t_bottom - t_top;
  for (int y = threadIdx.x; y < ly; y += kThreads) {
    m += profiles[0 * ly + y];
    ke += profiles[4 * ly + y];
    e += profiles[5 * ly + y];
    if (dT != 0.0) {
      double phi = (profiles[3 * ly + y] - t_top) / dT;
      phi = phi < 0.0 ? 0.0 : (phi > 1.0 ? 1.0 : phi);
      w += phi * (1.0 - phi);
    }
  }
  m = block_sum(m);
  __syncthreads();
  ke = block_sum(ke);
  __syncthreads();
  e = block_sum(e);
  __syncthreads();
  w = block_sum(w);
  if (threadIdx.x == 0) {
    scalars[0] = m * lx;
    scalars[1] = ke * lx;
    scalars[2] = e * lx;
    scalars[3] = 6.0 * w;
  }
}

unsigned grid_1d(long long n) { return unsigned((n + kThreads - 1) / kThreads); }

}  // namespace

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------

// Calls fn(S{}, A{}) with the storage type S and the arithmetic type A of a
// precision mode -> (storage type, accumulation type): FP64 storage and
// collision; shifted FP32 storage with the FP64 collision; shifted FP32
// storage with FP32 Hermite sums; the local-reference FP32 form with the
// FP32 collision (LocalRef) or the FP64 collision (LocalRef64).
// Moments, equilibrium coefficients and bc are FP64 in every mode.
template <class Fn>
hipError_t by_precision(int prec, Fn fn) {
  if (prec == kF64)
    fn(double{}, double{});
  else if (prec == kF32Shifted)
    fn(float{}, double{});
  else if (prec == kF32ShiftedF32Sum)
    fn(float{}, float{});
  else if (prec == kF32Collide)
    fn(float{}, LocalRef{});
  else
    fn(float{}, LocalRef64{});
  return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  const long long n = (long long)(bytes / 4);
  if (n == 0) return hipSuccess;
  const unsigned grid = std::min(grid_1d(n), 1u << 20);  // grid-stride beyond 2^28 words
  hipLaunchKernelGGL(k_zero, dim3(grid), dim3(kThreads), 0, s,
                     static_cast<unsigned int*>(p), n);
  return hipGetLastError();
}

hipError_t launch_halo(void* buf, const Geom& g, int prec, hipStream_t s) {
  const long long nx_el = 6LL * g.ny * g.np, ny_el = 6LL * g.nx * g.np;
  return by_precision(prec, [&](auto sv, auto) {
    using S = decltype(sv);
    hipLaunchKernelGGL(k_halo_x<S>, dim3(grid_1d(nx_el)), dim3(kThreads), 0, s,
                       static_cast<S*>(buf), g);
    if (!g.walls)
      hipLaunchKernelGGL(k_halo_y<S>, dim3(grid_1d(ny_el)), dim3(kThreads), 0, s,
                         static_cast<S*>(buf), g);
  });
}

hipError_t launch_fused(const void* src, void* dst, const Geom& g, const Phys& p, int prec,
                        int regularize, double* tape, hipStream_t s) {
  if (tape && prec != kF64) return hipErrorInvalidValue;
  const Tiling t = make_tiling(g.lx, g.ly);
  return by_precision(prec, [&](auto sv, auto av) {
    using S = decltype(sv);
    using A = decltype(av);
    const S* a = static_cast<const S*>(src);
    S* b = static_cast<S*>(dst);
    const dim3 grid(t.nb), block(kThreads);
    if constexpr (is_local<A>) {
      // column layout: buffer-addressed kernel (its per-tile resources span
      // bx + 6 columns, which must fit the 32-bit byte range of a buffer
      // resource); SoA, or columns too tall for that: global addressing
      constexpr bool k64 = A::f64_collide;
      const bool column = g.ps < g.cs &&
                          (long long)(t.bx + 2 * HX) * g.cs * (long long)sizeof(float) < (1LL << 32);
      if (column && regularize)
        hipLaunchKernelGGL((k_fused_local_col<true, k64>), grid, block, 0, s, a, b, g, p, t.by,
                           t.bx, t.nty, t.nb);
      else if (column)
        hipLaunchKernelGGL((k_fused_local_col<false, k64>), grid, block, 0, s, a, b, g, p, t.by,
                           t.bx, t.nty, t.nb);
      else if (regularize)
        hipLaunchKernelGGL((k_fused_local<true, k64>), grid, block, 0, s, a, b, g, p, t.by, t.bx,
                           t.nty, t.nb);
      else
        hipLaunchKernelGGL((k_fused_local<false, k64>), grid, block, 0, s, a, b, g, p, t.by,
                           t.bx, t.nty, t.nb);
    } else if (regularize && tape)
      hipLaunchKernelGGL((k_fused<S, A, true, true>), grid, block, 0, s, a, b, g, p, tape, t.by,
                         t.bx, t.nty, t.nb);
    else if (regularize)
      hipLaunchKernelGGL((k_fused<S, A, true, false>), grid, block, 0, s, a, b, g, p, tape,
                         t.by, t.bx, t.nty, t.nb);
    else if (tape)
      hipLaunchKernelGGL((k_fused<S, A, false, true>), grid, block, 0, s, a, b, g, p, tape,
                         t.by, t.bx, t.nty, t.nb);
    else
      hipLaunchKernelGGL((k_fused<S, A, false, false>), grid, block, 0, s, a, b, g, p, tape,
                         t.by, t.bx, t.nty, t.nb);
  });
}

hipError_t launch_propagate(const void* src, void* dst, const Geom& g, int prec,
                            hipStream_t s) {
  const Tiling t = make_tiling(g.lx, g.ly);
  return by_precision(prec, [&](auto sv, auto) {
    using S = decltype(sv);
    hipLaunchKernelGGL(k_propagate<S>, dim3(t.nb), dim3(kThreads), 0, s,
                       static_cast<const S*>(src), static_cast<S*>(dst), g, t.by, t.bx, t.nty,
                       t.nb);
  });
}

hipError_t launch_bc(void* buf, const Geom& g, const Phys& p, int prec, hipStream_t s) {
  if (!g.walls) return hipSuccess;
  const unsigned grid = grid_1d(6LL * g.lx);
  return by_precision(prec, [&](auto sv, auto) {
    using S = decltype(sv);
    hipLaunchKernelGGL(k_bc<S>, dim3(grid), dim3(kThreads), 0, s, static_cast<S*>(buf), g, p);
  });
}

hipError_t launch_collide(const void* src, void* dst, const Geom& g, const Phys& p, int prec,
                          int regularize, hipStream_t s) {
  const Tiling t = make_tiling(g.lx, g.ly);
  return by_precision(prec, [&](auto sv, auto av) {
    using S = decltype(sv);
    using A = decltype(av);
    const S* a = static_cast<const S*>(src);
    S* b = static_cast<S*>(dst);
    if constexpr (is_local<A>)
      return;  // the local-reference form has no split collide (lb_api rejects it)
    else if (regularize)
      hipLaunchKernelGGL((k_collide<S, A, true>), dim3(t.nb), dim3(kThreads), 0, s, a, b, g, p,
                         t.by, t.bx, t.nty, t.nb);
    else
      hipLaunchKernelGGL((k_collide<S, A, false>), dim3(t.nb), dim3(kThreads), 0, s, a, b, g,
                         p, t.by, t.bx, t.nty, t.nb);
  });
}

hipError_t launch_init_feq(void* dst, const double* rho, const double* ux, const double* uy,
                           const double* T, const Geom& g, const Phys& p, int prec,
                           hipStream_t s) {
  const Tiling t = make_tiling(g.lx, g.ly);
  return by_precision(prec, [&](auto sv, auto av) {
    using S = decltype(sv);
    if constexpr (is_local<decltype(av)>)
      hipLaunchKernelGGL(k_init_local, dim3(t.nb), dim3(kThreads), 0, s, static_cast<float*>(dst),
                         rho, ux, uy, T, g, t.by, t.bx, t.nty, t.nb);
    else
      hipLaunchKernelGGL((k_init_feq<S, double>), dim3(t.nb), dim3(kThreads), 0, s,
                         static_cast<S*>(dst), rho, ux, uy, T, g, p, t.by, t.bx, t.nty, t.nb);
  });
}

hipError_t launch_moments(const void* src, double* rho, double* ux, double* uy, double* T,
                          const Geom& g, const Phys& p, int prec, hipStream_t s) {
  const Tiling t = make_tiling(g.lx, g.ly);
  return by_precision(prec, [&](auto sv, auto av) {
    using S = decltype(sv);
    hipLaunchKernelGGL((k_moments<S, decltype(av)>), dim3(t.nb), dim3(kThreads), 0, s,
                       static_cast<const S*>(src), rho, ux, uy, T, g, p, t.by, t.bx, t.nty,
                       t.nb);
  });
}

// workgroups of the compact copies: lx columns of ceil(ly / kThreads) blocks
// along x, the 37 populations along y
struct CompactGrid {
  dim3 grid;
  unsigned nyb;
};

CompactGrid compact_grid(const Geom& g, int planes) {
  const unsigned nyb = unsigned((g.ly + kThreads - 1) / kThreads);
  return {dim3(unsigned(g.lx) * nyb, unsigned(planes)), nyb};
}

hipError_t launch_pack(const void* padded_buf, void* compact, const Geom& g, int prec,
                       hipStream_t s) {
  const CompactGrid cg = compact_grid(g, g.np);
  return by_precision(prec, [&](auto sv, auto) {
    using S = decltype(sv);
    hipLaunchKernelGGL(k_pack<S>, cg.grid, dim3(kThreads), 0, s,
                       static_cast<const S*>(padded_buf), static_cast<S*>(compact), g, cg.nyb);
  });
}

hipError_t launch_unpack(const void* compact, void* padded_buf, const Geom& g, int prec,
                         hipStream_t s) {
  const CompactGrid cg = compact_grid(g, g.np);
  return by_precision(prec, [&](auto sv, auto) {
    using S = decltype(sv);
    hipLaunchKernelGGL(k_unpack<S>, cg.grid, dim3(kThreads), 0, s,
                       static_cast<const S*>(compact), static_cast<S*>(padded_buf), g, cg.nyb);
  });
}

hipError_t launch_populations_f64(const void* padded_buf, double* out, const Geom& g,
                                  const Phys& p, int prec, hipStream_t s) {
  const CompactGrid cg = compact_grid(g, Q);
  return by_precision(prec, [&](auto sv, auto av) {
    using S = decltype(sv);
    hipLaunchKernelGGL((k_populations_f64<S, decltype(av)>), cg.grid, dim3(kThreads), 0, s,
                       static_cast<const S*>(padded_buf), out, g, p.rho_ref, cg.nyb);
  });
}

hipError_t launch_check(const void* src, unsigned int* flag, const Geom& g, const Phys& p,
                        int prec, hipStream_t s) {
  const Tiling t = make_tiling(g.lx, g.ly);
  return by_precision(prec, [&](auto sv, auto av) {
    using S = decltype(sv);
    hipLaunchKernelGGL((k_check<S, decltype(av)>), dim3(t.nb), dim3(kThreads), 0, s, static_cast<const S*>(src),
                       flag, g, p, t.by, t.bx, t.nty, t.nb);
  });
}

int observable_chunks(const Geom& g) { return g.lx < 64 ? g.lx : 64; }

hipError_t launch_observables(const void* src, double* partial, double* profiles,
                              double* scalars, const Geom& g, const Phys& p, int prec,
                              double t_bottom, double t_top, hipStream_t s) {
  const int nc = observable_chunks(g);
  hipError_t e = by_precision(prec, [&](auto sv, auto av) {
    using S = decltype(sv);
    hipLaunchKernelGGL((k_obs_rows<S, decltype(av)>), dim3(grid_1d(g.ly), nc), dim3(kThreads), 0, s,
                       static_cast<const S*>(src), partial, g, p, nc);
  });
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_obs_reduce, dim3(grid_1d((long long)kObservables * g.ly)), dim3(kThreads),
                     0, s, partial, profiles, g.lx, g.ly, nc);
  e = hipGetLastError();
  if (e != hipSuccess || !scalars) return e;
  hipLaunchKernelGGL(k_obs_scalars, dim3(1), dim3(kThreads), 0, s, profiles, scalars, g.lx, g.ly,
                     t_bottom, t_top);
  return hipGetLastError();
}

int loss_ke_blocks(const Geom& g) { return int(make_tiling(g.lx, g.ly).nb); }

hipError_t launch_loss_ke(const void* src, double* ke, double* lambda, double* partials,
                          const Geom& g, hipStream_t s) {
  const Tiling t = make_tiling(g.lx, g.ly);
  hipLaunchKernelGGL(k_loss_ke, dim3(t.nb), dim3(kThreads), 0, s,
                     static_cast<const double*>(src), lambda, partials, g, t.by, t.bx, t.nty,
                     t.nb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(kThreads), 0, s, partials, int(t.nb), ke);
  return hipGetLastError();
}

hipError_t launch_adjoint_step(const double* tape, const double* lam_in, double* lam_out,
                               const Geom& g, const Phys& p, int regularize, hipStream_t s) {
  const Tiling t = make_tiling(g.lx, g.ly);
  if (regularize)
    hipLaunchKernelGGL(k_adjoint<true>, dim3(t.nb), dim3(kThreads), 0, s, tape, lam_in, lam_out,
                       g, p, t.by, t.bx, t.nty, t.nb);
  else
    hipLaunchKernelGGL(k_adjoint<false>, dim3(t.nb), dim3(kThreads), 0, s, tape, lam_in,
                       lam_out, g, p, t.by, t.bx, t.nty, t.nb);
  return hipGetLastError();
}

hipError_t launch_adjoint_mu(const double* tape, const double* in, bool from_compact, double* mu_out,
                             const Geom& g, const Phys& p, int regularize, hipStream_t s) {
  const Tiling t = make_tiling(g.lx, g.ly);
  const dim3 grid(t.nb), block(kThreads);
  if (regularize && from_compact)
    hipLaunchKernelGGL((k_adjoint_mu<true, true>), grid, block, 0, s, tape, in, mu_out, g, p, t.by,
                       t.bx, t.nty, t.nb);
  else if (regularize)
    hipLaunchKernelGGL((k_adjoint_mu<true, false>), grid, block, 0, s, tape, in, mu_out, g, p,
                       t.by, t.bx, t.nty, t.nb);
  else if (from_compact)
    hipLaunchKernelGGL((k_adjoint_mu<false, true>), grid, block, 0, s, tape, in, mu_out, g, p,
                       t.by, t.bx, t.nty, t.nb);
  else
    hipLaunchKernelGGL((k_adjoint_mu<false, false>), grid, block, 0, s, tape, in, mu_out, g, p,
                       t.by, t.bx, t.nty, t.nb);
  return hipGetLastError();
}

hipError_t launch_adjoint_gather(const double* mu, double* lam, const Geom& g, hipStream_t s) {
  const Tiling t = make_tiling(g.lx, g.ly);
  hipLaunchKernelGGL(k_adjoint_gather, dim3(t.nb), dim3(kThreads), 0, s, mu, lam, g, t.by, t.bx,
                     t.nty, t.nb);
  return hipGetLastError();
}

hipError_t launch_zero_pad_rows(void* buf, const Geom& g, int prec, hipStream_t s) {
  const long long n = (long long)g.np * g.nx * (g.ny - g.ly);
  return by_precision(prec, [&](auto sv, auto) {
    using S = decltype(sv);
    hipLaunchKernelGGL(k_zero_pad_rows<S>, dim3(grid_1d(n)), dim3(kThreads), 0, s,
                       static_cast<S*>(buf), g);
  });
}

hipError_t launch_init_adjoint(const double* lam0, const double* rho, const double* ux,
                               const double* uy, const double* T, double* drho, double* dux,
                               double* duy, double* dT, const Geom& g, hipStream_t s) {
  const Tiling t = make_tiling(g.lx, g.ly);
  hipLaunchKernelGGL(k_init_adjoint, dim3(t.nb), dim3(kThreads), 0, s, lam0, rho, ux, uy, T,
                     drho, dux, duy, dT, g, t.by, t.bx, t.nty, t.nb);
  return hipGetLastError();
}

}  // namespace d2q37
