// Alternative kernels for two stages of the split step, kept so that the
// design choices of the main kernels can be measured against them on the
// same lattice (they compute the same values: propagate bit for bit, collide
// to FP64 rounding):
//
//  * k_propagate_lds: propagate with every population's source window (the
//    tile's rows plus the three-row halo on each side, Sec. 2: hops of up to
//    three sites) staged through LDS, so that all global loads of a
//    population are the same aligned row segment whatever its y hop;
//  * k_propagate_wide: propagate with 16-byte accesses (two FP64 or four FP32
//    sites per thread);
//  * k_collide_mfma: the FP64 collision with its Hermite projection and
//    reconstruction (Sec. 2) as dense products on the FP64 matrix cores.
//
// The main path reads each population straight into registers with one
// 4- or 8-byte access per site and does both Hermite sums as separable vector
// sums; these kernels are the alternatives that choice is measured against.
#include <hip/hip_runtime.h>

#include "d2q37_device.h"
#include "d2q37_launch.h"

namespace d2q37 {
namespace {

constexpr int kVThreads = 256;

// ---------------------------------------------------------------------------
// Propagate through LDS.  One workgroup: `kVThreads` consecutive rows
// y0 .. y0 + n - 1 of one column x (n < kVThreads only at the top of the
// lattice).  Populations are staged in two groups (19 + 18) so that one
// group's windows fit the 64 KB of LDS a workgroup may hold in FP64:
// window of population l = rows y0 - 3 .. y0 + n + 2 of source column
// x - e_lx; thread t loads row y0 + t of every window (one aligned row
// segment per population and wave), and the six halo rows of every window are
// loaded by the first 6 * (group size) threads.  After a barrier, thread t
// reads row t + 3 - e_ly of window l: f_l(x, y0 + t) = src(l, x - e_lx,
// y0 + t - e_ly).
// ---------------------------------------------------------------------------
constexpr int kLdsGroup = 19;
constexpr int kLdsRows = kVThreads + 6;

template <class S>
__global__ __launch_bounds__(kVThreads) void k_propagate_lds(const S* __restrict__ src,
                                                             S* __restrict__ dst, Geom g,
                                                             int nty) {
  __shared__ S win[kLdsGroup * kLdsRows];
  const int x = int(blockIdx.x) / nty;
  const int y0 = (int(blockIdx.x) % nty) * kVThreads;
  const int n = min(kVThreads, g.ly - y0);
  const int t = threadIdx.x;
  const long long row0 = (long long)(g.hy + y0);  // padded row of y0
  const long long own = (long long)(x + HX) * g.cs + row0;
#pragma unroll
  for (int l0 = 0; l0 < Q; l0 += kLdsGroup) {
    const int cnt = min(kLdsGroup, Q - l0);
    // main rows
    if (t < n) {
#pragma unroll
      for (int i = 0; i < kLdsGroup; ++i) {
        if (i < cnt) {
          const int l = l0 + i;
          win[i * kLdsRows + 3 + t] = src[l * g.ps + own - EX[l] * g.cs + t];
        }
      }
    }
    // halo rows: 3 below y0 and 3 above y0 + n - 1 of every window
    if (t < 6 * cnt) {
      const int i = t / 6, h = t % 6;
      const int l = l0 + i;
      const int r = h < 3 ? h - 3 : n + (h - 3);  // row offset from y0
      int ex = 0;
#pragma unroll
      for (int k = 0; k < Q; ++k) ex = (k == l) ? EX[k] : ex;
      win[i * kLdsRows + 3 + r] = src[l * g.ps + own - ex * g.cs + r];
    }
    __syncthreads();
    if (t < n) {
#pragma unroll
      for (int i = 0; i < kLdsGroup; ++i) {
        if (i < cnt) {
          const int l = l0 + i;
          __builtin_nontemporal_store(win[i * kLdsRows + 3 + t - EY[l]], &dst[l * g.ps + own + t]);
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Propagate with 16-byte accesses: thread t of a workgroup handles the
// V = 16 / sizeof(S) rows y0 + V t .. y0 + V t + V - 1 of one column.  The
// destination vector is 16-byte aligned (padded rows and columns are
// 256-byte aligned); the source vector is shifted by -e_ly rows and so only
// element aligned (the unaligned-access mode of the HSA runtime serves it).
// A vector that runs past row ly - 1 (ragged top) stores element by element.
// ---------------------------------------------------------------------------
template <class S>
struct Wide;
template <>
struct Wide<double> {
  typedef double vec __attribute__((ext_vector_type(2)));
  typedef vec vec_u __attribute__((aligned(8)));
  static constexpr int V = 2;
};
template <>
struct Wide<float> {
  typedef float vec __attribute__((ext_vector_type(4)));
  typedef vec vec_u __attribute__((aligned(4)));
  static constexpr int V = 4;
};

template <class S>
__global__ __launch_bounds__(kVThreads) void k_propagate_wide(const S* __restrict__ src,
                                                              S* __restrict__ dst, Geom g,
                                                              int nty) {
  using W = Wide<S>;
  constexpr int V = W::V;
  const int x = int(blockIdx.x) / nty;
  const int y = (int(blockIdx.x) % nty) * (kVThreads * V) + V * int(threadIdx.x);
  if (y >= g.ly) return;
  const long long own = (long long)(x + HX) * g.cs + g.hy + y;
  typename W::vec v[Q];
#pragma unroll
  for (int l = 0; l < Q; ++l)
    v[l] = *reinterpret_cast<const typename W::vec_u*>(src + l * g.ps + own - EX[l] * g.cs - EY[l]);
  if (y + V <= g.ly) {
#pragma unroll
    for (int l = 0; l < Q; ++l)
      __builtin_nontemporal_store(v[l], reinterpret_cast<typename W::vec*>(dst + l * g.ps + own));
  } else {
#pragma unroll
    for (int l = 0; l < Q; ++l)
#pragma unroll
      for (int e = 0; e < V; ++e)
        if (y + e < g.ly) dst[l * g.ps + own + e] = v[l][e];
  }
}

// ---------------------------------------------------------------------------
// FP64 collision on the matrix cores.
//
// v_mfma_f64_16x16x4_f64 computes D = A B + C for A 16 x 4, B 4 x 16 and
// C, D 16 x 16.  Lane L = 16 G + J (G = 0..3, J = 0..15) holds A[J][G],
// B[G][J] and D[G + 4 r][J] in its r-th result register (the rows of a
// result register interleave over the lane groups).  A wave collides
// 64 consecutive rows of one column as four sets of 16 sites, site J of a
// set in column J of B and D:
//   projection      D[row][site] = sum_l Hp[row][l] f_l(site): 10 products
//                   over populations l = 4k + G (37 padded to 40); the 16
//                   rows are a_00, a_10, a_01, a_20 + a_02 (for the moments,
//                   Eq. (2)) and the 12 Hermite coefficients a_20 .. a_04;
//   moments         rows 0..3 of site J are register 0 of lanes J, 16 + J,
//                   32 + J, 48 + J; every lane fetches them (ds_bpermute),
//                   then relaxes its own four rows G + 4 r towards the
//                   equilibrium coefficients;
//   reconstruction  f'_l(site) = sum_row Hr[l][row] b[row][site]: for each
//                   tile of 16 populations, 4 products whose B operand is
//                   the lane's own relaxed row G + 4 m (so no data moves
//                   between the two products: the A tables are laid out for
//                   it); result register r of lane (G, J) is population
//                   16 t + G + 4 r of site J.
// Hp[row][l] = H_pq(c_l); Hr[l][row] = w_l H_pq(c_l) / (p! q!) (0 for the
// a_20 + a_02 row); the tables hold each lane's entries.
// ---------------------------------------------------------------------------
typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kRowP[16] = {0, 1, 0, -1, 2, 1, 0, 3, 2, 1, 0, 4, 3, 2, 1, 0};
constexpr int kRowQ[16] = {0, 0, 1, -1, 0, 1, 2, 0, 1, 2, 3, 0, 1, 2, 3, 4};

struct MfmaTables {
  double proj[10][64];    // A operand of projection step k, lane L
  double rec[3][4][64];   // A operand of reconstruction tile t, step m, lane L
};

constexpr MfmaTables make_mfma_tables() {
  MfmaTables T{};
  for (int k = 0; k < 10; ++k)
    for (int L = 0; L < 64; ++L) {
      const int G = L / 16, row = L % 16, l = 4 * k + G;
      double v = 0.0;
      if (l < Q) {
        if (row == 3)
          v = he(EX[l], 2) + he(EY[l], 2);
        else
          v = he(EX[l], kRowP[row]) * he(EY[l], kRowQ[row]);
      }
      T.proj[k][L] = v;
    }
  for (int t = 0; t < 3; ++t)
    for (int m = 0; m < 4; ++m)
      for (int L = 0; L < 64; ++L) {
        const int G = L / 16, l = 16 * t + L % 16, row = G + 4 * m;
        double v = 0.0;
        if (l < Q && row != 3) v = W[l] * hef(EX[l], kRowP[row]) * hef(EY[l], kRowQ[row]);
        T.rec[t][m][L] = v;
      }
  return T;
}

__constant__ MfmaTables kMfma = make_mfma_tables();

__device__ __forceinline__ double lane_fetch(int byte_addr, double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_ds_bpermute(byte_addr, int(unsigned(u)));
  const int hi = __builtin_amdgcn_ds_bpermute(byte_addr, int(unsigned(u >> 32)));
  return __builtin_bit_cast(double, (unsigned long long)unsigned(lo) |
                                        ((unsigned long long)unsigned(hi) << 32));
}

// equilibrium coefficient of row `row` (compile-time) from h_p(U_x), h_q(U_y)
__device__ __forceinline__ double eq_row(int row, double rho, const double (&hx)[5],
                                         const double (&hy)[5]) {
  return row == 3 ? 0.0 : rho * hx[kRowP[row]] * hy[kRowQ[row]];
}

constexpr int kSets = 2;  // site sets per round (divides 4; 2 keeps 3 waves per SIMD)

template <bool kReg>
__global__ __launch_bounds__(kVThreads) void k_collide_mfma(const double* __restrict__ src,
                                                            double* __restrict__ dst, Geom g,
                                                            Phys P, int nyb) {
  const int lane = threadIdx.x & 63;
  const int wave = int(blockIdx.x) * (kVThreads / 64) + int(threadIdx.x >> 6);
  const int x = wave / nyb, yb = wave % nyb;
  if (x >= g.lx) return;  // the whole wave
  const int G = lane >> 4, J = lane & 15;
  double pa[10], ra[3][4];
#pragma unroll
  for (int k = 0; k < 10; ++k) pa[k] = kMfma.proj[k][lane];
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int m = 0; m < 4; ++m) ra[t][m] = kMfma.rec[t][m][lane];
  const double keep = 1.0 - P.omega, om = P.omega;
  const long long col = (long long)(x + HX) * g.cs + g.hy;
  // kSets site sets at a time, their products interleaved so that
  // consecutive matrix instructions are independent (a chain of dependent
  // ones waits out each one's latency)
#pragma unroll 1
  for (int s0 = 0; s0 < 4; s0 += kSets) {
    bool valid[kSets];
    long long site[kSets];
    double bv[kSets][10];
#pragma unroll
    for (int s = 0; s < kSets; ++s) {
      const int y = yb * 64 + 16 * (s0 + s) + J;
      valid[s] = y < g.ly;
      site[s] = col + y;
#pragma unroll
      for (int k = 0; k < 10; ++k) {
        const int l = 4 * k + G;
        bv[s][k] = (valid[s] && l < Q) ? src[l * g.ps + site[s]] : 0.0;
      }
    }
    v4d acc[kSets];
#pragma unroll
    for (int s = 0; s < kSets; ++s) acc[s] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 10; ++k)
#pragma unroll
      for (int s = 0; s < kSets; ++s)
        acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[k], bv[s][k], acc[s], 0, 0, 0);
    double b[kSets][4];
#pragma unroll
    for (int s = 0; s < kSets; ++s) {
      // rows 0..3 (a_00, a_10, a_01, a_20 + a_02) of site J: register 0 of
      // lanes J, 16 + J, 32 + J, 48 + J
      const double a00 = lane_fetch(J * 4, acc[s][0]);
      const double a10 = lane_fetch((16 + J) * 4, acc[s][0]);
      const double a01 = lane_fetch((32 + J) * 4, acc[s][0]);
      const double a2s = lane_fetch((48 + J) * 4, acc[s][0]);
      const double rho = valid[s] ? a00 : 1.0;
      const double inv_rho = 1.0 / rho;
      const double ux = a10 * inv_rho, uy = a01 * inv_rho;
      const double th = 0.5 * (a2s * inv_rho - (ux * ux + uy * uy));
      double hx[5], hy[5];
      gauss_hermite(ux + P.tau_gx, th + P.dtheta, hx);
      gauss_hermite(uy + P.tau_gy, th + P.dtheta, hy);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // this register's row is G + 4 r
        const double e0 = eq_row(4 * r, rho, hx, hy), e1 = eq_row(4 * r + 1, rho, hx, hy);
        const double e2 = eq_row(4 * r + 2, rho, hx, hy), e3 = eq_row(4 * r + 3, rho, hx, hy);
        const double aeq = G == 0 ? e0 : G == 1 ? e1 : G == 2 ? e2 : e3;
        if (kReg)
          // mass is conserved exactly: b_00 = rho
          b[s][r] = (r == 0 && G == 0) ? rho : keep * acc[s][r] + om * aeq;
        else
          b[s][r] = aeq;
      }
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      v4d out[kSets];
#pragma unroll
      for (int s = 0; s < kSets; ++s) out[s] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int s = 0; s < kSets; ++s)
          out[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(ra[t][m], b[s][m], out[s], 0, 0, 0);
#pragma unroll
      for (int s = 0; s < kSets; ++s)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int l = 16 * t + G + 4 * r;
          if (valid[s] && l < Q) {
            const long long a = l * g.ps + site[s];
            double v = out[s][r];
            if (!kReg) v = keep * src[a] + om * v;
            __builtin_nontemporal_store(v, &dst[a]);
          }
        }
    }
  }
}

unsigned blocks(long long n, long long per) { return unsigned((n + per - 1) / per); }

}  // namespace

hipError_t launch_propagate_variant(const void* src, void* dst, const Geom& g, int prec,
                                    int variant, hipStream_t s) {
  auto run = [&](auto sv) {
    using S = decltype(sv);
    const S* a = static_cast<const S*>(src);
    S* b = static_cast<S*>(dst);
    if (variant == kPropagateLds) {
      const int nty = int(blocks(g.ly, kVThreads));
      hipLaunchKernelGGL(k_propagate_lds<S>, dim3(unsigned(g.lx) * unsigned(nty)),
                         dim3(kVThreads), 0, s, a, b, g, nty);
    } else {
      const int nty = int(blocks(g.ly, (long long)kVThreads * Wide<S>::V));
      hipLaunchKernelGGL(k_propagate_wide<S>, dim3(unsigned(g.lx) * unsigned(nty)),
                         dim3(kVThreads), 0, s, a, b, g, nty);
    }
  };
  if (variant != kPropagateLds && variant != kPropagateWide) return hipErrorInvalidValue;
  if (prec == kF64)
    run(double{});
  else if (prec == kF32Shifted || prec == kF32ShiftedF32Sum)
    run(float{});
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_collide_mfma(const void* src, void* dst, const Geom& g, const Phys& p,
                               int regularize, hipStream_t s) {
  const int nyb = int(blocks(g.ly, 64));
  const unsigned grid = blocks((long long)g.lx * nyb, kVThreads / 64);
  const double* a = static_cast<const double*>(src);
  double* b = static_cast<double*>(dst);
  if (regularize)
    hipLaunchKernelGGL(k_collide_mfma<true>, dim3(grid), dim3(kVThreads), 0, s, a, b, g, p, nyb);
  else
    hipLaunchKernelGGL(k_collide_mfma<false>, dim3(grid), dim3(kVThreads), 0, s, a, b, g, p,
                       nyb);
  return hipGetLastError();
}

}  // namespace d2q37
