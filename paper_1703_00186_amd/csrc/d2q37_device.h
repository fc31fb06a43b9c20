// Device-side building blocks of the D2Q37 step for gfx950.
//
// Everything here works on one lattice site held in registers.  All loops
// over populations and Hermite orders are fully unrolled, so every velocity,
// weight and Hermite value from d2q37_constants.h becomes a literal operand
// (scalar register or inline constant) instead of a memory load; this is the
// CDNA counterpart of the constant-bank effect the paper measures for its
// CUDA collide (Sec. 5).
//
// Hermite form of the collision (Sec. 2: regularized BGK, Eq. (1)).  With
// H_pq(c) = He_p(c_x) He_q(c_y), p + q <= 4 (15 components):
//   project      a_pq = sum_l f_l H_pq(c_l)
//   moments      rho = a_00, u = (a_10, a_01)/rho,
//                Theta = T - 1 = (a_20 + a_02 - rho |u|^2) / (2 rho)   (Eq. (2))
//   equilibrium  a^eq_pq = rho h_p(u*_x) h_q(u*_y), with the Hermite moments of
//                a unit-variance-shifted Gaussian h_0..4(U) = 1, U, U^2+Th,
//                U^3+3U Th, U^4+6U^2 Th+3Th^2, evaluated at the forced
//                u* = u + tau g, Th* = Theta + tau (1-tau) |g|^2 / 2
//   relax        a'_pq = (1 - 1/tau) a_pq + a^eq_pq / tau
//   reconstruct  f'_l = w_l sum_pq a'_pq H_pq(c_l) / (p! q!)
// Both sums are done separably: populations are grouped by their x hop, so a
// projection costs about 37*4 + 7*15 multiply-adds instead of 37*15.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "d2q37_constants.h"

namespace d2q37 {

// Padded lattice geometry.  Physical site (x, y), 0 <= x < lx, 0 <= y < ly,
// lives at padded column X = x + HX and row Y = y + hy; population l of padded
// site (X, Y) is at element l*ps + X*cs + Y.
constexpr int HX = 3;  // halo columns on each side (Sec. 2: three columns)

struct Geom {
  int lx, ly;      // physical sizes
  int nx, ny;      // padded sizes (nx = lx + 2*HX)
  int hy;          // physical row 0 is padded row hy (hy >= 3)
  int walls;       // 1: thermal walls in y, 0: periodic y
  int np;          // planes per padded site: Q, or Q + 1 in the local-reference
                   // form (its packed reference)
  long long ps;    // element stride between populations
  long long cs;    // element stride between padded columns
};

struct Phys {
  double omega;        // 1 / tau
  double tau_gx;       // tau * g_x (velocity shift of the equilibrium)
  double tau_gy;       // tau * g_y
  double dtheta;       // tau (1 - tau) |g|^2 / 2 (temperature shift)
  double th_bottom;    // T_bottom - 1
  double th_top;       // T_top - 1
  double rho_ref;      // shift of FP32 populations (0 for FP64)
};

// He_n(R e) and He_n(R e)/n! for an integer hop component e in [-3, 3].
__host__ __device__ constexpr double he(int e, int n) {
  return (e < 0 && (n & 1)) ? -HE[-e][n] : HE[e < 0 ? -e : e][n];
}
__host__ __device__ constexpr double hef(int e, int n) {
  return (e < 0 && (n & 1)) ? -HEF[-e][n] : HEF[e < 0 ? -e : e][n];
}
// |c_l|^2 = R^2 |e_l|^2
__host__ __device__ constexpr double c2(int l) {
  return R * R * double(EX[l] * EX[l] + EY[l] * EY[l]);
}

// ---------------------------------------------------------------------------
// project: a_pq = sum_l f_l He_p(c_lx) He_q(c_ly), accumulated in type A.
// ---------------------------------------------------------------------------
template <class A>
__device__ __forceinline__ void project(const A (&f)[Q], A (&a)[5][5]) {
#pragma unroll
  for (int p = 0; p < 5; ++p)
#pragma unroll
    for (int q = 0; q < 5; ++q) a[p][q] = A(0);
#pragma unroll
  for (int ex = 3; ex >= -3; --ex) {
    A s[5] = {A(0), A(0), A(0), A(0), A(0)};
#pragma unroll
    for (int l = 0; l < Q; ++l) {
      if (EX[l] != ex) continue;
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const double h = he(EY[l], q);
        if (h == 0.0) continue;
        if (h == 1.0)
          s[q] += f[l];
        else if (h == -1.0)
          s[q] -= f[l];
        else
          s[q] += A(h) * f[l];
      }
    }
#pragma unroll
    for (int p = 0; p < 5; ++p) {
      const double hp = he(ex, p);
      if (hp == 0.0) continue;
#pragma unroll
      for (int q = 0; q + p < 5; ++q) {
        if (hp == 1.0)
          a[p][q] += s[q];
        else if (hp == -1.0)
          a[p][q] -= s[q];
        else
          a[p][q] += A(hp) * s[q];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// reconstruct: f_l = w_l sum_pq b_pq He_p(c_lx) He_q(c_ly) / (p! q!).
// ---------------------------------------------------------------------------
template <class A>
__device__ __forceinline__ void reconstruct(const A (&b)[5][5], A (&f)[Q]) {
#pragma unroll
  for (int ex = 3; ex >= -3; --ex) {
    // P_q = sum_p b_pq He_p(c_x) / p!
    A P[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      A s = A(0);
#pragma unroll
      for (int p = 0; p + q < 5; ++p) {
        const double hp = hef(ex, p);
        if (hp == 0.0) continue;
        if (hp == 1.0)
          s += b[p][q];
        else
          s += A(hp) * b[p][q];
      }
      P[q] = s;
    }
#pragma unroll
    for (int l = 0; l < Q; ++l) {
      if (EX[l] != ex) continue;
      A v = A(0);
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const double hq = W[l] * hef(EY[l], q);
        if (hq == 0.0) continue;
        v += A(hq) * P[q];
      }
      f[l] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// expand: v_l = sum_pq b_pq He_p(c_lx) He_q(c_ly)  (the transpose of project;
// used by the adjoint).
// ---------------------------------------------------------------------------
template <class A>
__device__ __forceinline__ void expand(const A (&b)[5][5], A (&v)[Q]) {
#pragma unroll
  for (int ex = 3; ex >= -3; --ex) {
    A P[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      A s = A(0);
#pragma unroll
      for (int p = 0; p + q < 5; ++p) {
        const double hp = he(ex, p);
        if (hp == 0.0) continue;
        if (hp == 1.0)
          s += b[p][q];
        else
          s += A(hp) * b[p][q];
      }
      P[q] = s;
    }
#pragma unroll
    for (int l = 0; l < Q; ++l) {
      if (EX[l] != ex) continue;
      A t = A(0);
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const double hq = he(EY[l], q);
        if (hq == 0.0) continue;
        t += A(hq) * P[q];
      }
      v[l] = t;
    }
  }
}

// Hermite moments of the shifted Gaussian: h_n(U, Th), n = 0..4.
__device__ __forceinline__ void gauss_hermite(double U, double th, double (&h)[5]) {
  const double U2 = U * U;
  h[0] = 1.0;
  h[1] = U;
  h[2] = U2 + th;
  h[3] = U * (U2 + 3.0 * th);
  h[4] = U2 * (U2 + 6.0 * th) + 3.0 * th * th;
}

// Their derivatives with respect to U and to Th.
__device__ __forceinline__ void gauss_hermite_d(double U, double th, double (&dU)[5],
                                                double (&dT)[5]) {
  const double U2 = U * U;
  dU[0] = 0.0;
  dU[1] = 1.0;
  dU[2] = 2.0 * U;
  dU[3] = 3.0 * (U2 + th);
  dU[4] = 4.0 * U * (U2 + 3.0 * th);
  dT[0] = 0.0;
  dT[1] = 0.0;
  dT[2] = 1.0;
  dT[3] = 3.0 * U;
  dT[4] = 6.0 * (U2 + th);
}

// Macroscopic state from the Hermite coefficients (FP64), Eq. (2).
struct Macro {
  double rho, inv_rho, ux, uy, th;
};

__device__ __forceinline__ Macro macro_from(double a00, double a10, double a01, double a20,
                                            double a02) {
  Macro m;
  m.rho = a00;
  m.inv_rho = 1.0 / a00;
  m.ux = a10 * m.inv_rho;
  m.uy = a01 * m.inv_rho;
  m.th = 0.5 * ((a20 + a02) * m.inv_rho - (m.ux * m.ux + m.uy * m.uy));
  return m;
}

// a^eq_pq = rho h_p(Ux) h_q(Uy) in FP64.
__device__ __forceinline__ void equilibrium_coeffs(double rho, double Ux, double Uy, double th,
                                                   double (&aeq)[5][5]) {
  double hx[5], hy[5];
  gauss_hermite(Ux, th, hx);
  gauss_hermite(Uy, th, hy);
#pragma unroll
  for (int p = 0; p < 5; ++p)
#pragma unroll
    for (int q = 0; q + p < 5; ++q) aeq[p][q] = rho * hx[p] * hy[q];
}

// w_l * f^eq_l(rho = 1, u = 0, T = 1 + th): the wall Maxwellian.
__device__ __forceinline__ double wall_feq(int l, double th) {
  const double x2 = c2(l);
  return W[l] * (1.0 + 0.5 * th * (x2 - 2.0) + 0.125 * th * th * (x2 * x2 - 8.0 * x2 + 8.0));
}

// ---------------------------------------------------------------------------
// bc at one wall site (rows 0..2 or ly-3..ly-1): unknown populations (source
// row outside [0, ly)) become rho_w v_l, v_l = f^eq_l(1, 0, T_wall),
// rho_w = sum_K f / sum_K v over the known ones K.  f holds shifted values
// f_l - w_l rho_ref (rho_ref = 0 for unshifted populations).
// ---------------------------------------------------------------------------
template <class A>
__device__ __forceinline__ void wall_site(A (&f)[Q], int y, int ly, double th_bottom,
                                          double th_top, double rho_ref) {
  const bool bottom = y < 3;
  const double th = bottom ? th_bottom : th_top;
  double sk = 0.0, vk = 0.0;
#pragma unroll
  for (int l = 0; l < Q; ++l) {
    const int ys = y - EY[l];
    const bool unknown = ys < 0 || ys >= ly;
    if (!unknown) {
      sk += double(f[l]) + rho_ref * W[l];
      vk += wall_feq(l, th);
    }
  }
  const double rho_w = sk / vk;
#pragma unroll
  for (int l = 0; l < Q; ++l) {
    const int ys = y - EY[l];
    const bool unknown = ys < 0 || ys >= ly;
    if (unknown) f[l] = A(rho_w * wall_feq(l, th) - rho_ref * W[l]);
  }
}

// Pre-collision moments for the adjoint tape: (rho, rho u_x, rho u_y, sum |c|^2 f).
struct Tape4 {
  double rho, jx, jy, e;
};

// ---------------------------------------------------------------------------
// collide one site in Hermite space.  f: populations (shifted by w rho_ref if
// rho_ref != 0); on return f holds the post-collision values (same shift).
// A is the accumulation type of the projection and reconstruction (double, or
// float for the FP32 form); moments, equilibrium and relaxation are FP64.
// ---------------------------------------------------------------------------
template <class A, bool kRegularize>
__device__ __forceinline__ Tape4 collide_site(A (&f)[Q], const Phys& P) {
  A a[5][5];
  project<A>(f, a);
  // a_00 of shifted populations is rho - rho_ref; the shift adds nothing to
  // the other coefficients (sum_l w_l H_pq(c_l) = 0 for (p, q) != (0, 0)).
  const double da00 = double(a[0][0]);
  const Macro m = macro_from(P.rho_ref + da00, double(a[1][0]), double(a[0][1]),
                             double(a[2][0]), double(a[0][2]));
  Tape4 t;
  t.rho = m.rho;
  t.jx = double(a[1][0]);
  t.jy = double(a[0][1]);
  t.e = double(a[2][0]) + double(a[0][2]) + 2.0 * m.rho;
  double aeq[5][5];
  equilibrium_coeffs(m.rho, m.ux + P.tau_gx, m.uy + P.tau_gy, m.th + P.dtheta, aeq);
  aeq[0][0] = da00;  // mass is conserved: rho - rho_ref (shifted) or rho
  if (kRegularize) {
    const double keep = 1.0 - P.omega;
    A b[5][5];
#pragma unroll
    for (int p = 0; p < 5; ++p)
#pragma unroll
      for (int q = 0; q + p < 5; ++q) {
        const double ap = (p == 0 && q == 0) ? aeq[0][0]
                                             : keep * double(a[p][q]) + P.omega * aeq[p][q];
        b[p][q] = A(ap);
      }
    reconstruct<A>(b, f);
  } else {
    A b[5][5];
#pragma unroll
    for (int p = 0; p < 5; ++p)
#pragma unroll
      for (int q = 0; q + p < 5; ++q) b[p][q] = A(aeq[p][q]);
    A feq[Q];
    reconstruct<A>(b, feq);
    const A keep = A(1.0 - P.omega), om = A(P.omega);
#pragma unroll
    for (int l = 0; l < Q; ++l) f[l] = keep * f[l] + om * feq[l];
  }
  return t;
}

// ---------------------------------------------------------------------------
// FP32 storage relative to the local rest Maxwellian, and the FP32 collision.
//
// A population is stored as its deviation from the rest Maxwellian of the
// site that last collided it,
//   g_l = f_l - M_l(rho_s, th_s),
//   M_l(rho, th) = w_l rho [1 + th (|c_l|^2 - 2)/2 + th^2 (|c_l|^4 - 8|c_l|^2 + 8)/8]
// (f^eq at u = 0 and temperature 1 + th, exact Eq. (2) moments), in FP32,
// and that site's (rho_s, th_s) as two FP16 numbers packed into one 32-bit
// word: a 38th plane beside the 37 populations.  The deviation carries only
// the flow and the non-equilibrium part of f (a few per cent of f in a slow
// flow), so its FP32 rounding is that much smaller than a rounding of f or of
// f - w_l rho_0.  The FP16 reference needs no accuracy of its own: writer and
// reader evaluate M from the same stored pair, in FP64.
// ---------------------------------------------------------------------------
constexpr int kFamilies = 8;
// weight family of hop l, numbered by |e_l|^2 = 0, 1, 2, 4, 5, 8, 9, 10
__host__ __device__ constexpr int family_of(int l) {
  return (EX[l] * EX[l] + EY[l] * EY[l]) == 0    ? 0
         : (EX[l] * EX[l] + EY[l] * EY[l]) == 1 ? 1
         : (EX[l] * EX[l] + EY[l] * EY[l]) == 2 ? 2
         : (EX[l] * EX[l] + EY[l] * EY[l]) == 4 ? 3
         : (EX[l] * EX[l] + EY[l] * EY[l]) == 5 ? 4
         : (EX[l] * EX[l] + EY[l] * EY[l]) == 8 ? 5
         : (EX[l] * EX[l] + EY[l] * EY[l]) == 9 ? 6
                                                 : 7;
}
constexpr int kFamilyE2[kFamilies] = {0, 1, 2, 4, 5, 8, 9, 10};
// a hop of each family (for its weight)
constexpr int kFamilyLabel[kFamilies] = {18, 17, 10, 16, 9, 3, 15, 8};
// hops (0,0), (1,0), (-1,0), (0,1), (0,-1): the populations that absorb the
// conservation correction of the FP32 reconstruction
constexpr int kRest = 18, kEast = 11, kWest = 25, kNorth = 19, kSouth = 17;
// planes of a padded buffer in the local-reference form: 37 deviations + the
// packed reference
constexpr int kLocalPlanes = Q + 1;

// (the weights folded into the polynomial's compile-time coefficients, so
// that a rebuilt population rho P_l(th) + g is three FMAs)
__device__ __forceinline__ double rest_maxwellian(int l, double rho, double th) {
  const double x2 = c2(l);
  const double w1 = W[l] * (0.5 * (x2 - 2.0)), w2 = W[l] * (0.125 * (x2 * x2 - 8.0 * x2 + 8.0));
  return rho * fma(th, fma(w2, th, w1), W[l]);
}

// (rho_s, th_s) <-> one 32-bit word of two FP16 numbers (rho_s low, th_s high)
__device__ __forceinline__ unsigned pack_ref(double rho, double th) {
  const unsigned short a = __builtin_bit_cast(unsigned short, (_Float16)float(rho));
  const unsigned short b = __builtin_bit_cast(unsigned short, (_Float16)float(th));
  return unsigned(a) | (unsigned(b) << 16);
}
__device__ __forceinline__ void unpack_ref(unsigned v, double& rho, double& th) {
  rho = double(float(__builtin_bit_cast(_Float16, (unsigned short)(v & 0xffffu))));
  th = double(float(__builtin_bit_cast(_Float16, (unsigned short)(v >> 16))));
}

// The reference a site takes from its FP64 populations: its density and
// th_s = sum |c|^2 f / (2 rho) - 1, rounded to FP16; the deviations from it.
__device__ __forceinline__ unsigned encode_site(const double (&f)[Q], float (&g)[Q]) {
  double rho = 0.0, e2 = 0.0;
#pragma unroll
  for (int l = 0; l < Q; ++l) {
    rho += f[l];
    e2 += c2(l) * f[l];
  }
  const unsigned ref = pack_ref(rho, 0.5 * e2 / rho - 1.0);
  double rs, ts;
  unpack_ref(ref, rs, ts);
#pragma unroll
  for (int l = 0; l < Q; ++l) g[l] = float(f[l] - rest_maxwellian(l, rs, ts));
  return ref;
}

// Collision of one site from its FP64 populations f (rebuilt from the stored
// deviations and their writers' references); returns the site's new packed
// reference and writes the post-collision deviations g from it:
//   1. collision invariants in FP64: rho, momentum j, energy E = sum |c|^2 f;
//      new reference (rho, E / (2 rho) - 1) rounded to FP16;
//   2. n_l = f_l - M_l(rho_s, th_s) in FP64, rounded to FP32;
//   3. Hermite coefficients of n in FP32 (the FP32-accumulated moments), the
//      invariant ones (a_00, a_10, a_01, a_20 + a_02) from step 1 instead;
//   4. the forced equilibrium coefficients in FP64 (Hermite orders up to
//      four) minus those of the reference, and the relaxed deviation
//      b_pq = (1 - 1/tau) a^n_pq + (a^eq_pq - a^M_pq) / tau in FP64, rounded
//      once to FP32 (a^M: a_00 = rho_s, a_20 = a_02 = rho_s th_s,
//      a_40 = a_04 = 3 rho_s th_s^2, a_22 = rho_s th_s^2, the others 0);
//   5. g_l = w_l sum_pq b_pq H_pq(c_l) / (p! q!) in FP32;
//   6. conservation: the invariants of the FP32 values g are summed in FP64
//      and their shortfall against b_00, b_10, b_01, b_20 + b_02 (exact) is
//      put into the five populations (0,0), (+-1,0), (0,+-1) (in FP32
//      rounding errors are systematic over a slowly varying flow, and a
//      shortfall in an invariant would accumulate from step to step).
// Plain BGK relaxes n itself: g = (1 - 1/tau) n + reconstruction of
// (a^eq - a^M) / tau, with the same correction.
template <bool kRegularize>
__device__ __forceinline__ unsigned collide_site_local(const double (&f)[Q], float (&g)[Q],
                                                       const Phys& P) {
  // 1. invariants: per-family, per-e_x and per-e_y sums
  double sf[kFamilies], sx[7], sy[7];
#pragma unroll
  for (int k = 0; k < kFamilies; ++k) sf[k] = 0.0;
#pragma unroll
  for (int k = 0; k < 7; ++k) sx[k] = sy[k] = 0.0;
#pragma unroll
  for (int l = 0; l < Q; ++l) {
    sf[family_of(l)] += f[l];
    if (EX[l] != 0) sx[EX[l] + 3] += f[l];
    if (EY[l] != 0) sy[EY[l] + 3] += f[l];
  }
  double rho = 0.0, s2 = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
  for (int k = 0; k < kFamilies; ++k) {
    rho += sf[k];
    s2 += double(kFamilyE2[k]) * sf[k];
  }
#pragma unroll
  for (int e = 1; e <= 3; ++e) {
    jx += double(e) * (sx[3 + e] - sx[3 - e]);
    jy += double(e) * (sy[3 + e] - sy[3 - e]);
  }
  jx *= R;
  jy *= R;
  const double inv_rho = 1.0 / rho;
  const double e2 = R * R * s2;  // sum |c|^2 f
  const unsigned ref = pack_ref(rho, 0.5 * e2 * inv_rho - 1.0);
  double rs, ts;
  unpack_ref(ref, rs, ts);
  // 2. deviation from the new reference
  double m[kFamilies];
#pragma unroll
  for (int k = 0; k < kFamilies; ++k) m[k] = rest_maxwellian(kFamilyLabel[k], rs, ts);
  float n[Q];
#pragma unroll
  for (int l = 0; l < Q; ++l) n[l] = float(f[l] - m[family_of(l)]);
  // 3. FP32 Hermite coefficients of n
  float an[5][5];
  project<float>(n, an);
  // 4. equilibrium minus reference, relaxation (FP64, one rounding)
  const double ux = jx * inv_rho, uy = jy * inv_rho;
  const double th = 0.5 * (e2 * inv_rho - (ux * ux + uy * uy)) - 1.0;
  double aeq[5][5];
  equilibrium_coeffs(rho, ux + P.tau_gx, uy + P.tau_gy, th + P.dtheta, aeq);
  const double aM20 = rs * ts, aM40 = 3.0 * rs * ts * ts, aM22 = rs * ts * ts;
  // a_20 + a_02 is sum (|c|^2 - 2) f: E - 2 rho for f, 2 aM20 for the reference
  const double sum2 = (e2 - 2.0 * rho) - 2.0 * aM20;
  const double half_diff = 0.5 * (double(an[2][0]) - double(an[0][2]));
  const double om = P.omega, keep = 1.0 - P.omega;
  float b[5][5];
  double b00 = 0.0, b10 = 0.0, b01 = 0.0, b2 = 0.0;
#pragma unroll
  for (int p = 0; p < 5; ++p)
#pragma unroll
    for (int q = 0; q + p < 5; ++q) {
      double am = 0.0, a = double(an[p][q]);
      if (p == 0 && q == 0) {
        am = rs;
        a = rho - rs;
      }
      if ((p == 2 && q == 0) || (p == 0 && q == 2)) am = aM20;
      if ((p == 4 && q == 0) || (p == 0 && q == 4)) am = aM40;
      if (p == 2 && q == 2) am = aM22;
      if (p == 1 && q == 0) a = jx;
      if (p == 0 && q == 1) a = jy;
      if (p == 2 && q == 0) a = 0.5 * sum2 + half_diff;
      if (p == 0 && q == 2) a = 0.5 * sum2 - half_diff;
      const double dm = (p == 0 && q == 0) ? rho - rs : aeq[p][q] - am;
      const double bv = kRegularize ? keep * a + om * dm : om * dm;
      b[p][q] = float(bv);
      if (p == 0 && q == 0) b00 = bv;
      if (p == 1 && q == 0) b10 = bv;
      if (p == 0 && q == 1) b01 = bv;
      if (p + q == 2 && p != 1) b2 += bv;
    }
  if (!kRegularize) {
    // BGK: the invariants of (1 - 1/tau) n come on top of those of d / tau
    b00 += keep * (rho - rs);
    b10 += keep * jx;
    b01 += keep * jy;
    b2 += keep * sum2;
  }
  // 5. FP32 reconstruction of the deviation
  float r[Q];
  reconstruct<float>(b, r);
#pragma unroll
  for (int l = 0; l < Q; ++l) g[l] = kRegularize ? r[l] : float(keep) * n[l] + r[l];
  // 6. conservation correction
  double cf[kFamilies], cx[7], cy[7];
#pragma unroll
  for (int k = 0; k < kFamilies; ++k) cf[k] = 0.0;
#pragma unroll
  for (int k = 0; k < 7; ++k) cx[k] = cy[k] = 0.0;
#pragma unroll
  for (int l = 0; l < Q; ++l) {
    const double v = double(g[l]);
    cf[family_of(l)] += v;
    if (EX[l] != 0) cx[EX[l] + 3] += v;
    if (EY[l] != 0) cy[EY[l] + 3] += v;
  }
  double m0 = 0.0, m2 = 0.0, mx = 0.0, my = 0.0;
#pragma unroll
  for (int k = 0; k < kFamilies; ++k) {
    m0 += cf[k];
    m2 += (R * R * double(kFamilyE2[k]) - 2.0) * cf[k];
  }
#pragma unroll
  for (int e = 1; e <= 3; ++e) {
    mx += double(e) * (cx[3 + e] - cx[3 - e]);
    my += double(e) * (cy[3 + e] - cy[3 - e]);
  }
  const double dm0 = b00 - m0, dx = b10 - R * mx, dy = b01 - R * my, d2 = b2 - m2;
  // corrections z (rest), a, b (east, west), c, d (north, south) with
  //   z + a + b + c + d = dm0, R (a - b) = dx, R (c - d) = dy,
  //   -2 z + (R^2 - 2)(a + b + c + d) = d2, a + b = c + d
  const double sq = (d2 + 2.0 * dm0) / (R * R);
  g[kRest] = float(double(g[kRest]) + (dm0 - sq));
  g[kEast] = float(double(g[kEast]) + 0.5 * (0.5 * sq + dx / R));
  g[kWest] = float(double(g[kWest]) + 0.5 * (0.5 * sq - dx / R));
  g[kNorth] = float(double(g[kNorth]) + 0.5 * (0.5 * sq + dy / R));
  g[kSouth] = float(double(g[kSouth]) + 0.5 * (0.5 * sq - dy / R));
  return ref;
}

// The FP64 collision in the local-reference storage form: f (FP64, rebuilt
// from the stored deviations) is collided as in the FP64 form; the new
// reference is the site's density and th = E / (2 rho) - 1 of the
// pre-collision invariants (the collision changes E only by the forcing
// increment), and the deviations g = f' - M(rho_s, th_s) are rounded to FP32
// once.
template <bool kRegularize>
__device__ __forceinline__ unsigned collide_site_local64(double (&f)[Q], float (&g)[Q],
                                                         const Phys& P) {
  const Tape4 m = collide_site<double, kRegularize>(f, P);
  const unsigned ref = pack_ref(m.rho, 0.5 * m.e / m.rho - 1.0);
  double rs, ts;
  unpack_ref(ref, rs, ts);
  double mf[kFamilies];
#pragma unroll
  for (int k = 0; k < kFamilies; ++k) mf[k] = rest_maxwellian(kFamilyLabel[k], rs, ts);
#pragma unroll
  for (int l = 0; l < Q; ++l) g[l] = float(f[l] - mf[family_of(l)]);
  return ref;
}

// Collision dispatch on the accumulation type of the FP64 and shifted FP32
// forms (the local-reference form has kernels of its own).
template <class A, bool kRegularize>
__device__ __forceinline__ Tape4 collide(A (&f)[Q], const Phys& P) {
  return collide_site<A, kRegularize>(f, P);
}

}  // namespace d2q37
