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
// reconstruct: f_l = w_l sum_pq b_pq He_p(c_lx) He_q(c_ly) / (p! q!), over the
// Hermite orders p + q >= kMinOrder (the lower ones are left out).
// ---------------------------------------------------------------------------
template <class A, int kMinOrder = 0>
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
        if (hp == 0.0 || p + q < kMinOrder) continue;
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
// FP32 collision relative to a local reference (the FP32-arithmetic form).
//
// FP32 rounding is relative to the size of the numbers summed.  The
// populations of a site lie close to its rest Maxwellian
//   R_l = w_l rho [1 + th_R (|c_l|^2 - 2)/2 + th_R^2 (|c_l|^4 - 8|c_l|^2 + 8)/8]
// (f^eq at u = 0 and temperature 1 + th_R, Eq. (2) moments exact), so the
// non-conserved part of the collision is computed in FP32 on n_l = f_l - R_l,
// small wherever the flow is slow and near equilibrium, while the collision
// invariants are summed in FP64:
//   1. FP64 sums of the stored values: mass rho, momentum j, energy
//      E = sum |c|^2 f; th_R = E / (2 rho) - 1, so n carries no mass and no
//      energy and its momentum is j;
//   2. R_l - w_l rho_ref per weight family (|e_l|^2 fixes w_l and |c_l|^2),
//      in FP64, kept as an unevaluated FP32 pair hi + lo;
//   3. n_l = (g_l - hi) - lo in FP32 (the first difference is exact or off
//      by half an ulp of n);
//   4. the Hermite coefficients of n in FP32 (the FP32-accumulated moments),
//      with a_00 = 0, a_10 = j_x, a_01 = j_y and a_20 + a_02 = 0 taken from
//      step 1 instead;
//   5. the forced equilibrium coefficients in FP64 at rho, u = j / rho,
//      th = th_R - |u|^2 / 2 (Hermite orders up to four, where cancellation
//      against the reference needs the digits); d_pq = a^eq_pq - a^R_pq
//      rounded to FP32, with a^R_00 = rho, a^R_20 = a^R_02 = rho th_R,
//      a^R_40 = a^R_04 = 3 rho th_R^2, a^R_22 = rho th_R^2, all others 0;
//   6. the relaxed deviation b_pq = (1 - 1/tau) a^n_pq + d_pq / tau
//      (regularized) reconstructed in FP32 as r_l; plain BGK relaxes n_l
//      itself and adds the reconstruction of d / tau;
//   7. g'_l = hi + (lo + r_l): one FP32 rounding of the stored value.
// g holds f_l - w_l rho_ref in FP32 on entry and on return.
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

template <bool kRegularize>
__device__ __forceinline__ void collide_site_ref(float (&g)[Q], const Phys& P) {
  // 1. collision invariants in FP64: per-family, per-e_x and per-e_y sums
  double sf[kFamilies], sx[7], sy[7];
#pragma unroll
  for (int k = 0; k < kFamilies; ++k) sf[k] = 0.0;
#pragma unroll
  for (int k = 0; k < 7; ++k) sx[k] = sy[k] = 0.0;
#pragma unroll
  for (int l = 0; l < Q; ++l) {
    const double v = double(g[l]);
    sf[family_of(l)] += v;
    if (EX[l] != 0) sx[EX[l] + 3] += v;
    if (EY[l] != 0) sy[EY[l] + 3] += v;
  }
  double s0 = 0.0, s2 = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
  for (int k = 0; k < kFamilies; ++k) {
    s0 += sf[k];
    s2 += double(kFamilyE2[k]) * sf[k];
  }
#pragma unroll
  for (int e = 1; e <= 3; ++e) {
    jx += double(e) * (sx[3 + e] - sx[3 - e]);
    jy += double(e) * (sy[3 + e] - sy[3 - e]);
  }
  // the shift w rho_ref adds rho_ref to the mass and 2 rho_ref to the energy
  const double rho = P.rho_ref + s0;
  const double inv_rho = 1.0 / rho;
  const double th_r = 0.5 * (R * R * s2 + 2.0 * P.rho_ref) * inv_rho - 1.0;
  jx *= R;
  jy *= R;
  // 2. reference per family: w (R/w - rho_ref) as hi + lo
  float hi[kFamilies], lo[kFamilies];
#pragma unroll
  for (int k = 0; k < kFamilies; ++k) {
    const double x2 = R * R * double(kFamilyE2[k]);
    const double c1 = 0.5 * (x2 - 2.0), c2 = 0.125 * (x2 * x2 - 8.0 * x2 + 8.0);
    const double v = W[kFamilyLabel[k]] * (rho * (1.0 + th_r * (c1 + c2 * th_r)) - P.rho_ref);
    hi[k] = float(v);
    lo[k] = float(v - double(hi[k]));
  }
  // 3. deviation from the reference
  float n[Q];
#pragma unroll
  for (int l = 0; l < Q; ++l) n[l] = (g[l] - hi[family_of(l)]) - lo[family_of(l)];
  // 4. FP32 Hermite coefficients of n
  float an[5][5];
  project<float>(n, an);
  // 5. forced equilibrium minus the reference and the relaxed deviation, in
  // FP64, rounded once to FP32.  The invariants come from step 1: n has no
  // mass, momentum j and a_20 + a_02 = 0.
  const double ux = jx * inv_rho, uy = jy * inv_rho;
  const double th = th_r - 0.5 * (ux * ux + uy * uy);
  double aeq[5][5];
  equilibrium_coeffs(rho, ux + P.tau_gx, uy + P.tau_gy, th + P.dtheta, aeq);
  const double th2 = th_r * th_r;
  const double aR20 = rho * th_r, aR40 = 3.0 * rho * th2, aR22 = rho * th2;
  const double om = P.omega, keep = 1.0 - P.omega;
  const double half_diff = 0.5 * (double(an[2][0]) - double(an[0][2]));
  float b[5][5];
#pragma unroll
  for (int p = 0; p < 5; ++p)
#pragma unroll
    for (int q = 0; q + p < 5; ++q) {
      double ar = 0.0, a = double(an[p][q]);
      if ((p == 2 && q == 0) || (p == 0 && q == 2)) ar = aR20;
      if ((p == 4 && q == 0) || (p == 0 && q == 4)) ar = aR40;
      if (p == 2 && q == 2) ar = aR22;
      if (p == 1 && q == 0) a = jx;
      if (p == 0 && q == 1) a = jy;
      if (p == 2 && q == 0) a = half_diff;
      if (p == 0 && q == 2) a = -half_diff;
      b[p][q] = float(kRegularize ? keep * a + om * (aeq[p][q] - ar) : om * (aeq[p][q] - ar));
    }
  b[0][0] = 0.0f;  // a^eq_00 = rho = a^R_00: collision conserves mass
  // 6. reconstruct the deviation in FP32; the first-order (momentum) terms
  // on their own, not rounded inside the column sums of the larger
  // higher-order terms
  float r[Q];
  reconstruct<float, 2>(b, r);
#pragma unroll
  for (int l = 0; l < Q; ++l) {
    float r1 = 0.0f;
    if (EX[l] != 0) r1 += float(W[l] * R * EX[l]) * b[1][0];
    if (EY[l] != 0) r1 += float(W[l] * R * EY[l]) * b[0][1];
    r[l] = kRegularize ? r1 + r[l] : float(keep) * n[l] + (r1 + r[l]);
  }
  // 7. back to stored values
#pragma unroll
  for (int l = 0; l < Q; ++l) g[l] = hi[family_of(l)] + (lo[family_of(l)] + r[l]);
}

// Collision dispatch on the accumulation type: double or float run
// collide_site in that type; F32Ref (populations in float registers) runs
// collide_site_ref.  The tape is produced by the FP64 form only.
struct F32Ref {};
template <class A>
struct reg_of {
  using type = A;
};
template <>
struct reg_of<F32Ref> {
  using type = float;
};
template <class A>
using reg_t = typename reg_of<A>::type;

template <class A, bool kRegularize>
__device__ __forceinline__ Tape4 collide(reg_t<A> (&f)[Q], const Phys& P) {
  if constexpr (std::is_same<A, F32Ref>::value) {
    collide_site_ref<kRegularize>(f, P);
    return Tape4{0.0, 0.0, 0.0, 0.0};
  } else {
    return collide_site<A, kRegularize>(f, P);
  }
}

}  // namespace d2q37
