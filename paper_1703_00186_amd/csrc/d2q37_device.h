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

}  // namespace d2q37
