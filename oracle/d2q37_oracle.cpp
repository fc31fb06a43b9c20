// D2Q37 thermal lattice Boltzmann step: plain, slow CPU oracle.
//
// TEST INFRASTRUCTURE ONLY.  This library is loaded by the test-suite, by the
// smoke check and by the CPU-baseline leg of the benchmark, and by nothing
// else.  It shares no code, header, table or constant generator with the GPU
// library: it derives its own velocity set and weights at load time, and it
// evaluates the equilibrium from the closed-form polynomial rather than from
// Hermite coefficient tables.
//
// Source: Calore, Gabbana, Kraus, Schifano, Tripiccione, "Performance and
// Portability of Accelerated Lattice Boltzmann Applications with OpenACC".
//   Sec. 2, Eq. (1)  BGK update: the population arriving from x - c_l relaxes
//                    towards the local equilibrium with rate 1/tau.
//   Sec. 2, Eq. (2)  rho = sum f, rho u = sum c f, D rho T = sum |c-u|^2 f,
//                    perfect-gas equation of state p = rho T, D = 2.
//   Sec. 2           populations travel at most three sites per step;
//                    propagate, then bc (top/bottom walls at constant
//                    temperature and zero velocity), then collide; periodic x
//                    through three halo columns; a projection onto Hermite
//                    polynomials for stability.
//   Sec. 4, Fig. 4   the propagate listing: population 0 at a site is read
//                    from the site three columns to the left and one row up,
//                    population 1 from three columns to the left, same row.
// Where the paper is silent (equilibrium formula, weights, bc scheme, forcing)
// the readings are stated next to the code that takes them.
//
// Every routine is templated on the scalar type so that the same source runs
// in double, in std::complex<double> (complex-step differentiation) and in
// long double (x87 extended precision, 64-bit significand: the same model
// constants with 11 more bits in every operation, which measures how much of
// a difference between two FP64 implementations is FP64 rounding).
// Built with -O2 -ffp-contract=off, no fast-math.

#include <quadmath.h>

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

constexpr int Q = 37;
using cplx = std::complex<double>;
using quad = __float128;

// ---------------------------------------------------------------------------
// Velocity set and quadrature weights.
//
// Reading: the paper states only that populations travel at most three sites,
// and Fig. 4 shows two offsets.  The set is every integer vector c with |c|^2 <= 10
// (37 vectors: families (0,0) (1,0) (1,1) (2,0) (2,1) (2,2) (3,0) (3,1) with
// their images).  Labels follow cx descending, then cy ascending, which puts
// (3,-1) at l=0 and (3,0) at l=1 as in Fig. 4 and makes l and 36-l opposite.
//
// Weights w_l (one per family) and the scale r (xi_l = r c_l) are fixed by
// requiring the rule to integrate the standard 2-D Gaussian exactly:
//   sum_l w_l xi_lx^p xi_ly^q = m_p m_q,  m_0=1, m_2=1, m_4=3, m_6=15, m_8=105
// for the nine even conditions (p,q) in {00,20,40,22,60,42,80,62,44}.
// For fixed r this is linear in the 8 weights; r is the value at which the
// 9x9 augmented matrix [A(r) | m] is singular.  The root is bracketed on a
// grid and bisected, then the weights follow from the normal equations, all
// in binary128 (__float128) so that the rounded doubles are exact to 1 ulp.
// ---------------------------------------------------------------------------
struct Model {
  int cx[Q], cy[Q], fam[Q];  // integer hop e_l = (cx, cy) and its family
  double w[Q];
  double r;
  double H[Q][5][5];  // He_p(r cx_l) He_q(r cy_l), filled for p + q <= 4
  // the same constants rounded from the binary128 solve to long double
  long double wx[Q], rx, Hx[Q][5][5];
  bool ok;
};

const int kFamilies[8][2] = {{0, 0}, {0, 1}, {1, 1}, {0, 2},
                             {1, 2}, {2, 2}, {0, 3}, {1, 3}};
const int kConds[9][2] = {{0, 0}, {2, 0}, {4, 0}, {2, 2}, {6, 0},
                          {4, 2}, {8, 0}, {6, 2}, {4, 4}};

quad gauss_moment(int p) {  // E[z^p] for standard normal z, p even
  quad m = quad(1);
  for (int k = p - 1; k > 0; k -= 2) m *= k;
  return m;
}

quad ipow(quad x, int p) {
  quad v = quad(1);
  for (int i = 0; i < p; ++i) v *= x;
  return v;
}

// rows = conditions, cols = 8 family weights (+ the right-hand side in col 8)
void quadrature_matrix(const Model& M, quad r, quad A[9][9]) {
  for (int i = 0; i < 9; ++i) {
    for (int j = 0; j < 9; ++j) A[i][j] = quad(0);
    const int p = kConds[i][0], q = kConds[i][1];
    for (int l = 0; l < Q; ++l)
      A[i][M.fam[l]] += ipow(r * M.cx[l], p) * ipow(r * M.cy[l], q);
    A[i][8] = gauss_moment(p) * gauss_moment(q);
  }
}

quad det9(quad A[9][9]) {  // Gaussian elimination, partial pivot
  quad a[9][9];
  std::memcpy(a, A, sizeof(a));
  quad d = quad(1);
  for (int c = 0; c < 9; ++c) {
    int piv = c;
    for (int i = c + 1; i < 9; ++i)
      if (fabsq(a[i][c]) > fabsq(a[piv][c])) piv = i;
    if (a[piv][c] == quad(0)) return quad(0);
    if (piv != c) {
      for (int j = 0; j < 9; ++j) std::swap(a[c][j], a[piv][j]);
      d = -d;
    }
    d *= a[c][c];
    for (int i = c + 1; i < 9; ++i) {
      const quad f = a[i][c] / a[c][c];
      for (int j = c; j < 9; ++j) a[i][j] -= f * a[c][j];
    }
  }
  return d;
}

bool solve_spd(quad N[8][8], quad b[8], quad x[8]) {
  // Gaussian elimination with partial pivoting on an 8x8 system.
  quad a[8][9];
  for (int i = 0; i < 8; ++i) {
    for (int j = 0; j < 8; ++j) a[i][j] = N[i][j];
    a[i][8] = b[i];
  }
  for (int c = 0; c < 8; ++c) {
    int piv = c;
    for (int i = c + 1; i < 8; ++i)
      if (fabsq(a[i][c]) > fabsq(a[piv][c])) piv = i;
    if (a[piv][c] == quad(0)) return false;
    for (int j = 0; j < 9; ++j) std::swap(a[c][j], a[piv][j]);
    for (int i = 0; i < 8; ++i) {
      if (i == c) continue;
      const quad f = a[i][c] / a[c][c];
      for (int j = c; j < 9; ++j) a[i][j] -= f * a[c][j];
    }
  }
  for (int i = 0; i < 8; ++i) x[i] = a[i][8] / a[i][i];
  return true;
}

// Probabilists' Hermite polynomials He_0..He_4.
quad hermite_q(int n, quad x) {
  switch (n) {
    case 0: return quad(1);
    case 1: return x;
    case 2: return x * x - 1;
    case 3: return x * x * x - 3 * x;
    default: return x * x * x * x - 6 * x * x + 3;
  }
}

Model build_model() {
  Model M{};
  int n = 0;
  for (int cx = 3; cx >= -3; --cx)
    for (int cy = -3; cy <= 3; ++cy)
      if (cx * cx + cy * cy <= 10) {
        M.cx[n] = cx;
        M.cy[n] = cy;
        ++n;
      }
  M.ok = (n == Q);
  if (!M.ok) return M;
  for (int l = 0; l < Q; ++l) {
    int a = std::abs(M.cx[l]), b = std::abs(M.cy[l]);
    if (a > b) std::swap(a, b);
    M.fam[l] = -1;
    for (int k = 0; k < 8; ++k)
      if (kFamilies[k][0] == a && kFamilies[k][1] == b) M.fam[l] = k;
    if (M.fam[l] < 0) M.ok = false;
  }
  // Bracket the root of det[A(r)|m] on r in [0.5, 2.5].
  quad A[9][9];
  quad lo = 0, hi = 0;
  bool found = false;
  quad prev_r = quad(0.5), prev_d;
  quadrature_matrix(M, prev_r, A);
  prev_d = det9(A);
  for (int i = 1; i <= 2000 && !found; ++i) {
    const quad rr = quad(0.5) + quad(i) / 1000;
    quadrature_matrix(M, rr, A);
    const quad d = det9(A);
    if ((d > 0) != (prev_d > 0)) {
      lo = prev_r;
      hi = rr;
      found = true;
    }
    prev_r = rr;
    prev_d = d;
  }
  if (!found) {
    M.ok = false;
    return M;
  }
  quadrature_matrix(M, lo, A);
  const bool lo_pos = det9(A) > 0;
  for (int it = 0; it < 200; ++it) {
    const quad mid = quad(0.5) * (lo + hi);
    if (mid == lo || mid == hi) break;
    quadrature_matrix(M, mid, A);
    if ((det9(A) > 0) == lo_pos)
      lo = mid;
    else
      hi = mid;
  }
  const quad r = quad(0.5) * (lo + hi);
  quadrature_matrix(M, r, A);
  // Normal equations A^T A W = A^T m over the nine conditions.
  quad N[8][8], b[8], W[8];
  for (int i = 0; i < 8; ++i) {
    b[i] = 0;
    for (int j = 0; j < 8; ++j) {
      N[i][j] = 0;
      for (int k = 0; k < 9; ++k) N[i][j] += A[k][i] * A[k][j];
    }
    for (int k = 0; k < 9; ++k) b[i] += A[k][i] * A[k][8];
  }
  if (!solve_spd(N, b, W)) M.ok = false;
  M.r = (double)r;
  for (int l = 0; l < Q; ++l) M.w[l] = (double)W[M.fam[l]];
  M.rx = (long double)r;
  for (int l = 0; l < Q; ++l) M.wx[l] = (long double)W[M.fam[l]];
  for (int l = 0; l < Q; ++l)
    for (int p = 0; p <= 4; ++p)
      for (int q = 0; q <= 4; ++q)
        M.Hx[l][p][q] = (p + q <= 4) ? (long double)(hermite_q(p, r * M.cx[l]) *
                                                      hermite_q(q, r * M.cy[l]))
                                     : 0.0L;
  // The Hermite table is rounded once from its binary128 value: evaluated in
  // FP64 from the rounded r, He_4(2r) = 16r^4 - 24r^2 + 3 would lose about
  // eight bits to cancellation, a perturbation of the model that the
  // Rayleigh-Taylor flow carries into the velocity field (~1e-12 of max|u|
  // after 50 steps).
  for (int l = 0; l < Q; ++l)
    for (int p = 0; p <= 4; ++p)
      for (int q = 0; q <= 4; ++q)
        M.H[l][p][q] = (p + q <= 4) ? (double)(hermite_q(p, r * M.cx[l]) *
                                               hermite_q(q, r * M.cy[l]))
                                    : 0.0;
  return M;
}

const Model& model() {
  static const Model M = build_model();
  return M;
}

// The model's constants in the working precision of S: the FP64 ones for
// double and complex<double>; for long double the ones rounded from the
// binary128 solve to long double, so that a long double run evaluates the
// model of the unrounded quadrature (to ~1e-19) rather than the FP64-rounded
// one.
template <class S>
struct Consts {
  static double w(int l) { return model().w[l]; }
  static double r() { return model().r; }
  static double H(int l, int p, int q) { return model().H[l][p][q]; }
};
template <>
struct Consts<long double> {
  static long double w(int l) { return model().wx[l]; }
  static long double r() { return model().rx; }
  static long double H(int l, int p, int q) { return model().Hx[l][p][q]; }
};

double factorial(int n) {
  double v = 1;
  for (int k = 2; k <= n; ++k) v *= k;
  return v;
}

// ---------------------------------------------------------------------------
// Units.  A population hops by the integer vector e_l per step (propagate);
// its lattice velocity, the c_l of Eqs. (1)-(2), is c_l = r e_l, with r the
// scale fixed by the quadrature above.  rho, u and T are measured with these
// c_l, so the quadrature's own Gaussian has T = 1 (the reference
// temperature) and u, T, g share the units of c_l (one time step = 1).
// Reading: the paper prints Eq. (2) with the lattice velocities c_l without
// giving them; the scaled set is the model's native one, and it is the unit
// in which the walls' 0.5 / 1.5 temperatures lie in the range where the
// uniform state is linearly stable at tau = 0.7.
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// Equilibrium.
//
// Reading: the paper says only that f^eq is a known function of (rho, u, T)
// and that the model works in a Hermite basis.  f^eq is the Hermite expansion
// of the Maxwellian up to fourth order, with Theta = T - 1:
//   f^eq_l = w_l rho [ 1 + cu + (cu^2 - u^2 + Theta (c2 - 2)) / 2
//            + cu (cu^2 - 3 u^2 + 3 Theta (c2 - 4)) / 6
//            + ( cu^4 - 6 cu^2 u^2 + 3 u^4
//                + 6 Theta (cu^2 (c2 - 6) + u^2 (4 - c2))
//                + 3 Theta^2 (c2^2 - 8 c2 + 8) ) / 24 ]
// with cu = c_l . u, c2 = |c_l|^2 (the D = 2 tensor-Hermite contractions of
// the Gaussian's Hermite moments of orders 0..4).
// ---------------------------------------------------------------------------
template <class S>
void equilibrium(S rho, S ux, S uy, S T, S* feq) {
  const Model& M = model();
  const auto r = Consts<S>::r();
  const S th = T - 1.0;
  const S U2 = ux * ux + uy * uy;
  for (int l = 0; l < Q; ++l) {
    const auto xx = r * M.cx[l], xy = r * M.cy[l];
    const auto x2 = xx * xx + xy * xy;
    const S xu = xx * ux + xy * uy;
    const S t1 = xu;
    const S t2 = (xu * xu - U2 + th * (x2 - 2.0)) / 2.0;
    const S t3 = xu * (xu * xu - 3.0 * U2 + 3.0 * th * (x2 - 4.0)) / 6.0;
    const S t4 = (xu * xu * xu * xu - 6.0 * xu * xu * U2 + 3.0 * U2 * U2 +
                  6.0 * th * (xu * xu * (x2 - 6.0) + U2 * (4.0 - x2)) +
                  3.0 * th * th * (x2 * x2 - 8.0 * x2 + 8.0)) /
                 24.0;
    feq[l] = Consts<S>::w(l) * rho * (1.0 + t1 + t2 + t3 + t4);
  }
}

// Eq. (2): rho, u and T of one site's populations, with c_l = r e_l.
template <class S>
void macroscopic(const S* f, S& rho, S& ux, S& uy, S& T) {
  const Model& M = model();
  const auto r = Consts<S>::r();
  S m0(0.0), jx(0.0), jy(0.0), e(0.0);
  for (int l = 0; l < Q; ++l) {
    const auto cx = r * M.cx[l], cy = r * M.cy[l];
    m0 += f[l];
    jx += cx * f[l];
    jy += cy * f[l];
    e += (cx * cx + cy * cy) * f[l];
  }
  rho = m0;
  ux = jx / rho;
  uy = jy / rho;
  // D rho T = sum |c - u|^2 f = sum |c|^2 f - rho |u|^2, with D = 2.
  T = (e - rho * (ux * ux + uy * uy)) / (2.0 * rho);
}

struct Params {
  double tau, gx, gy, t_bottom, t_top;
  int32_t regularize, ybc;  // ybc: 0 = walls at y = 0 and y = Ly-1, 1 = periodic
};

inline long idx(int l, int x, int y, int lx, int ly) {
  return ((long)l * lx + x) * ly + y;
}

inline int wrap(int a, int n) { return ((a % n) + n) % n; }

// ---------------------------------------------------------------------------
// propagate (Sec. 2, Eq. (1) left side; Fig. 4): after the step the
// population l at x is the one that sat at x - c_l.  x is periodic (the halo
// columns of Sec. 2/4 hold copies of the opposite edge).  With walls, a source
// row outside [0, Ly) does not exist: that slot is "unknown" and is set to NaN
// here; bc fills it.  With ybc = periodic, y wraps as x does.
// ---------------------------------------------------------------------------
template <class S>
void propagate(int lx, int ly, int ybc, const S* f, S* ft) {
  const Model& M = model();
#pragma omp parallel for schedule(static)
  for (int x = 0; x < lx; ++x)
    for (int y = 0; y < ly; ++y)
      for (int l = 0; l < Q; ++l) {
        const int xs = wrap(x - M.cx[l], lx);
        int ys = y - M.cy[l];
        if (ybc == 1) {
          ys = wrap(ys, ly);
        } else if (ys < 0 || ys >= ly) {
          ft[idx(l, x, y, lx, ly)] = S(std::nan(""));
          continue;
        }
        ft[idx(l, x, y, lx, ly)] = f[idx(l, xs, ys, lx, ly)];
      }
}

// ---------------------------------------------------------------------------
// bc (Sec. 2: after propagate, fixes the populations at the top and bottom
// edges: constant temperature, zero velocity).
//
// Reading (the scheme is not given): at a site whose unknown set U is not
// empty (rows 0..2 take T_bottom, rows Ly-3..Ly-1 take T_top), let K be the
// known populations and v_l = f^eq_l(rho=1, u=0, T_wall).  The unknown ones
// are set to rho_w v_l with rho_w = (sum_K f_l) / (sum_K v_l): the wall emits
// a resting Maxwellian at the wall temperature, scaled so that it carries
// the same mass as what arrived.
// ---------------------------------------------------------------------------
template <class S>
void boundary_site(int y, int ly, const S* vb, const S* vt, S* ft) {
  const Model& M = model();
  if (y >= 3 && y < ly - 3) return;
  const S* v = (y < 3) ? vb : vt;
  bool unknown[Q];
  bool any = false;
  for (int l = 0; l < Q; ++l) {
    const int ys = y - M.cy[l];
    unknown[l] = (ys < 0 || ys >= ly);
    any = any || unknown[l];
  }
  if (!any) return;
  S num(0.0), den(0.0);
  for (int l = 0; l < Q; ++l)
    if (!unknown[l]) {
      num += ft[l];
      den += v[l];
    }
  const S rho_w = num / den;
  for (int l = 0; l < Q; ++l)
    if (unknown[l]) ft[l] = rho_w * v[l];
}

template <class S>
void boundary(int lx, int ly, double t_bottom, double t_top, S* ft) {
  S vb[Q], vt[Q];
  equilibrium<S>(S(1.0), S(0.0), S(0.0), S(t_bottom), vb);
  equilibrium<S>(S(1.0), S(0.0), S(0.0), S(t_top), vt);
#pragma omp parallel for schedule(static)
  for (int x = 0; x < lx; ++x)
    for (int y = 0; y < ly; ++y) {
      if (y >= 3 && y < ly - 3) continue;
      S site[Q];
      for (int l = 0; l < Q; ++l) site[l] = ft[idx(l, x, y, lx, ly)];
      boundary_site<S>(y, ly, vb, vt, site);
      for (int l = 0; l < Q; ++l) ft[idx(l, x, y, lx, ly)] = site[l];
    }
}

// ---------------------------------------------------------------------------
// collide (Sec. 2, Eq. (1) right side, with the Hermite projection).
//
// Per site: moments of Eq. (2); gravity g enters as a shift of the
// equilibrium's arguments (reading, forcing is not described):
//   u* = u + tau g,   T* = T + tau (1 - tau) |g|^2 / D,
// which adds exactly rho g to the momentum and rho (2 u.g + |g|^2) to
// sum |c|^2 f per step.  Then the BGK value
//   h_l = (1 - 1/tau) f_l + f^eq_l(rho, u*, T*) / tau
// and, with regularize = 1 (our reading of the Hermite-basis projection that
// Sec. 2 adds for stability), its projection onto the Hermite polynomials of
// total order <= 4:
//   A_pq = sum_m h_m He_p(xi_mx) He_q(xi_my),
//   f'_l = w_l sum_{p+q<=4} A_pq He_p(xi_lx) He_q(xi_ly) / (p! q!).
// regularize = 0 returns h (plain BGK of Eq. (1)).
// ---------------------------------------------------------------------------
template <class S>
void collide_site(const Params& P, const S* ft, S* out) {
  const Model& M = model();
  S rho, ux, uy, T;
  macroscopic<S>(ft, rho, ux, uy, T);
  const double tau = P.tau;
  const S uxs = ux + tau * P.gx;
  const S uys = uy + tau * P.gy;
  const S Ts = T + tau * (1.0 - tau) * (P.gx * P.gx + P.gy * P.gy) / 2.0;
  S feq[Q], h[Q];
  equilibrium<S>(rho, uxs, uys, Ts, feq);
  // the two BGK weights, 1/tau and 1 - 1/tau, are formed once in the working
  // precision; their sum is then exactly one (1 - omega is exact for
  // 1/2 <= omega <= 2), so the relaxation itself adds no bias to the mass
  const S omega = S(1.0) / S(tau);
  const S keep = S(1.0) - omega;
  for (int l = 0; l < Q; ++l) h[l] = keep * ft[l] + omega * feq[l];
  if (!P.regularize) {
    for (int l = 0; l < Q; ++l) out[l] = h[l];
    return;
  }
  S A[5][5];
  for (int p = 0; p <= 4; ++p)
    for (int q = 0; p + q <= 4; ++q) {
      S a(0.0);
      for (int m = 0; m < Q; ++m) a += h[m] * Consts<S>::H(m, p, q);
      A[p][q] = a;
    }
  for (int l = 0; l < Q; ++l) {
    S s(0.0);
    for (int p = 0; p <= 4; ++p)
      for (int q = 0; p + q <= 4; ++q)
        s += A[p][q] * Consts<S>::H(l, p, q) / (factorial(p) * factorial(q));
    out[l] = Consts<S>::w(l) * s;
  }
}

template <class S>
void collide(int lx, int ly, const Params& P, const S* ft, S* fout) {
#pragma omp parallel for schedule(static)
  for (int x = 0; x < lx; ++x)
    for (int y = 0; y < ly; ++y) {
      S in[Q], out[Q];
      for (int l = 0; l < Q; ++l) in[l] = ft[idx(l, x, y, lx, ly)];
      collide_site<S>(P, in, out);
      for (int l = 0; l < Q; ++l) fout[idx(l, x, y, lx, ly)] = out[l];
    }
}

// One full time step, in the order of Sec. 2: propagate, bc, collide.
template <class S>
void step(int lx, int ly, const Params& P, S* f, S* tmp) {
  propagate<S>(lx, ly, P.ybc, f, tmp);
  if (P.ybc == 0) boundary<S>(lx, ly, P.t_bottom, P.t_top, tmp);
  collide<S>(lx, ly, P, tmp, f);
}

template <class S>
void init_feq(int lx, int ly, const S* rho, const S* ux, const S* uy,
              const S* T, S* f) {
#pragma omp parallel for schedule(static)
  for (int x = 0; x < lx; ++x)
    for (int y = 0; y < ly; ++y) {
      const long s = (long)x * ly + y;
      S feq[Q];
      equilibrium<S>(rho[s], ux[s], uy[s], T[s], feq);
      for (int l = 0; l < Q; ++l) f[idx(l, x, y, lx, ly)] = feq[l];
    }
}

// Total kinetic energy (1/2) sum rho |u|^2 over the lattice.
template <class S>
S kinetic_energy(int lx, int ly, const S* f) {
  S ke(0.0);
  for (int x = 0; x < lx; ++x)
    for (int y = 0; y < ly; ++y) {
      S in[Q];
      for (int l = 0; l < Q; ++l) in[l] = f[idx(l, x, y, lx, ly)];
      S rho, ux, uy, T;
      macroscopic<S>(in, rho, ux, uy, T);
      ke += 0.5 * rho * (ux * ux + uy * uy);
    }
  return ke;
}

}  // namespace

extern "C" {

// Returns 0 when the quadrature solve succeeded.  cx, cy, w: 37 entries.
int oracle_model(int32_t* cx, int32_t* cy, double* w, double* r) {
  const Model& M = model();
  for (int l = 0; l < Q; ++l) {
    cx[l] = M.cx[l];
    cy[l] = M.cy[l];
    w[l] = M.w[l];
  }
  *r = M.r;
  return M.ok ? 0 : -1;
}

void oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int oracle_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_equilibrium(double rho, double ux, double uy, double T,
                        double* feq) {
  equilibrium<double>(rho, ux, uy, T, feq);
}

void oracle_macroscopic(const double* f, double* out4) {
  macroscopic<double>(f, out4[0], out4[1], out4[2], out4[3]);
}

void oracle_collide_site(const Params* P, const double* ft, double* out) {
  collide_site<double>(*P, ft, out);
}

// Fields are x-major [lx][ly]; populations are [37][lx][ly].
void oracle_init_feq(int lx, int ly, const double* rho, const double* ux,
                     const double* uy, const double* T, double* f) {
  init_feq<double>(lx, ly, rho, ux, uy, T, f);
}

void oracle_propagate(int lx, int ly, int ybc, const double* f, double* ft) {
  propagate<double>(lx, ly, ybc, f, ft);
}

void oracle_bc(int lx, int ly, double t_bottom, double t_top, double* ft) {
  boundary<double>(lx, ly, t_bottom, t_top, ft);
}

void oracle_collide(int lx, int ly, const Params* P, const double* ft,
                    double* fout) {
  collide<double>(lx, ly, *P, ft, fout);
}

// Advances f (in place) by nsteps full steps.
void oracle_run(int lx, int ly, const Params* P, double* f, int nsteps) {
  std::vector<double> tmp((size_t)Q * lx * ly);
  for (int n = 0; n < nsteps; ++n) step<double>(lx, ly, *P, f, tmp.data());
}

void oracle_moments(int lx, int ly, const double* f, double* rho, double* ux,
                    double* uy, double* T) {
#pragma omp parallel for schedule(static)
  for (int x = 0; x < lx; ++x)
    for (int y = 0; y < ly; ++y) {
      double in[Q];
      for (int l = 0; l < Q; ++l) in[l] = f[idx(l, x, y, lx, ly)];
      const long s = (long)x * ly + y;
      macroscopic<double>(in, rho[s], ux[s], uy[s], T[s]);
    }
}

// One full step evaluated at n chosen sites only: out[i*37 + l] is the
// post-collision population l at (xs[i], ys[i]) after propagate, bc and
// collide applied to the state f (for spot checks of large lattices).
void oracle_step_sites(int lx, int ly, const Params* P, const double* f, int n,
                       const int32_t* xs, const int32_t* ys, double* out) {
  const Model& M = model();
  double vb[Q], vt[Q];
  equilibrium<double>(1.0, 0.0, 0.0, P->t_bottom, vb);
  equilibrium<double>(1.0, 0.0, 0.0, P->t_top, vt);
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i) {
    const int x = xs[i], y = ys[i];
    double ft[Q];
    for (int l = 0; l < Q; ++l) {
      const int xs_ = wrap(x - M.cx[l], lx);
      int ys_ = y - M.cy[l];
      if (P->ybc == 1) ys_ = wrap(ys_, ly);
      ft[l] = (ys_ < 0 || ys_ >= ly) ? std::nan("") : f[idx(l, xs_, ys_, lx, ly)];
    }
    if (P->ybc == 0) boundary_site<double>(y, ly, vb, vt, ft);
    collide_site<double>(*P, ft, out + (size_t)i * Q);
  }
}

double oracle_kinetic_energy(int lx, int ly, const double* f) {
  return kinetic_energy<double>(lx, ly, f);
}

// Complex-step form: fields are complex (interleaved re, im).  Initialises
// f = f^eq(rho0, u0, T0), runs nsteps steps and returns the kinetic energy
// (complex) in ke[0], ke[1].  Im(KE) / h is dKE/dparam when the inputs carry
// i h dfield/dparam in their imaginary parts.
void oracle_ke_after_steps_complex(int lx, int ly, const Params* P,
                                   const double* rho0, const double* ux0,
                                   const double* uy0, const double* T0,
                                   int nsteps, double* ke) {
  const size_t S = (size_t)lx * ly;
  std::vector<cplx> f((size_t)Q * S), tmp((size_t)Q * S);
  init_feq<cplx>(lx, ly, reinterpret_cast<const cplx*>(rho0),
                 reinterpret_cast<const cplx*>(ux0),
                 reinterpret_cast<const cplx*>(uy0),
                 reinterpret_cast<const cplx*>(T0), f.data());
  for (int n = 0; n < nsteps; ++n) step<cplx>(lx, ly, *P, f.data(), tmp.data());
  const cplx k = kinetic_energy<cplx>(lx, ly, f.data());
  ke[0] = k.real();
  ke[1] = k.imag();
}

// Extended-precision run: f (FP64 [37][lx][ly]) advanced by nsteps full steps
// in long double; the moments of Eq. (2) of the result, also in long double,
// rounded to FP64 into rho, ux, uy, T ([lx][ly]); the populations into
// f_out when it is not NULL.
void oracle_run_moments_ld(int lx, int ly, const Params* P, const double* f, int nsteps,
                           double* rho, double* ux, double* uy, double* T, double* f_out) {
  using ld = long double;
  const size_t S = (size_t)lx * ly;
  std::vector<ld> g((size_t)Q * S), tmp((size_t)Q * S);
  for (size_t i = 0; i < (size_t)Q * S; ++i) g[i] = f[i];
  for (int n = 0; n < nsteps; ++n) step<ld>(lx, ly, *P, g.data(), tmp.data());
  for (int x = 0; x < lx; ++x)
    for (int y = 0; y < ly; ++y) {
      ld in[Q];
      for (int l = 0; l < Q; ++l) in[l] = g[idx(l, x, y, lx, ly)];
      ld r, u, v, t;
      macroscopic<ld>(in, r, u, v, t);
      const long s = (long)x * ly + y;
      rho[s] = double(r);
      ux[s] = double(u);
      uy[s] = double(v);
      T[s] = double(t);
    }
  if (f_out)
    for (size_t i = 0; i < (size_t)Q * S; ++i) f_out[i] = double(g[i]);
}

// Complex-step forms for linearisations: f_c is complex [37][lx][ly]
// (interleaved re, im), advanced in place by nsteps full steps.
void oracle_run_complex(int lx, int ly, const Params* P, double* f_c, int nsteps) {
  std::vector<cplx> tmp((size_t)Q * lx * ly);
  cplx* f = reinterpret_cast<cplx*>(f_c);
  for (int n = 0; n < nsteps; ++n) step<cplx>(lx, ly, *P, f, tmp.data());
}

void oracle_init_feq_complex(int lx, int ly, const double* rho, const double* ux,
                             const double* uy, const double* T, double* f_c) {
  init_feq<cplx>(lx, ly, reinterpret_cast<const cplx*>(rho), reinterpret_cast<const cplx*>(ux),
                 reinterpret_cast<const cplx*>(uy), reinterpret_cast<const cplx*>(T),
                 reinterpret_cast<cplx*>(f_c));
}

void oracle_kinetic_energy_complex(int lx, int ly, const double* f_c, double* ke) {
  const cplx k = kinetic_energy<cplx>(lx, ly, reinterpret_cast<const cplx*>(f_c));
  ke[0] = k.real();
  ke[1] = k.imag();
}

}  // extern "C"
