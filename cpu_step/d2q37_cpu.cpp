// Optimised multicore CPU implementation of the D2Q37 step, for comparison
// with the GPU library.  It is a separate program: the GPU binding never
// calls it, and it is not the oracle (which stays plain and slow).
//
// Method as in the GPU library (Sec. 2 of Calore et al.: propagate, thermal
// walls, Hermite-regularized BGK collision with gravity), laid out for a
// CPU the way the paper's propagate v2 is (Sec. 6, Fig. 10): one column at a
// time, the populations of a column contiguous, the innermost loop running
// along y so that it vectorizes.  Sites are processed in chunks of kVL rows,
// held in vector registers (GCC vector types); every step of the collision is
// a vector operation over the chunk.  Columns are distributed over OpenMP
// threads; x is periodic through a column index wrap.
#include <omp.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>

#include "../paper_1703_00186_amd/csrc/d2q37_constants.h"

namespace {

using namespace d2q37;

constexpr int kVL = 8;   // lanes per chunk (one AVX-512 register of doubles)
constexpr int kPad = 16;  // padding rows above and below a column

struct Params {
  double tau, gx, gy, t_bottom, t_top;
  int32_t regularize, ybc;
};

struct Lattice {
  int lx, ly, ny;
  double* a;  // state, [lx][37][ny] with the physical rows at [kPad, kPad + ly)
  double* b;  // next state
  Params p;
};

typedef double V __attribute__((vector_size(kVL * sizeof(double))));

constexpr double he_val(int e, int n) {
  return (e < 0 && (n & 1)) ? -HE[-e][n] : HE[e < 0 ? -e : e][n];
}
constexpr double hef_val(int e, int n) {
  return (e < 0 && (n & 1)) ? -HEF[-e][n] : HEF[e < 0 ? -e : e][n];
}
constexpr double c2_val(int l) { return R * R * double(EX[l] * EX[l] + EY[l] * EY[l]); }

inline V splat(double v) { return V{} + v; }

inline size_t col(const Lattice& L, int x) { return size_t(x) * Q * L.ny; }

// Thermal wall at one site of rows 0..2 / ly-3..ly-1 (unknown populations
// become rho_w f^eq(1, 0, T_wall), rho_w = sum_known f / sum_known f^eq).
void wall_lane(V (&f)[Q], int k, int y, int ly, const Params& p) {
  const double th = (y < 3 ? p.t_bottom : p.t_top) - 1.0;
  double v[Q];
  double sk = 0.0, vk = 0.0;
  bool unknown[Q];
  for (int l = 0; l < Q; ++l) {
    const double x2 = c2_val(l);
    v[l] = W[l] * (1.0 + 0.5 * th * (x2 - 2.0) + 0.125 * th * th * (x2 * x2 - 8.0 * x2 + 8.0));
    const int ys = y - EY[l];
    unknown[l] = ys < 0 || ys >= ly;
    if (!unknown[l]) {
      sk += f[l][k];
      vk += v[l];
    }
  }
  const double rho_w = sk / vk;
  for (int l = 0; l < Q; ++l)
    if (unknown[l]) f[l][k] = rho_w * v[l];
}

// One chunk of kVL sites: projection onto the 15 Hermite polynomials (grouped
// by x hop), forced equilibrium, relaxation, reconstruction.  All loops have
// compile-time bounds and constant coefficients, so they unroll into vector
// FMAs with the zero coefficients folded away.
__attribute__((always_inline)) inline void collide_chunk(V (&f)[Q], const Params& p) {
  V a[5][5];
#pragma GCC unroll 5
  for (int i = 0; i < 5; ++i)
#pragma GCC unroll 5
    for (int j = 0; j < 5; ++j) a[i][j] = V{};
#pragma GCC unroll 7
  for (int gi = 0; gi < 7; ++gi) {
    const int ex = 3 - gi;
    V s[5] = {V{}, V{}, V{}, V{}, V{}};
#pragma GCC unroll 37
    for (int l = 0; l < Q; ++l) {
      if (EX[l] != ex) continue;
#pragma GCC unroll 5
      for (int q = 0; q < 5; ++q) {
        const double h = he_val(EY[l], q);
        if (h != 0.0) s[q] += h * f[l];
      }
    }
#pragma GCC unroll 5
    for (int i = 0; i < 5; ++i) {
      const double h = he_val(ex, i);
      if (h == 0.0) continue;
#pragma GCC unroll 5
      for (int j = 0; i + j < 5; ++j) a[i][j] += h * s[j];
    }
  }
  const double om = 1.0 / p.tau, keep = 1.0 - om;
  const double dth = p.tau * (1.0 - p.tau) * (p.gx * p.gx + p.gy * p.gy) / 2.0;
  const V rho = a[0][0], inv = 1.0 / rho;
  const V ux = a[1][0] * inv, uy = a[0][1] * inv;
  const V th = 0.5 * ((a[2][0] + a[0][2]) * inv - (ux * ux + uy * uy)) + dth;
  const V Ux = ux + p.tau * p.gx, Uy = uy + p.tau * p.gy;
  const V X2 = Ux * Ux, Y2 = Uy * Uy;
  const V hx[5] = {splat(1.0), Ux, X2 + th, Ux * (X2 + 3.0 * th), X2 * (X2 + 6.0 * th) + 3.0 * th * th};
  const V hy[5] = {splat(1.0), Uy, Y2 + th, Uy * (Y2 + 3.0 * th), Y2 * (Y2 + 6.0 * th) + 3.0 * th * th};
  V b[5][5];
#pragma GCC unroll 5
  for (int i = 0; i < 5; ++i)
#pragma GCC unroll 5
    for (int j = 0; i + j < 5; ++j) {
      const V eq = rho * hx[i] * hy[j];
      b[i][j] = (i == 0 && j == 0) ? rho : (p.regularize ? keep * a[i][j] + om * eq : eq);
    }
  V fin[Q];
  if (!p.regularize)
#pragma GCC unroll 37
    for (int l = 0; l < Q; ++l) fin[l] = f[l];
#pragma GCC unroll 7
  for (int gi = 0; gi < 7; ++gi) {
    const int ex = 3 - gi;
    V P[5];
#pragma GCC unroll 5
    for (int j = 0; j < 5; ++j) {
      V acc = V{};
#pragma GCC unroll 5
      for (int i = 0; i + j < 5; ++i) {
        const double h = hef_val(ex, i);
        if (h != 0.0) acc += h * b[i][j];
      }
      P[j] = acc;
    }
#pragma GCC unroll 37
    for (int l = 0; l < Q; ++l) {
      if (EX[l] != ex) continue;
      V v = V{};
#pragma GCC unroll 5
      for (int j = 0; j < 5; ++j) {
        const double h = W[l] * hef_val(EY[l], j);
        if (h != 0.0) v += h * P[j];
      }
      f[l] = p.regularize ? v : keep * fin[l] + om * v;
    }
  }
}

void step(Lattice& L) {
  const int lx = L.lx, ly = L.ly, ny = L.ny;
  const bool walls = L.p.ybc == 0;
#pragma omp parallel for schedule(static)
  for (int x = 0; x < lx; ++x) {
    const double* src_col[7];
    for (int gi = 0; gi < 7; ++gi) {
      const int xs = ((x - (3 - gi)) % lx + lx) % lx;
      src_col[gi] = L.a + col(L, xs);
    }
    double* dst = L.b + col(L, x);
    for (int y0 = 0; y0 < ly; y0 += kVL) {
      V f[Q];
      for (int l = 0; l < Q; ++l) {
        const double* s = src_col[3 - EX[l]] + size_t(l) * ny + kPad + y0 - EY[l];
        if (walls) {
          std::memcpy(&f[l], s, sizeof(V));
        } else {
          for (int k = 0; k < kVL; ++k) {
            const int ys = ((y0 + k - EY[l]) % ly + ly) % ly;
            f[l][k] = src_col[3 - EX[l]][size_t(l) * ny + kPad + ys];
          }
        }
      }
      const int nk = ly - y0 < kVL ? ly - y0 : kVL;
      if (walls && (y0 < 3 || y0 + kVL > ly - 3))
        for (int k = 0; k < nk; ++k) {
          const int y = y0 + k;
          if (y < 3 || y >= ly - 3) wall_lane(f, k, y, ly, L.p);
        }
      collide_chunk(f, L.p);
      for (int l = 0; l < Q; ++l) {
        double* d = dst + size_t(l) * ny + kPad + y0;
        if (nk == kVL)
          std::memcpy(d, &f[l], sizeof(V));
        else
          for (int k = 0; k < nk; ++k) d[k] = f[l][k];
      }
    }
  }
  double* t = L.a;
  L.a = L.b;
  L.b = t;
}

}  // namespace

extern "C" {

void* cpu_create(int lx, int ly, const Params* p) {
  if (lx < 6 || ly < 6 || !p) return nullptr;
  Lattice* L = new (std::nothrow) Lattice;
  if (!L) return nullptr;
  L->lx = lx;
  L->ly = ly;
  L->ny = (ly + 2 * kPad + kVL - 1) / kVL * kVL;
  L->p = *p;
  const size_t n = size_t(lx) * Q * L->ny;
  L->a = static_cast<double*>(std::aligned_alloc(64, ((n * 8 + 63) / 64) * 64));
  L->b = static_cast<double*>(std::aligned_alloc(64, ((n * 8 + 63) / 64) * 64));
  if (!L->a || !L->b) {
    std::free(L->a);
    std::free(L->b);
    delete L;
    return nullptr;
  }
  // zero everything so padding rows (read by the wall rows' gather) are finite
#pragma omp parallel for schedule(static)
  for (long long i = 0; i < (long long)n; ++i) L->a[i] = L->b[i] = 0.0;
  return L;
}

void cpu_free(void* h) {
  Lattice* L = static_cast<Lattice*>(h);
  if (!L) return;
  std::free(L->a);
  std::free(L->b);
  delete L;
}

// Populations f [37][lx][ly] (any origin, e.g. an equilibrium) -> state.
void cpu_set_populations(void* h, const double* f) {
  Lattice& L = *static_cast<Lattice*>(h);
#pragma omp parallel for schedule(static)
  for (int x = 0; x < L.lx; ++x)
    for (int l = 0; l < Q; ++l)
      for (int y = 0; y < L.ly; ++y)
        L.a[col(L, x) + size_t(l) * L.ny + kPad + y] = f[(size_t(l) * L.lx + x) * L.ly + y];
}

void cpu_get_populations(void* h, double* f) {
  Lattice& L = *static_cast<Lattice*>(h);
#pragma omp parallel for schedule(static)
  for (int x = 0; x < L.lx; ++x)
    for (int l = 0; l < Q; ++l)
      for (int y = 0; y < L.ly; ++y)
        f[(size_t(l) * L.lx + x) * L.ly + y] = L.a[col(L, x) + size_t(l) * L.ny + kPad + y];
}

void cpu_step(void* h, int n) {
  Lattice& L = *static_cast<Lattice*>(h);
  for (int i = 0; i < n; ++i) step(L);
}

void cpu_set_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
}

}  // extern "C"
