// Real Clebsch-Gordan tensors computed at compile time (l <= 3), so the
// tensor-product kernels can unroll over exactly the nonzero entries with
// immediate coefficients.  Same derivation and conventions as the host
// table (Racah's closed formula for the complex coefficients, real basis of
// spherical harmonics without the Condon-Shortley phase, l = 1 as (y, z, x),
// normalisation sum C^2 = 2 l3 + 1, first nonzero entry positive); the host
// checks the two agree when a model is created.
#pragma once

#include "plan.h"

namespace afm {
namespace ct {

constexpr double fact(int n) {
  double r = 1.0;
  for (int k = 2; k <= n; ++k) r *= k;
  return r;
}

constexpr double sqrt_(double x) {
  if (x <= 0.0) return 0.0;
  double r = x > 1.0 ? x : 1.0;
  for (int it = 0; it < 200; ++it) {
    const double nr = 0.5 * (r + x / r);
    if (nr == r) break;
    r = nr;
  }
  return r;
}

constexpr double abs_(double x) { return x < 0 ? -x : x; }

constexpr double cg_complex(int j1, int m1, int j2, int m2, int J, int M) {
  if (m1 + m2 != M || iabs(m1) > j1 || iabs(m2) > j2 || iabs(M) > J) return 0.0;
  if (J < iabs(j1 - j2) || J > j1 + j2) return 0.0;
  double pre = sqrt_((2 * J + 1) * fact(J + j1 - j2) * fact(J - j1 + j2) * fact(j1 + j2 - J) /
                     fact(j1 + j2 + J + 1));
  pre *= sqrt_(fact(J + M) * fact(J - M) * fact(j1 - m1) * fact(j1 + m1) * fact(j2 - m2) * fact(j2 + m2));
  double s = 0.0;
  for (int k = 0; k <= j1 + j2 + J; ++k) {
    const int a = j1 + j2 - J - k, b = j1 - m1 - k, c = j2 + m2 - k, d = J - j2 + m1 + k, e = J - j1 - m2 + k;
    if (a < 0 || b < 0 || c < 0 || d < 0 || e < 0) continue;
    s += ((k & 1) ? -1.0 : 1.0) / (fact(k) * fact(a) * fact(b) * fact(c) * fact(d) * fact(e));
  }
  return pre * s;
}

struct Cx {
  double re = 0.0, im = 0.0;
};
constexpr Cx mul(Cx a, Cx b) { return Cx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
constexpr Cx conj(Cx a) { return Cx{a.re, -a.im}; }

// U[row = m + l][col = mu + l] with Y_real = U Y_complex
constexpr Cx basis(int l, int row, int col) {
  const double r2 = 0.70710678118654752440;
  const int m = row - l, mu = col - l;
  if (m == 0) return (mu == 0) ? Cx{1.0, 0.0} : Cx{};
  if (m > 0) {
    if (mu == m) return Cx{((m & 1) ? -1.0 : 1.0) * r2, 0.0};
    if (mu == -m) return Cx{r2, 0.0};
    return Cx{};
  }
  const int am = -m;
  if (mu == am) return Cx{0.0, -((am & 1) ? -1.0 : 1.0) * r2};
  if (mu == -am) return Cx{0.0, r2};
  return Cx{};
}

struct Tensor {
  double v[343] = {};   // up to 7 x 7 x 7
};

constexpr Tensor real_cg(int l1, int l2, int l3) {
  Tensor T{};
  const int d1 = 2 * l1 + 1, d2 = 2 * l2 + 1, d3 = 2 * l3 + 1;
  Cx C[343] = {};
  double mr = 0.0, mi = 0.0;
  for (int i = 0; i < d1; ++i)
    for (int j = 0; j < d2; ++j)
      for (int k = 0; k < d3; ++k) {
        Cx acc{};
        // each real-basis row has at most two nonzero complex entries, so
        // test those before evaluating the Racah sum
        for (int a = 0; a < d1; ++a) {
          const Cx u1 = basis(l1, i, a);
          if (u1.re == 0.0 && u1.im == 0.0) continue;
          for (int b = 0; b < d2; ++b) {
            const Cx u2 = basis(l2, j, b);
            if (u2.re == 0.0 && u2.im == 0.0) continue;
            const int c = (a - l1) + (b - l2) + l3;
            if (c < 0 || c >= d3) continue;
            const Cx u3 = basis(l3, k, c);
            if (u3.re == 0.0 && u3.im == 0.0) continue;
            const double cc = cg_complex(l1, a - l1, l2, b - l2, l3, c - l3);
            if (cc == 0.0) continue;
            Cx t = mul(mul(conj(u1), conj(u2)), u3);
            acc.re += t.re * cc;
            acc.im += t.im * cc;
          }
        }
        C[(i * d2 + j) * d3 + k] = acc;
        mr = mr > abs_(acc.re) ? mr : abs_(acc.re);
        mi = mi > abs_(acc.im) ? mi : abs_(acc.im);
      }
  const bool use_im = mi > mr;
  double ss = 0.0;
  for (int q = 0; q < d1 * d2 * d3; ++q) {
    double v = use_im ? C[q].im : C[q].re;
    if (abs_(v) < 1e-14) v = 0.0;
    T.v[q] = v;
    ss += v * v;
  }
  const double sc = sqrt_(d3 / ss);
  double first = 0.0;
  for (int q = 0; q < d1 * d2 * d3; ++q) {
    T.v[q] *= sc;
    if (first == 0.0 && abs_(T.v[q]) > 1e-9) first = T.v[q];
  }
  if (first < 0)
    for (int q = 0; q < d1 * d2 * d3; ++q) T.v[q] = -T.v[q] + 0.0;
  return T;
}

// nonzero entries of one tensor
struct Nz {
  int n = 0;
  int m1[48] = {}, m2[48] = {}, m3[48] = {};   // at most 42 nonzeros for l <= 3
  float c[48] = {};
};

constexpr Nz nonzeros(int l1, int l2, int l3) {
  Nz z{};
  const Tensor T = real_cg(l1, l2, l3);
  const int d2 = 2 * l2 + 1, d3 = 2 * l3 + 1;
  for (int i = 0; i < 2 * l1 + 1; ++i)
    for (int j = 0; j < d2; ++j)
      for (int k = 0; k < d3; ++k) {
        const double v = T.v[(i * d2 + j) * d3 + k];
        if (abs_(v) > 1e-12) {
          z.m1[z.n] = i;
          z.m2[z.n] = j;
          z.m3[z.n] = k;
          z.c[z.n] = (float)v;
          ++z.n;
        }
      }
  return z;
}

template <int L1, int L2, int L3>
struct NzCT {
  static constexpr Nz nz = nonzeros(L1, L2, L3);
};

}  // namespace ct
}  // namespace afm
