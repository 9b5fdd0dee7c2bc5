// Device arithmetic on non-overlapping floating-point expansions of NC
// binary64 components (DD NC=2, TD NC=3, QD NC=4).
//
// These are the multiple-precision operations the LU keeps outside the
// Ozaki-II product (Sec. 3.4 of the paper: panel, row interchanges, U12
// solve, plus the native comparator).  They follow one fixed specification so
// that every result is reproducible bit for bit:
//   * TwoSum (Knuth) and TwoProd (exact error from one FMA);
//   * terms are sorted by decreasing magnitude with Batcher's merge-exchange
//     network (Knuth, TAOCP 3, 5.2.2, Algorithm M), then renormalised by a
//     bottom-up VecSum followed by a top-down error-branch compression that
//     keeps the first NC non-zero partial sums (Joldes, Muller, Popescu);
//   * a*b: partial products of order i+j <= NC-2 exact (TwoProd; the error
//     joins the next order), order NC-1 plain products, higher orders
//     dropped;
//   * c - a*b: the rounded product subtracted with the addition above;
//   * a/b: long division producing NC+1 quotient digits.
// All loops have compile-time trip counts and are unrolled, so the terms live
// in registers; the code must be built with -ffp-contract=off.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define OZX_HD __host__ __device__ __forceinline__

namespace ozx {

OZX_HD void two_sum(double a, double b, double &s, double &e) {
  double ss = a + b;
  double bp = ss - a;
  double ap = ss - bp;
  e = (a - ap) + (b - bp);
  s = ss;
}

OZX_HD void two_prod(double a, double b, double &p, double &e) {
  double pp = a * b;
  e = __builtin_fma(a, b, -pp);
  p = pp;
}

// ---------------------------------------------------------------------------
// Batcher merge-exchange network, generated at compile time.
// ---------------------------------------------------------------------------
template <int K>
struct SortNet {
  int n;
  unsigned char a[128];
  unsigned char b[128];
};

template <int K>
constexpr SortNet<K> make_sortnet() {
  SortNet<K> net{};
  net.n = 0;
  if (K < 2) return net;
  int t = 0;
  while ((1 << t) < K) ++t;
  for (int p = 1 << (t - 1); p > 0; p >>= 1) {
    int q = 1 << (t - 1), r = 0, d = p;
    for (;;) {
      for (int i = 0; i + d < K; ++i) {
        if ((i & p) == r) {
          net.a[net.n] = (unsigned char)i;
          net.b[net.n] = (unsigned char)(i + d);
          ++net.n;
        }
      }
      if (q == p) break;
      d = q - p;
      q >>= 1;
      r = p;
    }
  }
  return net;
}

template <int K>
OZX_HD void sort_desc(double (&x)[K]) {
  constexpr SortNet<K> net = make_sortnet<K>();
#pragma unroll
  for (int c = 0; c < net.n; ++c) {
    double u = x[net.a[c]], v = x[net.b[c]];
    bool sw = __builtin_fabs(v) > __builtin_fabs(u);
    x[net.a[c]] = sw ? v : u;
    x[net.b[c]] = sw ? u : v;
  }
}

// Renormalise K sorted terms into NC components.
template <int K, int NC>
OZX_HD void renorm(double (&x)[K], double (&y)[NC]) {
  double s = x[K - 1];
#pragma unroll
  for (int i = K - 2; i >= 0; --i) {
    double t;
    two_sum(x[i], s, s, t);
    x[i + 1] = t;
  }
  x[0] = s;
#pragma unroll
  for (int i = 0; i < NC; ++i) y[i] = 0.0;
  int j = 0;
  double eps = x[0];
#pragma unroll
  for (int i = 1; i < K; ++i) {
    double r, e;
    two_sum(eps, x[i], r, e);
    const bool live = j < NC;
    const bool emit = live && (e != 0.0);
#pragma unroll
    for (int q = 0; q < NC; ++q)
      if (emit && j == q) y[q] = r;
    eps = live ? (e != 0.0 ? e : r) : eps;
    j += emit ? 1 : 0;
  }
#pragma unroll
  for (int q = 0; q < NC; ++q)
    if (j == q) y[q] = eps;
}

template <int NC>
OZX_HD void add(const double (&a)[NC], const double (&b)[NC], double (&r)[NC]) {
  double x[2 * NC];
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    x[i] = a[i];
    x[NC + i] = b[i];
  }
  sort_desc<2 * NC>(x);
  renorm<2 * NC, NC>(x, r);
}

template <int NC>
OZX_HD void mul(const double (&a)[NC], const double (&b)[NC], double (&r)[NC]) {
  double terms[NC * NC];
  double err[NC + 1][NC + 1];
  int k = 0;
#pragma unroll
  for (int o = 0; o < NC; ++o) {
#pragma unroll
    for (int i = 0; i <= o; ++i) {
      const int j = o - i;
      if (o <= NC - 2) {
        double p, e;
        two_prod(a[i], b[j], p, e);
        terms[k++] = p;
        err[o + 1][i] = e;
      } else {
        terms[k++] = a[i] * b[j];
      }
    }
    if (o >= 1) {
#pragma unroll
      for (int i = 0; i < o; ++i) terms[k++] = err[o][i];
    }
  }
  sort_desc<NC * NC>(terms);
  renorm<NC * NC, NC>(terms, r);
}

// r = c - a*b
template <int NC>
OZX_HD void fms(const double (&c)[NC], const double (&a)[NC], const double (&b)[NC],
                                    double (&r)[NC]) {
  double p[NC];
  mul<NC>(a, b, p);
#pragma unroll
  for (int i = 0; i < NC; ++i) p[i] = -p[i];
  add<NC>(c, p, r);
}

// r = b * q, q a double
template <int NC>
OZX_HD void mul_d(const double (&b)[NC], double q, double (&r)[NC]) {
  double terms[2 * NC - 1];
  int k = 0;
  double e_prev = 0.0;
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    if (i <= NC - 2) {
      double p, e;
      two_prod(b[i], q, p, e);
      terms[k++] = p;
      if (i >= 1) terms[k++] = e_prev;
      e_prev = e;
    } else {
      terms[k++] = b[i] * q;
      if (i >= 1) terms[k++] = e_prev;
    }
  }
  sort_desc<2 * NC - 1>(terms);
  renorm<2 * NC - 1, NC>(terms, r);
}

template <int NC>
OZX_HD void div(const double (&a)[NC], const double (&b)[NC], double (&r)[NC]) {
  double q[NC + 1];
  double rem[NC];
#pragma unroll
  for (int i = 0; i < NC; ++i) rem[i] = a[i];
#pragma unroll
  for (int k = 0; k <= NC; ++k) {
    q[k] = rem[0] / b[0];
    if (k < NC) {
      double t[NC], nr[NC];
      mul_d<NC>(b, q[k], t);
#pragma unroll
      for (int i = 0; i < NC; ++i) t[i] = -t[i];
      add<NC>(rem, t, nr);
#pragma unroll
      for (int i = 0; i < NC; ++i) rem[i] = nr[i];
    }
  }
  sort_desc<NC + 1>(q);
  renorm<NC + 1, NC>(q, r);
}

// |a| > |b| in the pivot order: lexicographic on sign-normalised components.
template <int NC>
OZX_HD bool abs_greater(const double (&a)[NC], const double (&b)[NC]) {
  const double sa = a[0] < 0.0 ? -1.0 : 1.0, sb = b[0] < 0.0 ? -1.0 : 1.0;
  int res = 0;  // 0 undecided, 1 greater, -1 smaller
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double x = sa * a[c], y = sb * b[c];
    if (res == 0) res = x > y ? 1 : (x < y ? -1 : 0);
  }
  return res > 0;
}

template <int NC>
OZX_HD bool is_zero(const double (&a)[NC]) {
  bool z = true;
#pragma unroll
  for (int c = 0; c < NC; ++c) z = z && (a[c] == 0.0);
  return z;
}

template <int NC>
OZX_HD void load(const double *p, double (&x)[NC]) {
#pragma unroll
  for (int c = 0; c < NC; ++c) x[c] = p[c];
}

template <int NC>
OZX_HD void store(double *p, const double (&x)[NC]) {
#pragma unroll
  for (int c = 0; c < NC; ++c) p[c] = x[c];
}

}  // namespace ozx
