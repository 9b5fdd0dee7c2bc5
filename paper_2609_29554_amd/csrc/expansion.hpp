// Device arithmetic on non-overlapping floating-point expansions of NC
// binary64 components (DD NC=2, TD NC=3, QD NC=4).
//
// These are the multiple-precision operations the LU keeps outside the
// Ozaki-II product (Sec. 3.4 of the paper: panel, row interchanges, U12
// solve, plus the native comparator).  They follow one fixed specification so
// that every result is reproducible bit for bit:
//   * TwoSum (Knuth) and TwoProd (exact error from one FMA);
//   * renormalisation of K terms into NC components: a bottom-up VecSum, then
//     a top-down error-branch compression that keeps the first NC non-zero
//     partial sums (Joldes, Muller, Popescu);
//   * a+b: the components of a and b (each largest first) merged by
//     magnitude with Batcher's odd-even merge network (triple-double padded
//     with a zero to four), then renormalised;
//   * a*b: partial products summed by order i+j (Hida, Li, Bailey): orders
//     <= NC-2 by TwoProd, with the product errors and the TwoSum errors of
//     each order's sum carried to the next order; order NC-1 plain products
//     and carries summed left to right; higher orders dropped; the NC order
//     sums renormalised;
//   * c - a*b: the rounded product subtracted with the addition above;
//   * a/b: long division producing NC+1 quotient digits, renormalised.
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
// Batcher's odd-even merge network for two runs of M terms (M a power of
// two), generated at compile time in the order of its recursive definition:
// merge the even and the odd subsequences, then compare neighbours.
// ---------------------------------------------------------------------------
template <int M>
struct MergeNet {
  int n;
  unsigned char a[32];
  unsigned char b[32];
};

template <int M>
constexpr void merge_rec(MergeNet<M> &net, int lo, int hi, int r) {
  const int step = 2 * r;
  if (step < hi - lo) {
    merge_rec<M>(net, lo, hi, step);
    merge_rec<M>(net, lo + r, hi, step);
    for (int i = lo + r; i < hi - r; i += step) {
      net.a[net.n] = (unsigned char)i;
      net.b[net.n] = (unsigned char)(i + r);
      ++net.n;
    }
  } else {
    net.a[net.n] = (unsigned char)lo;
    net.b[net.n] = (unsigned char)(lo + r);
    ++net.n;
  }
}

template <int M>
constexpr MergeNet<M> make_mergenet() {
  MergeNet<M> net{};
  net.n = 0;
  merge_rec<M>(net, 0, 2 * M - 1, 1);
  return net;
}

// merge x[0..M-1] and x[M..2M-1] by decreasing magnitude; a compare-exchange
// moves the larger magnitude to the lower index, equal magnitudes stay
template <int M>
OZX_HD void merge_desc(double (&x)[2 * M]) {
  constexpr MergeNet<M> net = make_mergenet<M>();
#pragma unroll
  for (int c = 0; c < net.n; ++c) {
    const double u = x[net.a[c]], v = x[net.b[c]];
    const bool sw = __builtin_fabs(v) > __builtin_fabs(u);
    x[net.a[c]] = sw ? v : u;
    x[net.b[c]] = sw ? u : v;
  }
}

// Renormalise K terms into NC components.
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
  // Top-down compression.  When the first S error terms are all non-zero
  // every step emits its sum, the error carries on, and the components are
  // those sums (plus the last error when fewer than NC steps exist); steps
  // past the NC-th emit nothing.  Only lanes that met a zero error take the
  // general form below, which gives the same result on the others.  This
  // shortcut is taken for the renormalisations of products and quotients
  // (K <= NC + 1), whose terms rarely meet a zero error; the merged sums of
  // an addition often do (an exact step of the sweep above leaves a zero),
  // so they go to the general form directly.
  constexpr int S = K - 1 < NC ? K - 1 : NC;
  bool zero = K > NC + 1;
  if (!zero) {
    double eps = x[0];
#pragma unroll
    for (int i = 1; i <= S; ++i) {
      double r, e;
      two_sum(eps, x[i], r, e);
      y[i - 1] = r;
      zero = zero || (e == 0.0);
      eps = e;
    }
#pragma unroll
    for (int q = S; q < NC; ++q) y[q] = q == S ? eps : 0.0;
  }
  if (!zero) return;
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
    // before step i at most i-1 components are out, so only y[0..i-1] can
    // receive this one (q < i is decided at compile time)
#pragma unroll
    for (int q = 0; q < NC; ++q)
      if (q < i && emit && j == q) y[q] = r;
    eps = live ? (e != 0.0 ? e : r) : eps;
    j += emit ? 1 : 0;
  }
#pragma unroll
  for (int q = 0; q < NC; ++q)
    if (j == q) y[q] = eps;
}

template <int NC>
OZX_HD void add(const double (&a)[NC], const double (&b)[NC], double (&r)[NC]) {
  constexpr int M = NC == 3 ? 4 : NC;
  double x[2 * M];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    x[i] = i < NC ? a[i < NC ? i : 0] : 0.0;
    x[M + i] = i < NC ? b[i < NC ? i : 0] : 0.0;
  }
  merge_desc<M>(x);
  renorm<2 * M, NC>(x, r);
}

template <int NC>
OZX_HD void mul(const double (&a)[NC], const double (&b)[NC], double (&r)[NC]) {
  double s[NC];
  double carry[16];
  int nc = 0;
#pragma unroll
  for (int o = 0; o < NC; ++o) {
    double t[24], nx[16];
    int nt = 0, nn = 0;
#pragma unroll
    for (int i = 0; i <= o; ++i) {
      if (o <= NC - 2) {
        double p, e;
        two_prod(a[i], b[o - i], p, e);
        t[nt++] = p;
        nx[nn++] = e;
      } else {
        t[nt++] = a[i] * b[o - i];
      }
    }
#pragma unroll
    for (int q = 0; q < nc; ++q) t[nt++] = carry[q];
    double sum = t[0];
#pragma unroll
    for (int q = 1; q < nt; ++q) {
      if (o <= NC - 2) {
        double c;
        two_sum(sum, t[q], sum, c);
        nx[nn++] = c;
      } else {
        sum = sum + t[q];
      }
    }
    s[o] = sum;
#pragma unroll
    for (int q = 0; q < nn; ++q) carry[q] = nx[q];
    nc = nn;
  }
  renorm<NC, NC>(s, r);
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

// r = b * q, q a double: by order as in mul
template <int NC>
OZX_HD void mul_d(const double (&b)[NC], double q, double (&r)[NC]) {
  double s[NC];
  double carry[NC];
  int nc = 0;
#pragma unroll
  for (int o = 0; o < NC; ++o) {
    double t[NC + 1], nx[NC];
    int nt = 0, nn = 0;
    if (o <= NC - 2) {
      double p, e;
      two_prod(b[o], q, p, e);
      t[nt++] = p;
      nx[nn++] = e;
    } else {
      t[nt++] = b[o] * q;
    }
#pragma unroll
    for (int k = 0; k < nc; ++k) t[nt++] = carry[k];
    double sum = t[0];
#pragma unroll
    for (int k = 1; k < nt; ++k) {
      if (o <= NC - 2) {
        double c;
        two_sum(sum, t[k], sum, c);
        nx[nn++] = c;
      } else {
        sum = sum + t[k];
      }
    }
    s[o] = sum;
#pragma unroll
    for (int k = 0; k < nn; ++k) carry[k] = nx[k];
    nc = nn;
  }
  renorm<NC, NC>(s, r);
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
