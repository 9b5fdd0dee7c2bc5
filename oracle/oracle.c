/*
 * CPU oracle for the Ozaki-scheme-II multiple-precision LU.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  It shares no code with
 * the HIP library (no headers, helpers, tables or generators).
 *
 * Build:  gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 *
 * What it computes, in the paper's order and notation (Kouya, "Accelerating
 * Multiple-Precision LU Decomposition with Ozaki Scheme II"):
 *   Sec. 3.1 (S1)-(S6): shared exponents, Q-bit fixed point, residues,
 *     exact modular products, CRT, one final rounding;
 *   Sec. 3.2: balanced w-bit slices, digit groups g = S-1..2S-2, Eq. (crt);
 *   Sec. 3.3, Eq. (direct): per-component conversion of an expansion;
 *   Sec. 3.4, Eq. (schur): blocked right-looking LU with partial pivoting,
 *     plus the blocked-naive and unblocked (b = 1) comparators.
 * The Ozaki-II product is evaluated from its plain definition -- the exact
 * digit-group sums of the slices, rounded once -- and, separately, through
 * the residue / modular-GEMM / CRT mirror so that each stage can be compared.
 *
 * Expansion arithmetic (the panel, the triangular solves, the native update)
 * follows one written specification: error-free TwoSum (Knuth) and TwoProd
 * (FMA); a two-pass renormalisation (bottom-up VecSum, then top-down
 * error-branch compression, after Joldes-Muller-Popescu); addition merges the
 * two operands by magnitude with Batcher's odd-even merge network before
 * renormalising; multiplication sums partial products by order (Hida, Li,
 * Bailey); division is long division.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <limits.h>

#define EXP_ZERO INT_MIN
#define MAXNC 4

/* ===================================================================== */
/* Error-free transforms                                                 */
/* ===================================================================== */
static inline void two_sum(double a, double b, double *s, double *e) {
    double ss = a + b;
    double bp = ss - a;
    double ap = ss - bp;
    *e = (a - ap) + (b - bp);
    *s = ss;
}
static inline void two_prod(double a, double b, double *p, double *e) {
    double pp = a * b;
    *e = fma(a, b, -pp);
    *p = pp;
}

/* Renormalise k terms into n components (x is clobbered). */
static void renorm(double *x, int k, int n, double *y) {
    double s = x[k - 1];
    for (int i = k - 2; i >= 0; --i) {
        double t;
        two_sum(x[i], s, &s, &t);
        x[i + 1] = t;
    }
    x[0] = s;
    for (int i = 0; i < n; ++i) y[i] = 0.0;
    int j = 0;
    double eps = x[0];
    for (int i = 1; i < k && j < n; ++i) {
        double r, e;
        two_sum(eps, x[i], &r, &e);
        if (e != 0.0) {
            y[j++] = r;
            eps = e;
        } else {
            eps = r;
        }
    }
    if (j < n) y[j] = eps;
}

/* compare-exchange: the larger magnitude moves to the lower index; equal
 * magnitudes stay where they are */
static inline void ce(double *x, int i, int j) {
    if (fabs(x[j]) > fabs(x[i])) {
        double t = x[i];
        x[i] = x[j];
        x[j] = t;
    }
}

/* Batcher's odd-even merge network (Knuth, TAOCP vol. 3, Sec. 5.3.4) on
 * x[lo..hi] with comparator stride r, in the order of its recursive
 * definition: merge the even and the odd subsequences, then compare
 * neighbours.  Called as oe_merge(x, 0, 2m-1, 1) it merges two runs of m (a
 * power of two) terms sorted by decreasing magnitude, x[0..m-1] and
 * x[m..2m-1].  A fixed comparator sequence: the outcome, ties included, is a
 * function of the input alone. */
static void oe_merge(double *x, int lo, int hi, int r) {
    int step = 2 * r;
    if (step < hi - lo) {
        oe_merge(x, lo, hi, step);
        oe_merge(x, lo + r, hi, step);
        for (int i = lo + r; i < hi - r; i += step) ce(x, i, i + r);
    } else {
        ce(x, lo, lo + r);
    }
}

/* r = a + b: the components of a and b (each a non-overlapping expansion,
 * largest first) merged by magnitude -- triple-double operands padded with a
 * zero to four -- then all 2m terms renormalised. */
void orc_add(int n, const double *a, const double *b, double *r) {
    double x[2 * MAXNC];
    int m = n == 3 ? 4 : n;
    for (int i = 0; i < m; ++i) {
        x[i] = i < n ? a[i] : 0.0;
        x[m + i] = i < n ? b[i] : 0.0;
    }
    oe_merge(x, 0, 2 * m - 1, 1);
    renorm(x, 2 * m, n, r);
}

/* r = a * b, partial products summed by order o = i + j (Hida, Li, Bailey's
 * quad-double product, for any n):
 *   orders o <= n-2: products by TwoProd, a_0 b_o first; their errors and
 *   the terms carried into this order are added to the running sum by
 *   TwoSum, each TwoSum error carried to order o+1 after the product errors;
 *   order n-1: the plain products and everything carried, summed left to
 *   right; orders >= n are dropped.
 * The n order sums are then renormalised. */
void orc_mul(int n, const double *a, const double *b, double *r) {
    double s[MAXNC], carry[32], next[32], t[40];
    int nc = 0;
    for (int o = 0; o < n; ++o) {
        int nt = 0, nn = 0;
        for (int i = 0; i <= o; ++i) {
            if (o <= n - 2) {
                double p, e;
                two_prod(a[i], b[o - i], &p, &e);
                t[nt++] = p;
                next[nn++] = e;
            } else {
                t[nt++] = a[i] * b[o - i];
            }
        }
        for (int q = 0; q < nc; ++q) t[nt++] = carry[q];
        double sum = t[0];
        for (int q = 1; q < nt; ++q) {
            if (o <= n - 2) {
                double c;
                two_sum(sum, t[q], &sum, &c);
                next[nn++] = c;
            } else {
                sum = sum + t[q];
            }
        }
        s[o] = sum;
        for (int q = 0; q < nn; ++q) carry[q] = next[q];
        nc = nn;
    }
    renorm(s, n, n, r);
}

/* r = c - a*b: the rounded product, negated, added to c */
void orc_fms(int n, const double *c, const double *a, const double *b, double *r) {
    double p[MAXNC];
    orc_mul(n, a, b, p);
    for (int i = 0; i < n; ++i) p[i] = -p[i];
    orc_add(n, c, p, r);
}

/* r = b * q for a double q, by order as in orc_mul: b_o q by TwoProd for
 * o <= n-2 plus the carried errors (TwoSum), plain at order n-1. */
static void mul_d(int n, const double *b, double q, double *r) {
    double s[MAXNC], carry[8], next[8], t[8];
    int nc = 0;
    for (int o = 0; o < n; ++o) {
        int nt = 0, nn = 0;
        if (o <= n - 2) {
            double p, e;
            two_prod(b[o], q, &p, &e);
            t[nt++] = p;
            next[nn++] = e;
        } else {
            t[nt++] = b[o] * q;
        }
        for (int k = 0; k < nc; ++k) t[nt++] = carry[k];
        double sum = t[0];
        for (int k = 1; k < nt; ++k) {
            if (o <= n - 2) {
                double c;
                two_sum(sum, t[k], &sum, &c);
                next[nn++] = c;
            } else {
                sum = sum + t[k];
            }
        }
        s[o] = sum;
        for (int k = 0; k < nn; ++k) carry[k] = next[k];
        nc = nn;
    }
    renorm(s, n, n, r);
}

/* r = a / b by long division: n+1 quotient digits q_k = rem_0 / b_0 with
 * rem <- rem - q_k b, then the digits renormalised. */
void orc_div(int n, const double *a, const double *b, double *r) {
    double q[MAXNC + 1], rem[MAXNC], t[MAXNC];
    for (int i = 0; i < n; ++i) rem[i] = a[i];
    for (int k = 0; k <= n; ++k) {
        q[k] = rem[0] / b[0];
        if (k < n) {
            mul_d(n, b, q[k], t);
            for (int i = 0; i < n; ++i) t[i] = -t[i];
            double nr[MAXNC];
            orc_add(n, rem, t, nr);
            for (int i = 0; i < n; ++i) rem[i] = nr[i];
        }
    }
    renorm(q, n + 1, n, r);
}

/* |a| > |b| in the pivot order: lexicographic on sign-normalised components */
static int abs_greater(int n, const double *a, const double *b) {
    double sa = a[0] < 0 ? -1.0 : 1.0, sb = b[0] < 0 ? -1.0 : 1.0;
    for (int c = 0; c < n; ++c) {
        double x = sa * a[c], y = sb * b[c];
        if (x > y) return 1;
        if (x < y) return 0;
    }
    return 0;
}
int orc_abs_greater(int n, const double *a, const double *b) { return abs_greater(n, a, b); }

static int is_zero(int n, const double *a) {
    for (int c = 0; c < n; ++c)
        if (a[c] != 0.0) return 0;
    return 1;
}

/* Vectorised wrappers used by the tests (op: 0 add, 1 mul, 2 fms, 3 div). */
void orc_exp_vec(int op, int n, int64_t count, const double *a, const double *b,
                 const double *c, double *r) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) {
        const double *ai = a + i * n, *bi = b + i * n;
        double *ri = r + i * n;
        if (op == 0) orc_add(n, ai, bi, ri);
        else if (op == 1) orc_mul(n, ai, bi, ri);
        else if (op == 2) orc_fms(n, c + i * n, ai, bi, ri);
        else orc_div(n, ai, bi, ri);
    }
}

/* ===================================================================== */
/* Fixed-width two's-complement big integers (little-endian 64-bit limbs) */
/* ===================================================================== */
typedef unsigned __int128 u128;

static inline int bi_neg_p(int nw, const uint64_t *x) { return (int)(x[nw - 1] >> 63); }
static void bi_zero(int nw, uint64_t *x) { memset(x, 0, sizeof(uint64_t) * nw); }
static int bi_is_zero(int nw, const uint64_t *x) {
    for (int i = 0; i < nw; ++i)
        if (x[i]) return 0;
    return 1;
}
static void bi_negate(int nw, uint64_t *x) {
    uint64_t carry = 1;
    for (int i = 0; i < nw; ++i) {
        uint64_t v = ~x[i] + carry;
        carry = (carry && v == 0) ? 1 : 0;
        x[i] = v;
    }
}
static void bi_add(int nw, uint64_t *r, const uint64_t *a, const uint64_t *b) {
    uint64_t carry = 0;
    for (int i = 0; i < nw; ++i) {
        u128 s = (u128)a[i] + b[i] + carry;
        r[i] = (uint64_t)s;
        carry = (uint64_t)(s >> 64);
    }
}
static void bi_sub(int nw, uint64_t *r, const uint64_t *a, const uint64_t *b) {
    uint64_t borrow = 0;
    for (int i = 0; i < nw; ++i) {
        u128 d = (u128)a[i] - b[i] - borrow;
        r[i] = (uint64_t)d;
        borrow = (uint64_t)(d >> 64) ? 1 : 0;
    }
}
/* sign-extend a (na limbs) into r (nw limbs) */
static void bi_extend(int nw, uint64_t *r, int na, const uint64_t *a) {
    uint64_t fill = bi_neg_p(na, a) ? ~(uint64_t)0 : 0;
    for (int i = 0; i < nw; ++i) r[i] = i < na ? a[i] : fill;
}
/* x += m * 2^shift (m unsigned), or x -= when neg */
static void bi_addsub_shifted(int nw, uint64_t *x, uint64_t m, int shift, int neg) {
    uint64_t t[64];
    bi_zero(nw, t);
    int q = shift / 64, s = shift % 64;
    if (q < nw) t[q] = m << s;
    if (s && q + 1 < nw) t[q + 1] = m >> (64 - s);
    if (neg) bi_sub(nw, x, x, t);
    else bi_add(nw, x, x, t);
}
static void bi_shl(int nw, uint64_t *x, int s) {
    if (s <= 0) return;
    int q = s / 64, r = s % 64;
    for (int i = nw - 1; i >= 0; --i) {
        uint64_t lo = (i - q >= 0) ? x[i - q] : 0;
        uint64_t lo2 = (i - q - 1 >= 0) ? x[i - q - 1] : 0;
        x[i] = r ? (lo << r) | (lo2 >> (64 - r)) : lo;
    }
}
/* arithmetic right shift (floor division by 2^s) */
static void bi_sar(int nw, uint64_t *x, int s) {
    if (s <= 0) return;
    uint64_t fill = bi_neg_p(nw, x) ? ~(uint64_t)0 : 0;
    int q = s / 64, r = s % 64;
    for (int i = 0; i < nw; ++i) {
        uint64_t hi = (i + q < nw) ? x[i + q] : fill;
        uint64_t hi2 = (i + q + 1 < nw) ? x[i + q + 1] : fill;
        x[i] = r ? (hi >> r) | (hi2 << (64 - r)) : hi;
    }
}
/* unsigned magnitude multiply: r[na+nb] = a[na] * b[nb] */
static void mag_mul(uint64_t *r, const uint64_t *a, int na, const uint64_t *b, int nb) {
    memset(r, 0, sizeof(uint64_t) * (na + nb));
    for (int i = 0; i < na; ++i) {
        uint64_t carry = 0;
        for (int j = 0; j < nb; ++j) {
            u128 t = (u128)a[i] * b[j] + r[i + j] + carry;
            r[i + j] = (uint64_t)t;
            carry = (uint64_t)(t >> 64);
        }
        r[i + nb] = carry;
    }
}
/* acc (nacc limbs) += a * b, a and b signed (n limbs each, two's complement) */
static void bi_mac(int nacc, uint64_t *acc, int n, const uint64_t *a, const uint64_t *b) {
    uint64_t ma[32], mb[32], p[64], pe[64];
    int sa = bi_neg_p(n, a), sb = bi_neg_p(n, b);
    memcpy(ma, a, 8 * n);
    memcpy(mb, b, 8 * n);
    if (sa) bi_negate(n, ma);
    if (sb) bi_negate(n, mb);
    mag_mul(p, ma, n, mb, n);
    for (int i = 0; i < nacc; ++i) pe[i] = i < 2 * n ? p[i] : 0;
    if (sa ^ sb) bi_sub(nacc, acc, acc, pe);
    else bi_add(nacc, acc, acc, pe);
}
/* x mod m in [0, m) for signed x */
static uint32_t bi_mod_small(int nw, const uint64_t *x, uint32_t m) {
    uint64_t mag[64];
    memcpy(mag, x, 8 * nw);
    int neg = bi_neg_p(nw, x);
    if (neg) bi_negate(nw, mag);
    u128 r = 0;
    for (int i = nw - 1; i >= 0; --i) r = ((r << 64) | mag[i]) % m;
    uint32_t rr = (uint32_t)r;
    if (neg && rr) rr = m - rr;
    return rr;
}
static int bi_bitlen_mag(int nw, const uint64_t *mag) {
    for (int i = nw - 1; i >= 0; --i)
        if (mag[i]) return 64 * i + 64 - __builtin_clzll(mag[i]);
    return 0;
}
static int bi_cmp_signed(int nw, const uint64_t *a, const uint64_t *b) {
    int na = bi_neg_p(nw, a), nb = bi_neg_p(nw, b);
    if (na != nb) return na ? -1 : 1;
    for (int i = nw - 1; i >= 0; --i) {
        if (a[i] != b[i]) return a[i] > b[i] ? 1 : -1;
    }
    return 0;
}

/* ===================================================================== */
/* (S1) shared exponents and (S2) fixed point, Eq. (direct)               */
/* ===================================================================== */
/* frexp exponent of the leading non-zero component; EXP_ZERO for zero */
int orc_exponent(int nc, const double *x) {
    for (int c = 0; c < nc; ++c) {
        if (x[c] != 0.0) {
            int e;
            frexp(x[c], &e);
            return e;
        }
    }
    return EXP_ZERO;
}

/* e[i] = max_h E(A[i,h]) (rowwise=1, A is rows x cols) or
 * e[j] = max_h E(A[h,j]) (rowwise=0) */
void orc_exponents(int nc, int64_t rows, int64_t cols, const double *A, int64_t ld,
                   int rowwise, int32_t *e) {
    int64_t nout = rowwise ? rows : cols;
    for (int64_t o = 0; o < nout; ++o) {
        int best = EXP_ZERO;
        int64_t len = rowwise ? cols : rows;
        for (int64_t h = 0; h < len; ++h) {
            int64_t i = rowwise ? o : h, j = rowwise ? h : o;
            int ex = orc_exponent(nc, A + (i + j * ld) * nc);
            if (ex > best) best = ex;
        }
        e[o] = best;
    }
}

/* X = sum_c sgn(x_c) floor(|x_c| 2^mu), two's complement in nw limbs */
static void to_fixed(int nc, const double *x, int mu, int nw, uint64_t *X) {
    bi_zero(nw, X);
    for (int c = 0; c < nc; ++c) {
        if (x[c] == 0.0) continue;
        int e;
        double f = frexp(fabs(x[c]), &e);
        uint64_t m = (uint64_t)ldexp(f, 53); /* exact 53-bit integer */
        int shift = e - 53 + mu;
        if (shift >= 0) {
            bi_addsub_shifted(nw, X, m, shift, x[c] < 0);
        } else {
            int rs = -shift;
            uint64_t t = rs >= 64 ? 0 : (m >> rs);
            if (t) bi_addsub_shifted(nw, X, t, 0, x[c] < 0);
        }
    }
}

/* balanced slicing: X = sum_t v_t 2^{wt}; v_t in [-2^{w-1}, 2^{w-1}) for
 * t < S-1, v_{S-1} the remaining top part.  v is S x nv limbs. */
static void slice(int nw, const uint64_t *Xin, int S, int w, int nv, uint64_t *v) {
    uint64_t X[64], t[64];
    memcpy(X, Xin, 8 * nw);
    for (int s = 0; s < S - 1; ++s) {
        memcpy(t, X, 8 * nw);
        /* low w bits as unsigned */
        for (int i = 0; i < nw; ++i) {
            int lo = 64 * i;
            if (lo >= w) t[i] = 0;
            else if (lo + 64 > w) t[i] &= (((uint64_t)1) << (w - lo)) - 1;
        }
        /* centre: if u >= 2^{w-1} then u -= 2^w */
        int bit = w - 1;
        if ((t[bit / 64] >> (bit % 64)) & 1) bi_addsub_shifted(nw, t, 1, w, 1);
        bi_extend(nv, v + s * nv, nw, t);
        bi_sub(nw, X, X, t);
        bi_sar(nw, X, w);
    }
    bi_extend(nv, v + (S - 1) * nv, nw, X);
}

/* ===================================================================== */
/* Plan constants for the CRT mirror                                     */
/* ===================================================================== */
typedef struct {
    int S, w, nmod, g0;
    const int32_t *moduli;
} oplan;

/* ===================================================================== */
/* Stage entry points (mirror of (S1)-(S5)), used for stage parity tests  */
/* ===================================================================== */
static int chunk_limbs(int w) { return (w + 2 + 63) / 64 + 1; }
static int fixed_limbs(int Q) { return (Q + 8 + 63) / 64 + 1; }

/* mu from an exponent: mu = Q - 1 - e; zero rows/columns get mu = 0 */
static int mu_of(int Q, int e) { return e == EXP_ZERO ? 0 : Q - 1 - e; }

/* Residue planes of one operand.
 * rowwise=1: operand A (rows x K), element (i,h); output planes
 *   out[((t*nmod + l)*rows + i)*K + h]  (K contiguous)
 * rowwise=0: operand B (K x cols), element (h,j); output planes
 *   out[((t*nmod + l)*cols + j)*K + h]  (K contiguous)
 * Residues are centred: r in [-floor(m/2), ceil(m/2)-1] (int8 range for the
 * moduli <= 256, about +-2^22 for the binary64 back-end's primes). */
void orc_residues(int nc, int64_t rows, int64_t cols, const double *A, int64_t ld,
                  int rowwise, const int32_t *exps, int S, int w, int nmod,
                  const int32_t *moduli, int32_t *out) {
    int Q = S * w;
    int nw = fixed_limbs(Q), nv = chunk_limbs(w);
    int64_t K = rowwise ? cols : rows, nout = rowwise ? rows : cols;
#pragma omp parallel for schedule(static)
    for (int64_t o = 0; o < nout; ++o) {
        uint64_t X[64], v[64 * 8];
        for (int64_t h = 0; h < K; ++h) {
            int64_t i = rowwise ? o : h, j = rowwise ? h : o;
            int mu = mu_of(Q, exps[o]);
            if (exps[o] == EXP_ZERO) bi_zero(nw, X);
            else to_fixed(nc, A + (i + j * ld) * nc, mu, nw, X);
            slice(nw, X, S, w, nv, v);
            for (int t = 0; t < S; ++t) {
                for (int l = 0; l < nmod; ++l) {
                    uint32_t m = (uint32_t)moduli[l];
                    uint32_t r = bi_mod_small(nv, v + t * nv, m);
                    int32_t c = (int32_t)r;
                    if (r >= (m + 1) / 2) c -= (int32_t)m;
                    out[((t * nmod + l) * nout + o) * K + h] = c;
                }
            }
        }
    }
}

/* Modular GEMM per (group, modulus) with the t_l epilogue of Eq. (crt):
 * C = sum over pairs (ta,tb) with ta+tb=g of A_ta * B_tb^T (exact int64),
 * t = ((C mod m) y) mod m.  Output tpl[((gi*nmod + l)*N + j)*M + i]
 * (column major per plane), gi = g - g0.  *cmax receives max |C| over all
 * products, so callers can check the accumulator bound of a back-end. */
void orc_modgemm(int64_t M, int64_t N, int64_t K, const int32_t *pa, const int32_t *pb,
                 int S, int nmod, const int32_t *moduli, const int32_t *y, int g0,
                 uint32_t *tpl, int64_t *cmax) {
    int ng = 2 * S - 1 - g0;
    int64_t big = 0;
#pragma omp parallel for collapse(2) schedule(static) reduction(max : big)
    for (int gi = 0; gi < ng; ++gi) {
        for (int l = 0; l < nmod; ++l) {
            int g = g0 + gi;
            int64_t m = moduli[l];
            for (int64_t j = 0; j < N; ++j) {
                for (int64_t i = 0; i < M; ++i) {
                    int64_t C = 0;
                    for (int ta = 0; ta < S; ++ta) {
                        int tb = g - ta;
                        if (tb < 0 || tb >= S) continue;
                        const int32_t *ar = pa + ((int64_t)(ta * nmod + l) * M + i) * K;
                        const int32_t *br = pb + ((int64_t)(tb * nmod + l) * N + j) * K;
                        for (int64_t h = 0; h < K; ++h) C += (int64_t)ar[h] * br[h];
                    }
                    int64_t ac = C < 0 ? -C : C;
                    if (ac > big) big = ac;
                    int64_t cm = C % m;
                    if (cm < 0) cm += m;
                    tpl[((int64_t)(gi * nmod + l) * N + j) * M + i] = (uint32_t)((cm * y[l]) % m);
                }
            }
        }
    }
    if (cmax) *cmax = big;
}

/* Balanced base-17 digits of the FP8 back-end (Eq. fp8digits):
 * d1 = round(r/17) (17 is odd, so r/17 is never halfway), d0 = r - 17 d1. */
void orc_fp8_digits(int64_t count, const int32_t *r, int32_t *d0, int32_t *d1) {
    for (int64_t i = 0; i < count; ++i) {
        int32_t v = r[i];
        int32_t q = v >= 0 ? (2 * v + 17) / 34 : -((-2 * v + 17) / 34);
        d1[i] = q;
        d0[i] = v - 17 * q;
    }
}

/* OCP FP8 E4M3 encoding (1 sign bit, 4 exponent bits with bias 7, 3 fraction
 * bits) of a small integer |d| <= 16, every one of which is exact in it. */
uint8_t orc_e4m3_int(int32_t d) {
    uint8_t sign = d < 0 ? 0x80 : 0;
    uint32_t a = (uint32_t)(d < 0 ? -d : d);
    if (a == 0) return sign;
    int e = 31 - __builtin_clz(a);             /* a = 2^e (1 + f/8) */
    uint32_t f = ((a << 3) >> e) & 7u;         /* exact for a <= 16 */
    return (uint8_t)(sign | ((uint32_t)(e + 7) << 3) | f);
}

/* CRT by the CPU encoding (Sec. 3.5.1): X = (sum_l t_l M_l) mod P in [0,P),
 * then X -= P when X > floor(P/2).  Output nw-limb two's complement per
 * element: out[((gi*N + j)*M + i)*nw + k]. */
void orc_crt(int64_t M, int64_t N, const uint32_t *tpl, int ngroups, int nmod,
             const int32_t *moduli, int nw, uint64_t *out) {
    /* P and M_l as big integers */
    uint64_t P[64], halfP[64], Ml[64][64];
    bi_zero(nw, P);
    P[0] = 1;
    for (int l = 0; l < nmod; ++l) {
        uint64_t tmp[128], m1 = (uint64_t)moduli[l];
        mag_mul(tmp, P, nw, &m1, 1);
        memcpy(P, tmp, 8 * nw);
    }
    memcpy(halfP, P, 8 * nw);
    bi_sar(nw, halfP, 1);
    for (int l = 0; l < nmod; ++l) {
        bi_zero(nw, Ml[l]);
        Ml[l][0] = 1;
        for (int k = 0; k < nmod; ++k) {
            if (k == l) continue;
            uint64_t tmp[128], m1 = (uint64_t)moduli[k];
            mag_mul(tmp, Ml[l], nw, &m1, 1);
            memcpy(Ml[l], tmp, 8 * nw);
        }
    }
#pragma omp parallel for collapse(2) schedule(static)
    for (int gi = 0; gi < ngroups; ++gi) {
        for (int64_t j = 0; j < N; ++j) {
            for (int64_t i = 0; i < M; ++i) {
                uint64_t X[64];
                bi_zero(nw, X);
                for (int l = 0; l < nmod; ++l) {
                    uint64_t t = tpl[((int64_t)(gi * nmod + l) * N + j) * M + i];
                    uint64_t tmp[128];
                    mag_mul(tmp, Ml[l], nw, &t, 1);
                    bi_add(nw, X, X, tmp);
                }
                while (bi_cmp_signed(nw, X, P) >= 0) bi_sub(nw, X, X, P);
                if (bi_cmp_signed(nw, X, halfP) > 0) bi_sub(nw, X, X, P);
                memcpy(out + (((int64_t)gi * N + j) * M + i) * nw, X, 8 * nw);
            }
        }
    }
}

/* ===================================================================== */
/* (S6): greedy round-to-nearest expansion of C * 2^eps                   */
/* ===================================================================== */
/* x_0 = RN(v), x_c = RN(v - x_0 - ... - x_{c-1}); a component below
 * 2^-1022 in magnitude is flushed to zero and ends the expansion. */
static void round_out(int nw, const uint64_t *Cin, int eps, int nc, double *x) {
    uint64_t C[64], mag[64];
    memcpy(C, Cin, 8 * nw);
    for (int c = 0; c < nc; ++c) x[c] = 0.0;
    for (int c = 0; c < nc; ++c) {
        if (bi_is_zero(nw, C)) break;
        int neg = bi_neg_p(nw, C);
        memcpy(mag, C, 8 * nw);
        if (neg) bi_negate(nw, mag);
        int L = bi_bitlen_mag(nw, mag);
        uint64_t m;
        int ex = 0;
        if (L <= 53) {
            m = mag[0];
        } else {
            int sh = L - 53;
            uint64_t tmp[64];
            memcpy(tmp, mag, 8 * nw);
            bi_sar(nw, tmp, sh);
            m = tmp[0];
            /* round bit and sticky */
            int rb = (int)((mag[(sh - 1) / 64] >> ((sh - 1) % 64)) & 1);
            int sticky = 0, nb = sh - 1; /* bits 0 .. nb-1 */
            for (int q = 0; q < nb / 64 && !sticky; ++q)
                if (mag[q]) sticky = 1;
            if (!sticky && (nb % 64) &&
                (mag[nb / 64] & ((((uint64_t)1) << (nb % 64)) - 1)))
                sticky = 1;
            if (rb && (sticky || (m & 1))) m += 1;
            ex = sh;
        }
        int top = (63 - __builtin_clzll(m)) + ex + eps; /* floor(log2 |value|) */
        if (top < -1022) break;
        x[c] = neg ? -ldexp((double)m, ex + eps) : ldexp((double)m, ex + eps);
        /* C -= sign * m * 2^ex */
        uint64_t t[64];
        bi_zero(nw, t);
        t[0] = m;
        bi_shl(nw, t, ex);
        if (neg) bi_add(nw, C, C, t);
        else bi_sub(nw, C, C, t);
    }
}

/* Export of round_out for tests: C given as nw limbs, scale 2^eps */
void orc_round_out(int nw, const uint64_t *C, int eps, int nc, double *x) {
    round_out(nw, C, eps, nc, x);
}

/* ===================================================================== */
/* The Ozaki-II product from its definition                              */
/* ===================================================================== */
/* C = A*B (mode 0) or C = C - A*B (mode 1); A is M x K, B is K x N, all
 * column-major expansion matrices with nc components.  The exact digit-group
 * sums S_g = sum_{ta+tb=g} sum_h v_ta(i,h) u_tb(h,j) for g = g0..2S-2 are
 * accumulated as cbar = sum_g S_g 2^{w(g-g0)} and rounded once to
 * cbar * 2^{w g0 - mu_i - nu_j}.  If sbar_out is non-null, the group sums
 * are also written there (nw_out limbs per element, layout of orc_crt). */
void orc_ozgemm(int mode, int nc, int64_t M, int64_t N, int64_t K,
                const double *A, int64_t lda, const double *B, int64_t ldb,
                double *C, int64_t ldc, int S, int w, int g0,
                int nw_out, uint64_t *sbar_out) {
    int Q = S * w;
    int nw = fixed_limbs(Q), nv = chunk_limbs(w);
    int nacc = (2 * w + w * (2 * S - 2 - g0) + 64 + 63) / 64 + 2;
    if (nacc > 60) nacc = 60;
    int32_t *ea = (int32_t *)malloc(sizeof(int32_t) * (M > 0 ? M : 1));
    int32_t *eb = (int32_t *)malloc(sizeof(int32_t) * (N > 0 ? N : 1));
    orc_exponents(nc, M, K, A, lda, 1, ea);
    orc_exponents(nc, K, N, B, ldb, 0, eb);
    uint64_t *va = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(M * K * S * nv + 1));
    uint64_t *vb = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(N * K * S * nv + 1));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i) {
        uint64_t X[64];
        for (int64_t h = 0; h < K; ++h) {
            if (ea[i] == EXP_ZERO) bi_zero(nw, X);
            else to_fixed(nc, A + (i + h * lda) * nc, mu_of(Q, ea[i]), nw, X);
            slice(nw, X, S, w, nv, va + (i * K + h) * S * nv);
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j) {
        uint64_t X[64];
        for (int64_t h = 0; h < K; ++h) {
            if (eb[j] == EXP_ZERO) bi_zero(nw, X);
            else to_fixed(nc, B + (h + j * ldb) * nc, mu_of(Q, eb[j]), nw, X);
            slice(nw, X, S, w, nv, vb + (j * K + h) * S * nv);
        }
    }
    int ng = 2 * S - 1 - g0;
#pragma omp parallel for collapse(2) schedule(dynamic, 16)
    for (int64_t j = 0; j < N; ++j) {
        for (int64_t i = 0; i < M; ++i) {
            uint64_t cbar[64], sg[64];
            bi_zero(nacc, cbar);
            for (int gi = ng - 1; gi >= 0; --gi) {
                int g = g0 + gi;
                bi_zero(nacc, sg);
                for (int ta = 0; ta < S; ++ta) {
                    int tb = g - ta;
                    if (tb < 0 || tb >= S) continue;
                    for (int64_t h = 0; h < K; ++h)
                        bi_mac(nacc, sg, nv, va + ((i * K + h) * S + ta) * nv,
                               vb + ((j * K + h) * S + tb) * nv);
                }
                if (sbar_out) {
                    uint64_t *dst = sbar_out + (((int64_t)gi * N + j) * M + i) * nw_out;
                    bi_extend(nw_out, dst, nacc, sg);
                }
                /* Horner in 2^w: cbar = cbar * 2^w + S_g, top group first */
                if (gi != ng - 1) bi_shl(nacc, cbar, w);
                bi_add(nacc, cbar, cbar, sg);
            }
            double c[MAXNC];
            if (ea[i] == EXP_ZERO || eb[j] == EXP_ZERO) {
                for (int q = 0; q < nc; ++q) c[q] = 0.0;
            } else {
                int eps = w * g0 - mu_of(Q, ea[i]) - mu_of(Q, eb[j]);
                round_out(nacc, cbar, eps, nc, c);
            }
            double *dst = C + (i + j * ldc) * nc;
            if (mode == 0) {
                for (int q = 0; q < nc; ++q) dst[q] = c[q];
            } else {
                double nc_[MAXNC], r[MAXNC];
                for (int q = 0; q < nc; ++q) nc_[q] = -c[q];
                orc_add(nc, dst, nc_, r);
                for (int q = 0; q < nc; ++q) dst[q] = r[q];
            }
        }
    }
    free(ea);
    free(eb);
    free(va);
    free(vb);
}

/* Native product: C = C - A*B (mode 1) or C = 0 - A*B... (mode 0 starts from
 * zero and adds), sequential fms in ascending h for every element. */
void orc_naive_gemm(int mode, int nc, int64_t M, int64_t N, int64_t K,
                    const double *A, int64_t lda, const double *B, int64_t ldb,
                    double *C, int64_t ldc) {
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t j = 0; j < N; ++j) {
        for (int64_t i = 0; i < M; ++i) {
            double acc[MAXNC], r[MAXNC];
            double *dst = C + (i + j * ldc) * nc;
            for (int q = 0; q < nc; ++q) acc[q] = mode == 0 ? 0.0 : dst[q];
            for (int64_t h = 0; h < K; ++h) {
                if (mode == 0) {
                    /* acc = acc + a*b  ==  acc - (-a)*b */
                    double na[MAXNC];
                    for (int q = 0; q < nc; ++q) na[q] = -A[(i + h * lda) * nc + q];
                    orc_fms(nc, acc, na, B + (h + j * ldb) * nc, r);
                } else {
                    orc_fms(nc, acc, A + (i + h * lda) * nc, B + (h + j * ldb) * nc, r);
                }
                for (int q = 0; q < nc; ++q) acc[q] = r[q];
            }
            for (int q = 0; q < nc; ++q) dst[q] = acc[q];
        }
    }
}

/* ===================================================================== */
/* Blocked right-looking LU with partial pivoting, Eq. (schur)            */
/* ===================================================================== */
static void swap_rows(int nc, double *A, int64_t ld, int64_t r1, int64_t r2, int64_t c0, int64_t c1) {
    if (r1 == r2) return;
    for (int64_t c = c0; c < c1; ++c) {
        double *x = A + (r1 + c * ld) * nc, *y = A + (r2 + c * ld) * nc;
        for (int q = 0; q < nc; ++q) {
            double t = x[q];
            x[q] = y[q];
            y[q] = t;
        }
    }
}

/* method: 0 = Ozaki-II Schur update (S, w, g0 from the plan for K = b),
 *         1 = blocked naive (same panel, naive update).
 * Unblocked LU is method 1 with b = 1.  ipiv is 0-based (LAPACK semantics:
 * row j was interchanged with row ipiv[j]).  info = first j+1 with an exactly
 * zero pivot, else 0.  timing[0..1] receives panel+trsm seconds and update
 * seconds when non-null. */
#include <time.h>
static double now_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return ts.tv_sec + 1e-9 * ts.tv_nsec;
}
void orc_getrf(int nc, int64_t n, double *A, int64_t ld, int64_t b, int method,
               int S, int w, int g0, int64_t *ipiv, int32_t *info, double *timing) {
    *info = 0;
    double t_panel = 0, t_upd = 0;
    for (int64_t k = 0; k < n; k += b) {
        double t0 = now_s();
        int64_t kb = (n - k < b) ? n - k : b;
        /* (P1) panel */
        for (int64_t j = k; j < k + kb; ++j) {
            int64_t p = j;
            for (int64_t i = j + 1; i < n; ++i)
                if (abs_greater(nc, A + (i + j * ld) * nc, A + (p + j * ld) * nc)) p = i;
            ipiv[j] = p;
            if (is_zero(nc, A + (p + j * ld) * nc)) {
                if (*info == 0) *info = (int32_t)(j + 1);
                continue;
            }
            swap_rows(nc, A, ld, j, p, k, k + kb);
            const double *piv = A + (j + j * ld) * nc;
#pragma omp parallel for schedule(static)
            for (int64_t i = j + 1; i < n; ++i) {
                double *l = A + (i + j * ld) * nc;
                double r[MAXNC];
                orc_div(nc, l, piv, r);
                for (int q = 0; q < nc; ++q) l[q] = r[q];
                for (int64_t c = j + 1; c < k + kb; ++c) {
                    double *a = A + (i + c * ld) * nc;
                    orc_fms(nc, a, l, A + (j + c * ld) * nc, r);
                    for (int q = 0; q < nc; ++q) a[q] = r[q];
                }
            }
        }
        /* (P2) laswp on the columns left and right of the panel */
        for (int64_t j = k; j < k + kb; ++j) {
            swap_rows(nc, A, ld, j, ipiv[j], 0, k);
            swap_rows(nc, A, ld, j, ipiv[j], k + kb, n);
        }
        /* (P3) U12 = L11^{-1} A12, ascending k per element */
        if (k + kb < n) {
#pragma omp parallel for schedule(static)
            for (int64_t c = k + kb; c < n; ++c) {
                for (int64_t i = k; i < k + kb; ++i) {
                    double *a = A + (i + c * ld) * nc, r[MAXNC];
                    for (int64_t h = k; h < i; ++h) {
                        orc_fms(nc, a, A + (i + h * ld) * nc, A + (h + c * ld) * nc, r);
                        for (int q = 0; q < nc; ++q) a[q] = r[q];
                    }
                }
            }
        }
        double t1 = now_s();
        t_panel += t1 - t0;
        /* (P4) A22 -= L21 U12 */
        if (k + kb < n) {
            int64_t m2 = n - k - kb;
            const double *L21 = A + ((k + kb) + k * ld) * nc;
            const double *U12 = A + (k + (k + kb) * ld) * nc;
            double *A22 = A + ((k + kb) + (k + kb) * ld) * nc;
            if (method == 0)
                orc_ozgemm(1, nc, m2, m2, kb, L21, ld, U12, ld, A22, ld, S, w, g0, 0, NULL);
            else
                orc_naive_gemm(1, nc, m2, m2, kb, L21, ld, U12, ld, A22, ld);
        }
        t_upd += now_s() - t1;
    }
    if (timing) {
        timing[0] = t_panel;
        timing[1] = t_upd;
    }
}

/* Solve A X = B from the factors (Sec. 4.3: forward and backward
 * substitution): row interchanges in ipiv order; forward substitution with
 * unit L, element i updated for k ascending; backward substitution with U,
 * element i updated for k descending, and x_k divided by u_kk (the expansion
 * division of the specification) once all its updates are in.  B is
 * n x nrhs column-major. */
void orc_getrs(int nc, int64_t n, const double *LU, int64_t ld, const int64_t *ipiv,
               int64_t nrhs, double *B, int64_t ldb) {
    for (int64_t j = 0; j < n; ++j) swap_rows(nc, B, ldb, j, ipiv[j], 0, nrhs);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrhs; ++r) {
        double *x = B + r * ldb * nc, t[MAXNC];
        for (int64_t k = 0; k < n; ++k)
            for (int64_t i = k + 1; i < n; ++i) {
                orc_fms(nc, x + i * nc, LU + (i + k * ld) * nc, x + k * nc, t);
                for (int q = 0; q < nc; ++q) x[i * nc + q] = t[q];
            }
        for (int64_t k = n - 1; k >= 0; --k) {
            orc_div(nc, x + k * nc, LU + (k + k * ld) * nc, t);
            for (int q = 0; q < nc; ++q) x[k * nc + q] = t[q];
            for (int64_t i = 0; i < k; ++i) {
                orc_fms(nc, x + i * nc, LU + (i + k * ld) * nc, x + k * nc, t);
                for (int q = 0; q < nc; ++q) x[i * nc + q] = t[q];
            }
        }
    }
}
