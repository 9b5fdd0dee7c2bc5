/*
 * CPU oracle, part 2: p-bit binary floating point and the LU on it.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  It shares no code with
 * the HIP library.
 *
 * Number format (the arbitrary-precision numbers of Sec. 2 and Sec. 4.3 of
 * Kouya, "Accelerating Multiple-Precision LU Decomposition with Ozaki Scheme
 * II", whose GPU type rounds like MPFR's RNDN): p = 64 nl bits,
 *     x = (-1)^s * m * 2^(e - p),   2^(p-1) <= m < 2^p,
 * m held in nl 64-bit limbs, least significant first; zero has m = 0,
 * e = LF_EXP_ZERO and s = 0.  Every operation returns the exact result
 * rounded once to p bits, to nearest with ties to even.
 *
 * Arrays are element-major: element k has limbs m[k nl .. k nl + nl - 1],
 * exponent e[k] (int64) and sign s[k] (uint8).
 *
 * Uses: the 2p-bit reference LU of the DD/TD/QD runs (the error of a p-bit
 * result measured against the same LU at twice the precision) and the
 * Lotkin experiment of Sec. 4.3 (correct bits of the solution of A x = A 1),
 * whose printed values pin this code.
 */
#include <limits.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;
#define LF_EXP_ZERO INT64_MIN
#define LF_MAXL 256 /* limbs of a mantissa: p <= 16384 */

/* ------------------------------------------------------------------ */
/* unsigned multi-limb helpers (little-endian 64-bit limbs)            */
/* ------------------------------------------------------------------ */
static int bitlen64(uint64_t x) { return x ? 64 - __builtin_clzll(x) : 0; }

/* bit length of x[0..xl) */
static int64_t mag_bits(const uint64_t *x, int xl) {
    for (int t = xl - 1; t >= 0; --t)
        if (x[t]) return 64 * (int64_t)t + bitlen64(x[t]);
    return 0;
}

static int bit_at(const uint64_t *x, int xl, int64_t k) {
    if (k < 0 || k >= 64 * (int64_t)xl) return 0;
    return (int)((x[k >> 6] >> (k & 63)) & 1u);
}

/* any bit below position k set */
static int any_below(const uint64_t *x, int xl, int64_t k) {
    if (k <= 0) return 0;
    int64_t full = k >> 6;
    if (full > xl) full = xl;
    for (int64_t i = 0; i < full; ++i)
        if (x[i]) return 1;
    if ((k & 63) && full < xl && (x[full] & ((1ull << (k & 63)) - 1))) return 1;
    return 0;
}

/* out[0..ol) = bits [sh, sh + 64 ol) of x (zero beyond x) */
static void shr_window(const uint64_t *x, int xl, int64_t sh, uint64_t *out, int ol) {
    for (int q = 0; q < ol; ++q) {
        int64_t b = sh + 64 * (int64_t)q;
        int64_t li = b >> 6;
        int r = (int)(b & 63);
        uint64_t lo = (li >= 0 && li < xl) ? x[li] : 0;
        uint64_t hi = (li + 1 >= 0 && li + 1 < xl) ? x[li + 1] : 0;
        out[q] = r ? ((lo >> r) | (hi << (64 - r))) : lo;
    }
}

/* x[0..xl) <<= sh (bits), into out[0..ol) (ol >= needed) */
static void shl_into(const uint64_t *x, int xl, int64_t sh, uint64_t *out, int ol) {
    memset(out, 0, sizeof(uint64_t) * ol);
    int64_t q = sh >> 6;
    int r = (int)(sh & 63);
    for (int i = 0; i < xl; ++i) {
        if (i + q < ol) out[i + q] |= x[i] << r;
        if (r && i + q + 1 < ol) out[i + q + 1] |= x[i] >> (64 - r);
    }
}

static int cmp_mag(const uint64_t *a, const uint64_t *b, int n) {
    for (int i = n - 1; i >= 0; --i) {
        if (a[i] != b[i]) return a[i] > b[i] ? 1 : -1;
    }
    return 0;
}

/* Round the non-zero magnitude x[0..xl) (plus an inexact tail below bit 0
 * when sticky_in) to p = 64 nl bits, ties to even.  Writes the mantissa and
 * returns the bit length of the rounded magnitude (the value is then
 * m 2^(T - p) in units of x's bit 0). */
static int64_t round_mag(const uint64_t *x, int xl, int sticky_in, int nl, uint64_t *m) {
    const int64_t p = 64 * (int64_t)nl;
    const int64_t T = mag_bits(x, xl);
    if (T <= p) {
        /* exact: the value has at most p bits (sticky_in never occurs here
         * for the callers, which keep at least one guard limb) */
        shl_into(x, xl, p - T, m, nl);
        return T;
    }
    const int64_t drop = T - p;
    shr_window(x, xl, drop, m, nl);
    const int rb = bit_at(x, xl, drop - 1);
    const int st = sticky_in || any_below(x, xl, drop - 1);
    if (rb && (st || (m[0] & 1u))) {
        /* m += 1 */
        int i = 0;
        for (; i < nl; ++i)
            if (++m[i] != 0) break;
        if (i == nl) { /* carried out of p bits: m = 2^(p-1) */
            memset(m, 0, sizeof(uint64_t) * nl);
            m[nl - 1] = 1ull << 63;
            return T + 1;
        }
    }
    return T;
}

static void set_zero(int nl, uint64_t *m, int64_t *e, uint8_t *s) {
    memset(m, 0, sizeof(uint64_t) * nl);
    *e = LF_EXP_ZERO;
    *s = 0;
}

static int is_zero(int nl, const uint64_t *m) {
    for (int i = 0; i < nl; ++i)
        if (m[i]) return 0;
    return 1;
}

/* ------------------------------------------------------------------ */
/* the operations                                                       */
/* ------------------------------------------------------------------ */
/* r = RN(a b) */
static void lf_mul(int nl, const uint64_t *am, int64_t ae, int as, const uint64_t *bm, int64_t be,
                   int bs, uint64_t *rm, int64_t *re, uint8_t *rs) {
    if (is_zero(nl, am) || is_zero(nl, bm)) {
        set_zero(nl, rm, re, rs);
        return;
    }
    uint64_t prod[2 * LF_MAXL];
    memset(prod, 0, sizeof(uint64_t) * 2 * nl);
    for (int i = 0; i < nl; ++i) {
        uint64_t carry = 0;
        for (int j = 0; j < nl; ++j) {
            u128 t = (u128)am[i] * bm[j] + prod[i + j] + carry;
            prod[i + j] = (uint64_t)t;
            carry = (uint64_t)(t >> 64);
        }
        prod[i + nl] = carry;
    }
    const int64_t p = 64 * (int64_t)nl;
    const int64_t T = round_mag(prod, 2 * nl, 0, nl, rm);
    *re = T + ae + be - 2 * p;
    *rs = (uint8_t)((as ^ bs) & 1);
}

/* r = RN(a + (-1)^negb b) */
static void lf_add(int nl, const uint64_t *am, int64_t ae, int as, const uint64_t *bm, int64_t be,
                   int bs, int negb, uint64_t *rm, int64_t *re, uint8_t *rs) {
    bs = (bs ^ negb) & 1;
    const int za = is_zero(nl, am), zb = is_zero(nl, bm);
    if (za && zb) {
        set_zero(nl, rm, re, rs);
        return;
    }
    if (zb || za) {
        const uint64_t *xm = zb ? am : bm;
        memcpy(rm, xm, sizeof(uint64_t) * nl);
        *re = zb ? ae : be;
        *rs = (uint8_t)(zb ? as : bs);
        return;
    }
    /* order: |X| >= |Y| */
    int swap = 0;
    if (ae < be) swap = 1;
    else if (ae == be && cmp_mag(am, bm, nl) < 0) swap = 1;
    const uint64_t *Xm = swap ? bm : am, *Ym = swap ? am : bm;
    const int64_t Xe = swap ? be : ae, Ye = swap ? ae : be;
    const int Xs = swap ? bs : as, Ys = swap ? as : bs;
    const int64_t d = Xe - Ye;
    enum { G = 3 };                   /* guard limbs below the mantissa */
    const int L = nl + G + 1;         /* one more for the carry */
    uint64_t X[LF_MAXL + G + 1], Y[LF_MAXL + G + 1];
    memset(X, 0, sizeof(uint64_t) * L);
    memcpy(X + G, Xm, sizeof(uint64_t) * nl);
    int sticky = 0;
    if (d <= 64 * G) {
        shl_into(Ym, nl, 64 * G - d, Y, L);   /* exact */
    } else {
        const int64_t sh = d - 64 * G;
        shr_window(Ym, nl, sh, Y, L);
        sticky = any_below(Ym, nl, sh);
    }
    uint64_t S[LF_MAXL + G + 1];
    if (Xs == Ys) {
        uint64_t c = 0;
        for (int i = 0; i < L; ++i) {
            u128 t = (u128)X[i] + Y[i] + c;
            S[i] = (uint64_t)t;
            c = (uint64_t)(t >> 64);
        }
    } else {
        /* X - Y, minus one more unit when Y lost bits: the exact value then
         * lies strictly between S and S + 1, which the sticky bit records */
        uint64_t br = (uint64_t)sticky;
        for (int i = 0; i < L; ++i) {
            u128 t = (u128)X[i] - Y[i] - br;
            S[i] = (uint64_t)t;
            br = (uint64_t)(t >> 127);
        }
    }
    if (mag_bits(S, L) == 0) {
        set_zero(nl, rm, re, rs);   /* exact cancellation: +0 */
        return;
    }
    const int64_t p = 64 * (int64_t)nl;
    const int64_t T = round_mag(S, L, sticky, nl, rm);
    *re = T + Xe - p - 64 * G;
    *rs = (uint8_t)Xs;
}

/* Knuth's division (TAOCP vol. 2, 4.3.1, Algorithm D) on 32-bit digits:
 * q[0..m-n] = floor(u / v), r[0..n) = u mod v, for u of m digits and v of n
 * >= 2 digits whose top digit has its most significant bit set. */
static void divide_d(const uint32_t *u, int m, const uint32_t *v, int n, uint32_t *q, uint32_t *r) {
    const uint64_t b = 1ull << 32;
    uint32_t un[4 * LF_MAXL + 8];
    memcpy(un, u, sizeof(uint32_t) * m);
    un[m] = 0;
    for (int j = m - n; j >= 0; --j) {
        const uint64_t num = ((uint64_t)un[j + n] << 32) | un[j + n - 1];
        uint64_t qhat = num / v[n - 1];
        uint64_t rhat = num - qhat * v[n - 1];
        while (qhat >= b || qhat * v[n - 2] > ((rhat << 32) | un[j + n - 2])) {
            qhat -= 1;
            rhat += v[n - 1];
            if (rhat >= b) break;
        }
        /* un[j .. j+n] -= qhat v */
        int64_t k = 0;
        int64_t t;
        for (int i = 0; i < n; ++i) {
            const uint64_t pr = qhat * v[i];
            t = (int64_t)un[i + j] - k - (int64_t)(pr & 0xffffffffu);
            un[i + j] = (uint32_t)t;
            k = (int64_t)(pr >> 32) - (t >> 32);
        }
        t = (int64_t)un[j + n] - k;
        un[j + n] = (uint32_t)t;
        if (t < 0) {
            /* qhat was one too large: add v back */
            qhat -= 1;
            uint64_t c = 0;
            for (int i = 0; i < n; ++i) {
                const uint64_t s = (uint64_t)un[i + j] + v[i] + c;
                un[i + j] = (uint32_t)s;
                c = s >> 32;
            }
            un[j + n] = (uint32_t)((uint64_t)un[j + n] + c);
        }
        q[j] = (uint32_t)qhat;
    }
    memcpy(r, un, sizeof(uint32_t) * n);
}

/* r = RN(a / b); b must be non-zero (a zero b gives zero and returns 1) */
static int lf_div(int nl, const uint64_t *am, int64_t ae, int as, const uint64_t *bm, int64_t be,
                  int bs, uint64_t *rm, int64_t *re, uint8_t *rs) {
    if (is_zero(nl, bm)) {
        set_zero(nl, rm, re, rs);
        return 1;
    }
    if (is_zero(nl, am)) {
        set_zero(nl, rm, re, rs);
        return 0;
    }
    const int64_t p = 64 * (int64_t)nl;
    /* N = ma 2^(p+1): 2p+1 bits; quotient floor(N / mb) in [2^p, 2^(p+2)) */
    const int NL = 2 * nl + 1;
    uint64_t N[2 * LF_MAXL + 1];
    shl_into(am, nl, p + 1, N, NL);
    uint32_t u[4 * LF_MAXL + 2], v[2 * LF_MAXL], q[4 * LF_MAXL + 2], rem[2 * LF_MAXL];
    for (int i = 0; i < NL; ++i) {
        u[2 * i] = (uint32_t)N[i];
        u[2 * i + 1] = (uint32_t)(N[i] >> 32);
    }
    for (int i = 0; i < nl; ++i) {
        v[2 * i] = (uint32_t)bm[i];
        v[2 * i + 1] = (uint32_t)(bm[i] >> 32);
    }
    const int m = 2 * NL, n = 2 * nl;
    divide_d(u, m, v, n, q, rem);
    int sticky = 0;
    for (int i = 0; i < n; ++i)
        if (rem[i]) sticky = 1;
    const int QL = (m - n + 1 + 1) / 2;
    uint64_t Q[2 * LF_MAXL + 2];
    for (int i = 0; i < QL; ++i) {
        const uint64_t lo = 2 * i < m - n + 1 ? q[2 * i] : 0;
        const uint64_t hi = 2 * i + 1 < m - n + 1 ? q[2 * i + 1] : 0;
        Q[i] = lo | (hi << 32);
    }
    const int64_t T = round_mag(Q, QL, sticky, nl, rm);
    *re = T + ae - be - p - 1;
    *rs = (uint8_t)((as ^ bs) & 1);
    return 0;
}

/* |a| > |b| exactly */
static int abs_greater(int nl, const uint64_t *am, int64_t ae, const uint64_t *bm, int64_t be) {
    const int za = is_zero(nl, am), zb = is_zero(nl, bm);
    if (za) return 0;
    if (zb) return 1;
    if (ae != be) return ae > be;
    return cmp_mag(am, bm, nl) > 0;
}

/* ------------------------------------------------------------------ */
/* exported elementwise operations (for the pins)                      */
/* ------------------------------------------------------------------ */
/* op 0: a + b, 1: a - b, 2: a b, 3: a / b */
void orc_lf_vec(int op, int nl, int64_t cnt, const uint64_t *am, const int64_t *ae,
                const uint8_t *as, const uint64_t *bm, const int64_t *be, const uint8_t *bs,
                uint64_t *rm, int64_t *re, uint8_t *rs) {
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < cnt; ++k) {
        const uint64_t *a = am + k * nl, *b = bm + k * nl;
        uint64_t *r = rm + k * nl;
        if (op == 0 || op == 1)
            lf_add(nl, a, ae[k], as[k], b, be[k], bs[k], op, r, re + k, rs + k);
        else if (op == 2)
            lf_mul(nl, a, ae[k], as[k], b, be[k], bs[k], r, re + k, rs + k);
        else
            lf_div(nl, a, ae[k], as[k], b, be[k], bs[k], r, re + k, rs + k);
    }
}

/* RN_p of the exact sum of nc binary64 components per element (an
 * expansion, or any doubles): the sum is formed exactly in a fixed-point
 * buffer covering the whole binary64 range, then rounded once. */
void orc_lf_from_doubles(int nl, int64_t cnt, int nc, const double *x, uint64_t *rm,
                         int64_t *re, uint8_t *rs) {
    enum { BL = 36 }; /* 2304 bits: binary64 values are 2^-1074 .. 2^1024 */
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < cnt; ++k) {
        uint64_t acc[BL + 1];
        memset(acc, 0, sizeof(acc));
        for (int c = 0; c < nc; ++c) {
            const double v = x[k * nc + c];
            if (v == 0.0) continue;
            uint64_t bits;
            memcpy(&bits, &v, 8);
            const int neg = (int)(bits >> 63);
            const int bexp = (int)((bits >> 52) & 0x7ff);
            uint64_t mant = bits & ((1ull << 52) - 1);
            int64_t sh; /* v = mant 2^sh, placed at bit sh + 1074 of acc */
            if (bexp == 0) sh = -1074;
            else {
                mant |= 1ull << 52;
                sh = bexp - 1075;
            }
            uint64_t part[BL + 1];
            shl_into(&mant, 1, sh + 1074, part, BL + 1);
            if (!neg) {
                uint64_t cy = 0;
                for (int i = 0; i <= BL; ++i) {
                    u128 t = (u128)acc[i] + part[i] + cy;
                    acc[i] = (uint64_t)t;
                    cy = (uint64_t)(t >> 64);
                }
            } else {
                uint64_t br = 0;
                for (int i = 0; i <= BL; ++i) {
                    u128 t = (u128)acc[i] - part[i] - br;
                    acc[i] = (uint64_t)t;
                    br = (uint64_t)(t >> 127);
                }
            }
        }
        int neg = (int)(acc[BL] >> 63);
        if (neg) { /* two's complement magnitude */
            uint64_t cy = 1;
            for (int i = 0; i <= BL; ++i) {
                u128 t = (u128)(~acc[i]) + cy;
                acc[i] = (uint64_t)t;
                cy = (uint64_t)(t >> 64);
            }
        }
        uint64_t *r = rm + k * nl;
        if (mag_bits(acc, BL + 1) == 0) {
            set_zero(nl, r, re + k, rs + k);
            continue;
        }
        const int64_t T = round_mag(acc, BL + 1, 0, nl, r);
        re[k] = T - 1074; /* value = m 2^(T - p) 2^-1074 = m 2^(e - p) */
        rs[k] = (uint8_t)neg;
    }
}

/* ------------------------------------------------------------------ */
/* LU with partial pivoting and the solve (Sec. 3.4, Sec. 4.3)          */
/* ------------------------------------------------------------------ */
/* Unblocked right-looking LU with partial pivoting of the m x nc block
 * (m >= nc; element (i, j) at index i + j ld, i.e. the caller passes the
 * block's first element): for each column j the pivot is the largest exact
 * magnitude among rows j..m-1, ties to the lowest row; rows j and the pivot
 * row are interchanged across the block's nc columns; l = RN(a / pivot);
 * then every a_ic (c > j) takes RN(a_ic - RN(l_ij a_jc)).  Per element the
 * updates come in ascending j.  ipiv[j] is the block-relative pivot row,
 * info the first j+1 with an exactly zero pivot (that column is then
 * skipped: no division, no update, as LAPACK's panel does). */
void orc_lf_getf2(int nl, int64_t m_rows, int64_t nc, uint64_t *m, int64_t *e, uint8_t *s,
                  int64_t ld, int64_t *ipiv, int32_t *info) {
    *info = 0;
#define EL(i, j) ((i) + (j) * ld)
    for (int64_t j = 0; j < nc; ++j) {
        int64_t p = j;
        for (int64_t i = j + 1; i < m_rows; ++i)
            if (abs_greater(nl, m + EL(i, j) * nl, e[EL(i, j)], m + EL(p, j) * nl, e[EL(p, j)])) p = i;
        ipiv[j] = p;
        if (p != j) {
            for (int64_t c = 0; c < nc; ++c) {
                uint64_t t[LF_MAXL];
                memcpy(t, m + EL(j, c) * nl, 8 * nl);
                memcpy(m + EL(j, c) * nl, m + EL(p, c) * nl, 8 * nl);
                memcpy(m + EL(p, c) * nl, t, 8 * nl);
                int64_t te = e[EL(j, c)];
                e[EL(j, c)] = e[EL(p, c)];
                e[EL(p, c)] = te;
                uint8_t ts = s[EL(j, c)];
                s[EL(j, c)] = s[EL(p, c)];
                s[EL(p, c)] = ts;
            }
        }
        if (is_zero(nl, m + EL(j, j) * nl)) {
            if (*info == 0) *info = (int32_t)(j + 1);
            continue;
        }
        const uint64_t *pm = m + EL(j, j) * nl;
        const int64_t pe = e[EL(j, j)];
        const int ps = s[EL(j, j)];
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t i = j + 1; i < m_rows; ++i) {
            uint64_t lm[LF_MAXL], tm[LF_MAXL];
            int64_t le, te;
            uint8_t ls, ts;
            lf_div(nl, m + EL(i, j) * nl, e[EL(i, j)], s[EL(i, j)], pm, pe, ps, lm, &le, &ls);
            memcpy(m + EL(i, j) * nl, lm, 8 * nl);
            e[EL(i, j)] = le;
            s[EL(i, j)] = ls;
            for (int64_t c = j + 1; c < nc; ++c) {
                lf_mul(nl, lm, le, ls, m + EL(j, c) * nl, e[EL(j, c)], s[EL(j, c)], tm, &te, &ts);
                uint64_t *am = m + EL(i, c) * nl;
                lf_add(nl, am, e[EL(i, c)], s[EL(i, c)], tm, te, ts, 1, am, e + EL(i, c),
                       s + EL(i, c));
            }
        }
    }
#undef EL
}

/* The LU of Sec. 3.4 on the whole n x n matrix, unblocked: the panel above
 * with nc = m = n, so every interchange spans whole rows. */
void orc_lf_getrf(int nl, int64_t n, uint64_t *m, int64_t *e, uint8_t *s, int64_t ld,
                  int64_t *ipiv, int32_t *info) {
    orc_lf_getf2(nl, n, n, m, e, s, ld, ipiv, info);
}

/* B <- L^-1 B for the unit lower triangle of the kb x kb block L (the U12
 * block row of the blocked LU): per column, for k ascending, every row
 * i > k takes RN(b_ik' - RN(l_ik b_kc)). */
void orc_lf_trsm_lunit(int nl, int64_t kb, int64_t ncols, const uint64_t *lm, const int64_t *le,
                       const uint8_t *ls, int64_t ldl, uint64_t *bm, int64_t *be, uint8_t *bs,
                       int64_t ldb) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < ncols; ++c) {
        uint64_t tm[LF_MAXL];
        int64_t te;
        uint8_t ts;
        for (int64_t k = 0; k < kb; ++k) {
            const int64_t u = k + c * ldb;
            for (int64_t i = k + 1; i < kb; ++i) {
                const int64_t a = i + k * ldl, x = i + c * ldb;
                lf_mul(nl, lm + a * nl, le[a], ls[a], bm + u * nl, be[u], bs[u], tm, &te, &ts);
                lf_add(nl, bm + x * nl, be[x], bs[x], tm, te, ts, 1, bm + x * nl, be + x, bs + x);
            }
        }
    }
}

/* C <- C - A B by multiply-subtracts: every c_ij takes RN(c_ij - RN(a_ik
 * b_kj)) for k ascending (the native update; with the panel and the solve
 * above it reproduces the unblocked LU element by element). */
void orc_lf_gemm_sub(int nl, int64_t M, int64_t N, int64_t K, const uint64_t *am,
                     const int64_t *ae, const uint8_t *as, int64_t lda, const uint64_t *bm,
                     const int64_t *be, const uint8_t *bs, int64_t ldb, uint64_t *cm, int64_t *ce,
                     uint8_t *cs, int64_t ldc) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < M * N; ++t) {
        const int64_t i = t % M, j = t / M;
        const int64_t x = i + j * ldc;
        uint64_t tm[LF_MAXL];
        int64_t te;
        uint8_t ts;
        for (int64_t k = 0; k < K; ++k) {
            const int64_t a = i + k * lda, b = k + j * ldb;
            lf_mul(nl, am + a * nl, ae[a], as[a], bm + b * nl, be[b], bs[b], tm, &te, &ts);
            lf_add(nl, cm + x * nl, ce[x], cs[x], tm, te, ts, 1, cm + x * nl, ce + x, cs + x);
        }
    }
}

/* Solve A X = B from the factors: interchanges in ipiv order, forward
 * substitution with unit L (x_i takes RN(x_i - RN(l_ik x_k)), k ascending),
 * backward substitution with U (k descending; x_k = RN(x_k / u_kk) once its
 * updates are in).  B is n x nrhs, element (i, r) at i + r ldb. */
void orc_lf_getrs(int nl, int64_t n, const uint64_t *m, const int64_t *e, const uint8_t *s,
                  int64_t ld, const int64_t *ipiv, int64_t nrhs, uint64_t *bm, int64_t *be,
                  uint8_t *bs, int64_t ldb) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrhs; ++r) {
        uint64_t *xm = bm + r * ldb * nl;
        int64_t *xe = be + r * ldb;
        uint8_t *xs = bs + r * ldb;
        uint64_t tm[LF_MAXL];
        int64_t te;
        uint8_t ts;
        for (int64_t j = 0; j < n; ++j) {
            const int64_t p = ipiv[j];
            if (p == j) continue;
            memcpy(tm, xm + j * nl, 8 * nl);
            memcpy(xm + j * nl, xm + p * nl, 8 * nl);
            memcpy(xm + p * nl, tm, 8 * nl);
            te = xe[j]; xe[j] = xe[p]; xe[p] = te;
            ts = xs[j]; xs[j] = xs[p]; xs[p] = ts;
        }
        for (int64_t k = 0; k < n; ++k)
            for (int64_t i = k + 1; i < n; ++i) {
                const int64_t a = i + k * ld;
                lf_mul(nl, m + a * nl, e[a], s[a], xm + k * nl, xe[k], xs[k], tm, &te, &ts);
                lf_add(nl, xm + i * nl, xe[i], xs[i], tm, te, ts, 1, xm + i * nl, xe + i, xs + i);
            }
        for (int64_t k = n - 1; k >= 0; --k) {
            const int64_t d = k + k * ld;
            lf_div(nl, xm + k * nl, xe[k], xs[k], m + d * nl, e[d], s[d], tm, &te, &ts);
            memcpy(xm + k * nl, tm, 8 * nl);
            xe[k] = te;
            xs[k] = ts;
            for (int64_t i = 0; i < k; ++i) {
                const int64_t a = i + k * ld;
                lf_mul(nl, m + a * nl, e[a], s[a], xm + k * nl, xe[k], xs[k], tm, &te, &ts);
                lf_add(nl, xm + i * nl, xe[i], xs[i], tm, te, ts, 1, xm + i * nl, xe + i, xs + i);
            }
        }
    }
}
