// Lane-distributed p-bit binary floating point on one 64-lane wavefront.
//
// The LU on limb numbers keeps its panel, interchanges, U12 solve and
// substitutions outside the Ozaki-II product (Sec. 3.4); those steps need
// p-bit division, multiplication and subtraction of the number type of
// Sec. 2, which rounds like MPFR's RNDN.  One wavefront carries one number,
// p = 64 nl <= 4096:
//   x = (-1)^s m 2^(e - p),  2^(p-1) <= m < 2^p;   zero: m = 0, e = EXP_ZERO,
// lane q holding limb q of m (lanes nl..63 hold 0), e and s uniform.  Every
// operation returns the exact result rounded once to p bits, to nearest with
// ties to even; correct rounding makes that result unique.
//
// Carries and borrows between limbs are resolved for all lanes at once:
// lane k generates (g) or propagates (p) a carry, and the carry into every
// lane is read off the 64-bit sum (g|p) + g + cin, whose bit k is
// g_k ^ p_k ^ carry_k.  Products form each output column in its own lane
// (columns 64..127 in a second register) and resolve the column sums the
// same way; division is schoolbook long division on 64-bit digits (each
// digit from the remainder's top two digits over the divisor's top digit by
// Moller and Granlund's two-by-one division, at most two add-backs, Knuth's
// Theorem 4.3.1B).
//
// The includer provides LFP_FN and the cross-lane primitives lane_id,
// ballot, readlane64 (wave-uniform lane), shfl64 (any lane), up1_64 (from
// lane l-1, 0 into lane 0), rot1_64 (from lane (l-1) mod 64) and addc32
// (32-bit add with carry).
// Every function must be called by all 64 lanes of a converged wavefront;
// branches below depend on wave-uniform values only.
#pragma once
#include <stdint.h>

namespace lfp {

constexpr int32_t EXP_ZERO = INT32_MIN;

struct WF {
  uint64_t m;  // limb lane_id() of the mantissa
  int32_t e;   // exponent; EXP_ZERO for zero
  uint32_t s;  // sign: 0 positive, 1 negative
};

// a 128-limb fixed-point window: limb k in lane k of lo, limb 64+k in hi
struct W2 {
  uint64_t lo, hi;
};

LFP_FN WF wf_zero() {
  WF z;
  z.m = 0;
  z.e = EXP_ZERO;
  z.s = 0;
  return z;
}

LFP_FN bool is_zero(const WF &x) { return x.e == EXP_ZERO; }
LFP_FN int msb64(uint64_t x) { return 63 - __builtin_clzll(x); }
LFP_FN uint64_t low_mask(int k) { return k >= 64 ? ~0ull : ((1ull << k) - 1ull); }  // k >= 0
LFP_FN uint64_t bit_of(uint64_t mask, int l) { return (mask >> l) & 1ull; }

// Carry into every lane of a 64-lane chain (bit k of the result) for
// generate mask g, propagate mask p (disjoint) and carry-in cin of lane 0;
// cout = carry out of lane 63.
LFP_FN uint64_t chain(uint64_t g, uint64_t p, uint32_t cin, uint32_t &cout) {
  const uint64_t x = g | p;
  const uint64_t s1 = x + g;
  const uint64_t s2 = s1 + cin;
  cout = (uint32_t)((s1 < x) | (s2 < s1));
  return s2 ^ x ^ g;
}

// carry out of lane nl-1 of a chain whose lanes nl..63 kill
LFP_FN uint32_t out_at(uint64_t cmask, uint32_t cout63, int nl) {
  return nl >= 64 ? cout63 : (uint32_t)bit_of(cmask, nl);
}

// x + y + cin over lanes < nl (0 above); cout = carry out of lane nl-1
LFP_FN uint64_t add1(uint64_t x, uint64_t y, int nl, uint32_t cin, uint32_t &cout) {
  const int l = lane_id();
  const bool act = l < nl;
  const uint64_t s = x + y;
  uint32_t c63;
  const uint64_t cm = chain(ballot(act && s < x), ballot(act && s == ~0ull), cin, c63);
  cout = out_at(cm, c63, nl);
  return act ? s + bit_of(cm, l) : 0ull;
}

// x - y - bin over lanes < nl (0 above); bout = borrow out of lane nl-1
LFP_FN uint64_t sub1(uint64_t x, uint64_t y, int nl, uint32_t bin, uint32_t &bout) {
  const int l = lane_id();
  const bool act = l < nl;
  uint32_t b63;
  const uint64_t bm = chain(ballot(act && x < y), ballot(act && x == y), bin, b63);
  bout = out_at(bm, b63, nl);
  return act ? x - y - bit_of(bm, l) : 0ull;
}

LFP_FN W2 add2(W2 x, W2 y, uint32_t cin, uint32_t &cout) {
  const int l = lane_id();
  const uint64_t sl = x.lo + y.lo, sh = x.hi + y.hi;
  uint32_t c;
  const uint64_t cl = chain(ballot(sl < x.lo), ballot(sl == ~0ull), cin, c);
  const uint64_t ch = chain(ballot(sh < x.hi), ballot(sh == ~0ull), c, cout);
  W2 r;
  r.lo = sl + bit_of(cl, l);
  r.hi = sh + bit_of(ch, l);
  return r;
}

LFP_FN W2 sub2(W2 x, W2 y, uint32_t bin, uint32_t &bout) {
  const int l = lane_id();
  uint32_t b;
  const uint64_t bl = chain(ballot(x.lo < y.lo), ballot(x.lo == y.lo), bin, b);
  const uint64_t bh = chain(ballot(x.hi < y.hi), ballot(x.hi == y.hi), b, bout);
  W2 r;
  r.lo = x.lo - y.lo - bit_of(bl, l);
  r.hi = x.hi - y.hi - bit_of(bh, l);
  return r;
}

// limb j (per lane, any value) of the number held one limb per lane in v;
// 0 outside [0, 64)
LFP_FN uint64_t reg_limb(uint64_t v, int j) {
  const uint64_t t = shfl64(v, j & 63);
  return (j >= 0 && j < 64) ? t : 0ull;
}

// bits [base, base + 64) of the number in v; base & 63 must be wave-uniform
LFP_FN uint64_t reg_bits(uint64_t v, int64_t base) {
  const int li = (int)(base >> 6);
  const int r = (int)(base & 63);
  const uint64_t x0 = reg_limb(v, li), x1 = reg_limb(v, li + 1);
  return r ? ((x0 >> r) | (x1 << (64 - r))) : x0;
}

LFP_FN uint64_t win_limb(W2 w, int j) {
  const uint64_t a = shfl64(w.lo, j & 63), b = shfl64(w.hi, j & 63);
  return (j >= 0 && j < 64) ? a : ((j >= 64 && j < 128) ? b : 0ull);
}

// bits [base, base + 64) of the window; base & 63 wave-uniform
LFP_FN uint64_t win_bits(W2 w, int64_t base) {
  const int li = (int)(base >> 6);
  const int r = (int)(base & 63);
  const uint64_t x0 = win_limb(w, li), x1 = win_limb(w, li + 1);
  return r ? ((x0 >> r) | (x1 << (64 - r))) : x0;
}

// m + 1 over lanes < nl; ovf = 1 when it carried out of p bits, m is then
// 2^(p-1) (the caller adds one to the exponent)
LFP_FN uint64_t inc_mant(uint64_t m, int nl, uint32_t &ovf) {
  const int l = lane_id();
  const bool act = l < nl;
  uint32_t c63;
  const uint64_t cm = chain(0ull, ballot(act && m == ~0ull), 1u, c63);
  ovf = out_at(cm, c63, nl);
  uint64_t r = act ? m + bit_of(cm, l) : 0ull;
  if (ovf) r = (l == nl - 1) ? (1ull << 63) : 0ull;
  return r;
}

// RN_p of the non-zero window value w plus, when sticky, an inexact
// remainder below w's bit 0 (which must then lie below the rounding
// position).  Returns this lane's mantissa limb; bl = bit length of the
// rounded value in w's units (value = mantissa 2^(bl - p)).
LFP_FN uint64_t round_win(W2 w, uint32_t sticky, int nl, int64_t &bl) {
  const int l = lane_id();
  const uint64_t nzl = ballot(w.lo != 0), nzh = ballot(w.hi != 0);
  const int top = nzh ? 64 + msb64(nzh) : msb64(nzl);
  const uint64_t twh = readlane64(w.hi, nzh ? top - 64 : 0);
  const uint64_t twl = readlane64(w.lo, nzh ? 0 : top);
  const int64_t T = 64 * (int64_t)top + 64 - __builtin_clzll(nzh ? twh : twl);
  const int64_t D = T - 64 * (int64_t)nl;  // lowest kept bit
  const uint64_t mw = win_bits(w, D + 64 * (int64_t)l);
  uint64_t m = l < nl ? mw : 0ull;
  uint32_t rb = 0, st = sticky;
  if (D >= 1) {
    const int64_t rp = D - 1;
    const int rl = (int)(rp >> 6), rr = (int)(rp & 63);
    const uint64_t a = readlane64(w.lo, rl & 63), b = readlane64(w.hi, rl & 63);
    const uint64_t rlimb = rl < 64 ? a : b;
    rb = (uint32_t)((rlimb >> rr) & 1ull);
    const uint64_t ml = rl >= 64 ? ~0ull : low_mask(rl);
    const uint64_t mh = rl >= 64 ? low_mask(rl - 64) : 0ull;
    st |= (uint32_t)(((rlimb & low_mask(rr)) != 0) | ((nzl & ml) != 0) | ((nzh & mh) != 0));
  }
  const uint32_t lsb = (uint32_t)(readlane64(m, 0) & 1ull);
  uint32_t ovf = 0;
  if (rb && (st || lsb)) m = inc_mant(m, nl, ovf);
  bl = T + ovf;
  return m;
}

// mantissa comparison: sign of a - b
LFP_FN int cmp_mant(uint64_t a, uint64_t b) {
  const uint64_t diff = ballot(a != b);
  if (!diff) return 0;
  const int t = msb64(diff);
  const uint64_t x = readlane64(a, t), y = readlane64(b, t);
  return x > y ? 1 : -1;
}

// exact |a| against |b| (zero the smallest): -1, 0, 1
LFP_FN int cmp_abs(const WF &a, const WF &b) {
  const bool za = is_zero(a), zb = is_zero(b);
  if (za || zb) return (za && zb) ? 0 : (za ? -1 : 1);
  if (a.e != b.e) return a.e > b.e ? 1 : -1;
  return cmp_mant(a.m, b.m);
}

// limb j <- limb j-1 over the window (limb 0 <- 0)
LFP_FN W2 up_limb(W2 w) {
  const int l = lane_id();
  const uint64_t a = rot1_64(w.lo), b = up1_64(w.hi);
  W2 r;
  r.lo = l ? a : 0ull;
  r.hi = l ? b : a;
  return r;
}

// a b = lo + hi 2^64 from four 32 x 32 -> 64-bit multiply-adds
LFP_FN void mul128(uint64_t a, uint64_t b, uint64_t &lo, uint64_t &hi) {
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
  const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  const uint64_t p00 = (uint64_t)a0 * b0;
  const uint64_t p01 = (uint64_t)a0 * b1 + (p00 >> 32);
  const uint64_t p10 = (uint64_t)a1 * b0 + (uint32_t)p01;
  hi = (uint64_t)a1 * b1 + (p01 >> 32) + (p10 >> 32);
  lo = (p10 << 32) | (uint32_t)p00;
}

// w (five 32-bit words, least significant first) += a b
LFP_FN void mac5(uint32_t (&w)[5], uint64_t a, uint64_t b) {
  uint64_t lo, hi;
  mul128(a, b, lo, hi);
  uint32_t c;
  w[0] = addc32(w[0], (uint32_t)lo, 0u, &c);
  w[1] = addc32(w[1], (uint32_t)(lo >> 32), c, &c);
  w[2] = addc32(w[2], (uint32_t)hi, c, &c);
  w[3] = addc32(w[3], (uint32_t)(hi >> 32), c, &c);
  w[4] += c;
}

// RN_p(a b)
LFP_FN WF mul(const WF &a, const WF &b, int nl) {
  if (is_zero(a) || is_zero(b)) return wf_zero();
  const int l = lane_id();
  // Lane l sums column l of the schoolbook product (a_i b_(l-i), i <= l),
  // then column l + 64 (a_i b_(l+64-i), i > l), in one 160-bit accumulator
  // (a column sum is below 64 2^128); the running sum is copied aside when
  // i passes l, and the high column is the final sum minus that copy.
  uint32_t w[5] = {0u, 0u, 0u, 0u, 0u}, k[5] = {0u, 0u, 0u, 0u, 0u};
  uint64_t bv = b.m;  // b_((l - i) mod 64) at step i: rotated by one lane per step
  for (int i = 0; i < nl; ++i) {
    const uint64_t ai = readlane64(a.m, i);
    const bool sw = l + 1 == i;
#pragma unroll
    for (int q = 0; q < 5; ++q) k[q] = sw ? w[q] : k[q];
    mac5(w, ai, bv);
    bv = rot1_64(bv);
  }
  const bool banked = l + 1 < nl;  // lanes >= nl-1 never reach their high column
  uint32_t lw[5], hw[5], br = 0u;
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    lw[q] = banked ? k[q] : w[q];
    const uint32_t d = addc32(w[q], ~k[q], 1u - br, &br);  // w - k, br: borrow out
    br = 1u - br;
    hw[q] = banked ? d : 0u;
  }
  W2 A, B, C;
  A.lo = ((uint64_t)lw[1] << 32) | lw[0];
  A.hi = ((uint64_t)hw[1] << 32) | hw[0];
  B.lo = ((uint64_t)lw[3] << 32) | lw[2];
  B.hi = ((uint64_t)hw[3] << 32) | hw[2];
  C.lo = lw[4];
  C.hi = hw[4];
  B = up_limb(B);
  C = up_limb(up_limb(C));  // column 2nl-2 holds one product: its c2 is 0
  uint32_t co;
  W2 S = add2(A, B, 0u, co);
  S = add2(S, C, 0u, co);
  int64_t bl;
  WF r;
  r.m = round_win(S, 0u, nl, bl);
  r.e = (int32_t)(bl + a.e + b.e - 128 * (int64_t)nl);
  r.s = (a.s ^ b.s) & 1u;
  return r;
}

// RN_p(a + (-1)^negb b)
LFP_FN WF add(const WF &a, const WF &b, uint32_t negb, int nl) {
  const uint32_t bs = (b.s ^ negb) & 1u;
  const bool za = is_zero(a), zb = is_zero(b);
  if (za && zb) return wf_zero();
  if (zb) return a;
  if (za) {
    WF r = b;
    r.s = bs;
    return r;
  }
  // X the operand of larger magnitude
  const int c = (a.e != b.e) ? (a.e > b.e ? 1 : -1) : cmp_mant(a.m, b.m);
  const bool sw = c < 0;
  const uint64_t Xm = sw ? b.m : a.m, Ym = sw ? a.m : b.m;
  const int32_t Xe = sw ? b.e : a.e, Ye = sw ? a.e : b.e;
  const uint32_t Xs = sw ? bs : a.s, Ys = sw ? a.s : bs;
  const int64_t d = (int64_t)Xe - Ye;
  const int64_t p = 64 * (int64_t)nl;
  if (d >= p + 2) {
    // |Y| < 2^(Xe-p-2): below half the spacing on either side of X
    WF r;
    r.m = Xm;
    r.e = Xe;
    r.s = Xs;
    return r;
  }
  // X's bit 0 at window bit XB: room for a carry above a 4096-bit X and
  // far more guard bits than any rounding needs
  constexpr int64_t XB = 4032;
  const int l = lane_id();
  W2 X, Y;
  X.lo = reg_bits(Xm, 64 * (int64_t)l - XB);
  X.hi = reg_bits(Xm, 64 * (int64_t)(l + 64) - XB);
  Y.lo = reg_bits(Ym, 64 * (int64_t)l - XB + d);
  Y.hi = reg_bits(Ym, 64 * (int64_t)(l + 64) - XB + d);
  // Y's bits [0, k) fall below the window (k <= 65)
  uint32_t st = 0;
  const int64_t k = d - XB;
  if (k > 0) {
    const uint64_t y0 = readlane64(Ym, 0), y1 = readlane64(Ym, 1);
    st = k >= 64 ? (uint32_t)((y0 != 0) | ((y1 & low_mask((int)(k - 64))) != 0))
                 : (uint32_t)((y0 & low_mask((int)k)) != 0);
  }
  W2 S;
  uint32_t co;
  if (Xs == Ys) {
    S = add2(X, Y, 0u, co);
  } else {
    // one more unit off when Y lost bits: the exact difference then lies
    // strictly between S and S + 1, which the sticky bit records
    S = sub2(X, Y, st, co);
  }
  if (ballot(S.lo != 0 || S.hi != 0) == 0) return wf_zero();  // exact cancellation: +0
  int64_t bl;
  WF r;
  r.m = round_win(S, st, nl, bl);
  r.e = (int32_t)(bl + Xe - p - XB);
  r.s = Xs;
  return r;
}

// floor((2^128 - 1) / v) - 2^64 for 2^63 <= v < 2^64: the reciprocal with
// which Moller and Granlund divide two words by the invariant word v; by
// binary long division of (2^64 - 1 - v) 2^64 + (2^64 - 1), whose high word
// is below v.
LFP_FN uint64_t recip64(uint64_t v) {
  uint64_t r = ~v, q = 0;
  for (int i = 0; i < 64; ++i) {
    const uint64_t top = r >> 63;
    r = (r << 1) | 1ull;
    q <<= 1;
    if (top || r >= v) {
      r -= v;
      q |= 1ull;
    }
  }
  return q;
}

// floor((u1 2^64 + u0) / v) for u1 < v, v >= 2^63, vinv = recip64(v)
// (Moller and Granlund, "Improved division by invariant integers", 2011,
// the two-by-one division with its two conditional corrections)
LFP_FN uint64_t div2by1(uint64_t u1, uint64_t u0, uint64_t v, uint64_t vinv) {
  uint64_t p0, p1;
  mul128(vinv, u1, p0, p1);
  const uint64_t q0 = p0 + u0;
  uint64_t q1 = p1 + u1 + (q0 < p0 ? 1ull : 0ull) + 1ull;
  uint64_t r = u0 - q1 * v;
  if (r > q0) {
    q1 -= 1;
    r += v;
  }
  if (r >= v) q1 += 1;
  return q1;
}

// RN_p(a / b); b must be non-zero (a zero b gives zero).  Long division on
// 64-bit digits: digit = min(floor(top two remainder digits / top divisor
// digit), 2^64 - 1), at most two add-backs (Knuth, TAOCP 4.3.1, Theorem B).
LFP_FN WF div(const WF &a, const WF &b, int nl) {
  if (is_zero(a) || is_zero(b)) return wf_zero();
  const int l = lane_id();
  const bool act = l < nl;
  const uint64_t V = b.m;
  const uint64_t v1 = readlane64(V, nl - 1);  // top divisor digit, >= 2^63
  const uint64_t vinv = recip64(v1);
  // leading quotient digit d0 = floor(ma / mb) in {0, 1}
  const uint32_t d0 = cmp_mant(a.m, V) >= 0 ? 1u : 0u;
  uint64_t R = a.m;
  uint32_t bo;
  if (d0) R = sub1(R, V, nl, 0u, bo);
  // nl + 1 further digits: limb nl - i of Q takes digit i (i <= nl), dl the last
  const int K = nl + 1;
  uint64_t Q = 0, dl = 0;
  for (int i = 1; i <= K; ++i) {
    // R <- R 2^64 (R < V): its top limb becomes the digit above limb nl-1
    const uint64_t ut = readlane64(R, nl - 1);
    const uint64_t un = nl >= 2 ? readlane64(R, nl - 2) : 0ull;  // nl is uniform
    const uint64_t Rs = up1_64(R);
    R = act ? Rs : 0ull;
    uint64_t qh = ut >= v1 ? ~0ull : div2by1(ut, un, v1, vinv);
    // T = qh V: lane k's product lo + hi 2^64, hi moving to lane k+1
    uint64_t lo, hi;
    mul128(qh, V, lo, hi);
    const uint64_t hin = up1_64(hi);
    uint64_t T = lo + hin;
    uint32_t c63;
    const uint64_t cm = chain(ballot(act && T < lo), ballot(act && T == ~0ull), 0u, c63);
    T = act ? T + bit_of(cm, l) : 0ull;
    const uint64_t ttop = readlane64(hi, nl - 1) + out_at(cm, c63, nl);  // <= 2^64 - 1
    uint32_t bt;
    R = sub1(R, T, nl, 0u, bt);
    // the remainder lies in [-2V, V): its top digit, signed, is -2, -1 or 0
    int64_t top = (int64_t)(ut - ttop - bt);
    for (int k = 0; k < 2 && top < 0; ++k) {
      qh -= 1;
      uint32_t cy;
      R = add1(R, V, nl, 0u, cy);
      top += cy;
    }
    if (i < K) {
      Q = (l == nl - i) ? qh : Q;
    } else {
      dl = qh;
    }
  }
  const uint32_t rem = ballot(R != 0) != 0 ? 1u : 0u;
  uint64_t m;
  uint32_t rb, st;
  if (!d0) {
    // quotient bits: Q (p bits), then the last digit
    m = Q;
    rb = (uint32_t)(dl >> 63);
    st = (uint32_t)((dl << 1) != 0) | rem;
  } else {
    // a leading 1 before Q: shift right by one
    const uint64_t above = shfl64(Q, (l + 1) & 63);
    m = act ? ((Q >> 1) | ((l + 1 < nl ? above : 0ull) << 63)) : 0ull;
    if (l == nl - 1) m |= 1ull << 63;
    rb = (uint32_t)(readlane64(Q, 0) & 1ull);
    st = (uint32_t)(dl != 0) | rem;
  }
  const uint32_t lsb = (uint32_t)(readlane64(m, 0) & 1ull);
  uint32_t ovf = 0;
  if (rb && (st || lsb)) m = inc_mant(m, nl, ovf);
  WF r;
  r.m = m;
  r.e = a.e - b.e + (int32_t)d0 + (int32_t)ovf;
  r.s = (a.s ^ b.s) & 1u;
  return r;
}

// RN_p(c - RN_p(a b)): the multiply-subtract of the panel, the U12 solve
// and the substitutions
LFP_FN WF fms(const WF &c, const WF &a, const WF &b, int nl) {
  return add(c, mul(a, b, nl), 1u, nl);
}

}  // namespace lfp
