// Per-element building blocks of the Ozaki-II product (Sec. 3.1-3.3 of the
// paper): fixed-point conversion of an expansion (Eq. direct), balanced
// slicing, centred residues, CRT of one digit group (Eq. crt) and the final
// greedy round-to-nearest.  Everything is exact integer arithmetic on 32-bit
// words or 16-bit digits held in fixed-size arrays with compile-time sizes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#define OZ_HD __host__ __device__ __forceinline__

namespace ozk {

constexpr int MAXMOD = 64;   // moduli a plan may use
constexpr int NHMAX = 20;    // 16-bit digits of one slice (w <= 300)
constexpr int NDCRT = 32;    // 16-bit digits of sum_l t_l M_l (log2 P <= 470)
constexpr int32_t EXP_ZERO = INT32_MIN;

// Tables of one plan, resident in device memory (read with uniform indices).
struct DevPlan {
  int32_t S, w, Q, nmod, g0, ng, nwx, nh;
  int32_t m[MAXMOD];
  int32_t y[MAXMOD];
  double inv_m[MAXMOD];
  uint32_t pw16[MAXMOD][NHMAX];   // 2^(16k) mod m
  uint32_t p2w[MAXMOD];           // 2^w mod m
  uint16_t Mdig[MAXMOD][NDCRT];   // M_l = P/m_l in 16-bit digits
  uint16_t Pdig[NDCRT];           // P in 16-bit digits
  int32_t nd;                     // digits used for the CRT sums
  // Byte back-ends (moduli <= 256): one 16-word record per modulus, read by
  // the producer with scalar loads.  Words 0..9: the bytes 2^(8b) mod m,
  // four per word (b = 4j .. 4j+3), zero beyond the nwt words of a slice
  // window; then h = floor(m/2), h + ((-2^w) mod m), h + ((-2^(32 nwt)) mod m),
  // magic = ceil(2^(32-k) / m) < 2^24, m and the pre-shift k.
  int32_t nwt;                    // 32-bit words of a slice window: ceil((w+2)/32)
  uint32_t rec[MAXMOD][16];
  // CRT of the byte back-ends, four moduli per table word: for moduli
  // 4c .. 4c+3, word k < CRT4_NB packs byte k of each M_l, word CRT4_NB the
  // low and word CRT4_NB + 1 the high byte of f_l = round(2^16 / m_l)
  // (zero for moduli beyond nmod).  pbyte: the bytes of P.
  uint32_t crt4[MAXMOD / 4][50];
  int32_t pbyte[48];
  // The same CRT on the matrix cores: table column j of modulus l is f_l's
  // low (j = 0) or high (j = 1) balanced byte, or balanced byte j - 2 of M_l
  // (j < 48; balanced bytes lie in [-128, 127], so sum_j b_j 2^(8 (j-2))
  // is M_l exactly: bytes 46, 47 of M_l < 2^363 are 0).  crtm holds the columns as the A operand of
  // v_mfma_i32_16x16x64_i8, one 1 KiB block per 16 columns: lane L owns
  // column 16 blk + L % 16 for moduli 16 (L / 16) .. + 15 (zero beyond
  // nmod).  The t-values enter as t - 128; crtc[j] = 128 sum_l (column j of
  // modulus l) restores sum_l t_l b_jl.
  int8_t crtm[3][64][16];
  int32_t crtc[48];
};
constexpr int CRT4_NB = 48, CRT4_W = 50;
constexpr int REC_H = 10, REC_HW = 11, REC_HT = 12, REC_MAGIC = 13, REC_M = 14, REC_K = 15;
constexpr int REC_PWMAX = 10;

// Bits [32k, 32k+32) of mag * 2^s (mag < 2^54, s may be negative: the bits
// below 2^0 are dropped, i.e. the value is truncated toward zero).
OZ_HD uint32_t word_of_shifted(uint64_t mag, int s, int k) {
  int d = s - 32 * k;
  if (d >= 0) return d < 32 ? (uint32_t)(mag << d) : 0u;
  int r = -d;
  return r < 64 ? (uint32_t)(mag >> r) : 0u;
}

// Decompose a non-zero finite double: |x| = mag * 2^(e - 53), e = frexp
// exponent for normal numbers.
OZ_HD void split_double(double x, uint64_t &mag, int &e) {
  uint64_t bits;
  __builtin_memcpy(&bits, &x, 8);
  int be = (int)((bits >> 52) & 0x7ff);
  uint64_t f = bits & ((1ull << 52) - 1);
  if (be == 0) {  // subnormal: |x| = f * 2^-1074
    mag = f;
    e = -1074 + 53;
  } else {
    mag = f | (1ull << 52);
    e = be - 1022;
  }
}

// frexp exponent of the leading non-zero component, EXP_ZERO for zero.
template <int NC>
OZ_HD int32_t exponent_of(const double *x) {
  int32_t r = EXP_ZERO;
  bool found = false;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    double v = x[c];
    if (!found && v != 0.0) {
      found = true;
      uint64_t bits;
      __builtin_memcpy(&bits, &v, 8);
      int be = (int)((bits >> 52) & 0x7ff);
      if (be != 0) {
        r = be - 1022;
      } else {
        uint64_t f = bits & ((1ull << 52) - 1);
        r = -1074 + (64 - __builtin_clzll(f));
      }
    }
  }
  return r;
}

// X = sum_c sgn(x_c) floor(|x_c| 2^mu) in NWX-word two's complement.
template <int NC, int NWX>
OZ_HD void to_fixed(const double *x, int mu, uint32_t (&X)[NWX]) {
#pragma unroll
  for (int k = 0; k < NWX; ++k) X[k] = 0u;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    double v = x[c];
    if (v != 0.0) {
      uint64_t mag;
      int e;
      split_double(v, mag, e);
      int s = e - 53 + mu;
      uint32_t carry = 0;
      if (v > 0.0) {
#pragma unroll
        for (int k = 0; k < NWX; ++k) {
          uint64_t t = (uint64_t)X[k] + word_of_shifted(mag, s, k) + carry;
          X[k] = (uint32_t)t;
          carry = (uint32_t)(t >> 32);
        }
      } else {
        uint32_t borrow = 0;
#pragma unroll
        for (int k = 0; k < NWX; ++k) {
          uint64_t sub = (uint64_t)word_of_shifted(mag, s, k) + borrow;
          uint64_t t = (uint64_t)X[k] - sub;
          X[k] = (uint32_t)t;
          borrow = (uint32_t)((t >> 63) & 1u);
        }
      }
      (void)carry;
    }
  }
}

// residue in [0, m) of x < 2^53 given as a double-exact integer
OZ_HD uint32_t mod_small(double x, int32_t m, double inv_m) {
  double q = __builtin_floor(x * inv_m);
  double r = __builtin_fma(-q, (double)m, x);
  if (r < 0.0) r += (double)m;
  if (r >= (double)m) r -= (double)m;
  return (uint32_t)r;
}

// Residues mod every modulus of the NH 16-bit digits dig (an unsigned value):
// r_l = (sum_k dig_k (2^16k mod m_l)) mod m_l.  WIDE: moduli up to 2^23 (the
// binary64 back-end), summed in 64 bits (< 2^44); otherwise m <= 256 and the
// sum stays below 2^29.
template <int NH, bool WIDE>
OZ_HD uint32_t digits_mod(const uint32_t (&dig)[NH], const DevPlan *pl, int l) {
  if (WIDE) {
    uint64_t acc = 0;
#pragma unroll
    for (int k = 0; k < NH; ++k) acc += (uint64_t)dig[k] * pl->pw16[l][k];
    return mod_small((double)acc, pl->m[l], pl->inv_m[l]);
  }
  uint32_t acc = 0;
#pragma unroll
  for (int k = 0; k < NH; ++k) acc += dig[k] * pl->pw16[l][k];
  return mod_small((double)acc, pl->m[l], pl->inv_m[l]);
}

// centred residue in [-floor(m/2), ceil(m/2)-1] of r in [0, m)
OZ_HD int32_t centre(uint32_t r, int32_t m) {
  return (int32_t)r >= (m + 1) / 2 ? (int32_t)r - m : (int32_t)r;
}

// ---------------------------------------------------------------------------
// CRT of one digit group (Eq. crt, GPU encoding): Sbar = sum t_l M_l -
// round(F) P with F = sum t_l / m_l.  Output as two's-complement 16-bit digits
// held in int32 (after carry propagation every digit is in [0, 2^16) except
// the top one, which carries the sign).
// ---------------------------------------------------------------------------
// ND digits (ND*16 bits) must hold sum_l t_l M_l < nmod P; the plan checks.
// TT: uint8_t t-values (moduli <= 256: digit sums t M_dig < 2^24 each, summed
// in int32) or uint32_t (moduli < 2^23: products < 2^39, summed in int64).
template <int ND, class TT>
OZ_HD void crt_digits(const TT *t, int64_t stride, const DevPlan *pl, int32_t (&d)[ND]) {
  typedef typename std::conditional<sizeof(TT) == 1, int32_t, int64_t>::type Acc;
  Acc a[ND];
#pragma unroll
  for (int k = 0; k < ND; ++k) a[k] = 0;
  double F = 0.0;
  for (int l = 0; l < pl->nmod; ++l) {
    const uint32_t tl = (uint32_t)t[l * stride];
    F += (double)tl * pl->inv_m[l];
#pragma unroll
    for (int k = 0; k < ND; ++k) a[k] += (Acc)tl * (Acc)pl->Mdig[l][k];
  }
  const Acc q = (Acc)__builtin_floor(F + 0.5);
#pragma unroll
  for (int k = 0; k < ND; ++k) a[k] -= q * (Acc)pl->Pdig[k];
  Acc carry = 0;
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    Acc v = a[k] + carry;
    d[k] = (int32_t)(v & 0xffff);
    carry = v >> 16;  // arithmetic
  }
  // |Sbar| < P/2 fits the ND digits, so they are the two's complement of Sbar
  // and the top digit carries the sign; the final carry holds nothing more.
  (void)carry;
  d[ND - 1] = (int32_t)(int16_t)(uint16_t)d[ND - 1];
}

// ---------------------------------------------------------------------------
// Multiword helpers and the final rounding (S6)
// ---------------------------------------------------------------------------
template <int NW>
OZ_HD void negate_words(uint32_t (&a)[NW]) {
  uint32_t carry = 1;
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    uint64_t t = (uint64_t)(~a[k]) + carry;
    a[k] = (uint32_t)t;
    carry = (uint32_t)(t >> 32);
  }
}

// funnel shift: the 32 bits of (hi:lo) << s, 0 <= s < 32
OZ_HD uint32_t shl_funnel(uint32_t hi, uint32_t lo, int s) {
  return s ? (uint32_t)((((uint64_t)hi << 32) | lo) >> (32 - s)) : hi;
}

// Greedy round-to-nearest (ties to even) of the NW-word two's-complement
// integer cb times 2^eps into NC doubles: x_0 = RN(c), x_k = RN(c - x_0 -
// ... - x_(k-1)) with every remainder exact; a component below 2^-1022 is
// flushed and ends the expansion.  Worked on sign and magnitude: every
// component first normalises the remainder's magnitude so that its leading
// bit is bit 32 NW - 1 (a shift by whole words through a fixed network of
// selects, then one funnel shift), after which the 53-bit head, the
// rounding bit and the sticky bits sit at fixed word positions.  The next
// remainder is the magnitude below the head, negated (2^P - low, P the
// head's lowest bit position) when the head was rounded up, which also
// flips the sign.
template <int NW, int NC>
OZ_HD void round_out_n(const uint32_t (&cb)[NW], int eps, double (&x)[NC]) {
  static_assert(NW >= 3 && NW <= 16, "word count");
  uint32_t N[NW];
  bool neg = (cb[NW - 1] >> 31) != 0;
  {
    uint32_t carry = 1;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      const uint32_t v = neg ? ~cb[k] : cb[k];
      const uint64_t t = (uint64_t)v + (neg ? carry : 0u);
      N[k] = (uint32_t)t;
      carry = (uint32_t)(t >> 32);
    }
  }
  int sh = 0;  // N = |remainder| 2^sh
#pragma unroll
  for (int c = 0; c < NC; ++c) x[c] = 0.0;
  bool done = false;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    int tw = -1;
#pragma unroll
    for (int k = 0; k < NW; ++k) tw = N[k] != 0u ? k : tw;
    done = done || tw < 0;
    // whole-word shift by NW - 1 - tw
    const int sw = done ? 0 : NW - 1 - tw;
#pragma unroll
    for (int b = 8; b >= 1; b >>= 1) {
      if (b < NW) {
        const bool on = (sw & b) != 0;
#pragma unroll
        for (int k = NW - 1; k >= 0; --k) N[k] = on ? (k >= b ? N[k - b] : 0u) : N[k];
      }
    }
    const int lz = done ? 0 : __builtin_clz(N[NW - 1] | 1u);
#pragma unroll
    for (int k = NW - 1; k >= 1; --k) N[k] = shl_funnel(N[k], N[k - 1], lz);
    N[0] = lz ? N[0] << lz : N[0];
    sh += 32 * sw + lz;
    const uint64_t hi = ((uint64_t)N[NW - 1] << 32) | N[NW - 2];
    uint64_t m = hi >> 11;
    const uint32_t rb = (uint32_t)((hi >> 10) & 1u);
    uint32_t below = (uint32_t)(hi & 0x3ffu);
#pragma unroll
    for (int k = 0; k < NW - 2; ++k) below |= N[k];
    const bool up = rb && (below != 0u || (m & 1ull));
    m += up ? 1u : 0u;
    const int ex = 32 * NW - sh - 53;  // value of the head: m 2^ex
    const int top = (63 - __builtin_clzll(m | 1ull)) + ex + eps;
    done = done || top < -1022;
    if (!done) {
      const double v = __builtin_ldexp((double)m, ex + eps);
      x[c] = neg ? -v : v;
    }
    // the remainder below the head, P = 32 (NW - 2) + 11 bits
    N[NW - 1] = 0u;
    N[NW - 2] &= 0x7ffu;
    uint32_t carry = 1;
#pragma unroll
    for (int k = 0; k < NW - 1; ++k) {
      const uint64_t t = (uint64_t)(up ? ~N[k] : N[k]) + (up ? carry : 0u);
      N[k] = (uint32_t)t;
      carry = (uint32_t)(t >> 32);
    }
    N[NW - 2] &= 0x7ffu;
    neg = neg != up;
  }
}

// ---------------------------------------------------------------------------
// Producer, one element: fixed point (Eq. direct), balanced slices
// v_0 .. v_{S-1} of width w (Sec. 3.2), centred residues of every slice for
// every modulus, handed to store(t, l, r).  st: STG words of scratch
// (thread-private) used for the arithmetic right shift by w.
// ---------------------------------------------------------------------------
constexpr int STG = 29;

template <int NC, int NWX, int NH, bool WIDE, class Store>
OZ_HD void produce_element(const double *src, int mu, const DevPlan *pl, uint32_t *st, Store store) {
  static_assert(NWX + 16 <= STG, "staging too small");
  const int S = pl->S, w = pl->w, nmod = pl->nmod;
  const int q0 = w >> 5, b0 = w & 31;
  uint32_t Xw[NWX];
#pragma unroll
  for (int k = 0; k < NWX; ++k) Xw[k] = 0u;
  if (src) to_fixed<NC, NWX>(src, mu, Xw);
  for (int t = 0; t < S; ++t) {
    uint32_t dig[NH];
    bool neg = false;
    uint32_t flag = 0;
    if (t < S - 1) {
      // the low w bits as 16-bit digits
#pragma unroll
      for (int k = 0; k < NH; ++k) {
        uint32_t word = (k / 2 < NWX) ? Xw[k / 2] : 0u;
        uint32_t d = (word >> (16 * (k & 1))) & 0xffffu;
        int nb = w - 16 * k;
        d = nb >= 16 ? d : (nb <= 0 ? 0u : (d & ((1u << nb) - 1u)));
        dig[k] = d;
      }
      // the slice is centred (v = field - 2^w) when bit w-1 is set
#pragma unroll
      for (int k = 0; k < NWX; ++k)
        if (k == ((w - 1) >> 5)) flag = (Xw[k] >> ((w - 1) & 31)) & 1u;
    } else {
      uint32_t mag[NWX];
#pragma unroll
      for (int k = 0; k < NWX; ++k) mag[k] = Xw[k];
      neg = (mag[NWX - 1] >> 31) != 0;
      if (neg) negate_words<NWX>(mag);
#pragma unroll
      for (int k = 0; k < NH; ++k) {
        uint32_t word = (k / 2 < NWX) ? mag[k / 2] : 0u;
        dig[k] = (word >> (16 * (k & 1))) & 0xffffu;
      }
    }
    for (int l = 0; l < nmod; ++l) {
      const int32_t m = pl->m[l];
      uint32_t r = digits_mod<NH, WIDE>(dig, pl, l);
      if (t < S - 1) {
        if (flag) {
          r += (uint32_t)m - pl->p2w[l];  // r - 2^w (mod m)
          r = r >= (uint32_t)m ? r - (uint32_t)m : r;
        }
      } else if (neg) {
        r = r == 0 ? 0u : (uint32_t)m - r;
      }
      store(t, l, centre(r, m));
    }
    if (t < S - 1) {
      // X <- (X >> w) + flag, an exact division since the slice was removed
      const uint32_t fill = (Xw[NWX - 1] >> 31) ? 0xffffffffu : 0u;
#pragma unroll
      for (int k = 0; k < NWX; ++k) st[k] = Xw[k];
#pragma unroll
      for (int k = NWX; k < STG; ++k) st[k] = fill;
      uint32_t carry = flag;
#pragma unroll
      for (int k = 0; k < NWX; ++k) {
        int s = k + q0;
        uint32_t lo = st[s < STG ? s : STG - 1];
        uint32_t hi = st[s + 1 < STG ? s + 1 : STG - 1];
        uint32_t v = b0 ? ((lo >> b0) | (hi << (32 - b0))) : lo;
        uint64_t tt = (uint64_t)v + carry;
        Xw[k] = (uint32_t)tt;
        carry = (uint32_t)(tt >> 32);
      }
    }
  }
}

// cb += Sbar 2^off (mod 2^(32 NWC)), Sbar given as ND two's-complement 16-bit
// digits (the top one signed); st: STG words of thread-private scratch.  The
// digits fill st[0, ND/2) and the sign fill the rest; a shifted read past the
// end takes the last word, which is a fill word, so STG = ND/2 + 1 suffices.
// An odd STG keeps the per-thread rows in distinct LDS banks.
constexpr int CST = 33;
template <int ND>
constexpr int stage_words() { return (ND / 2 + 1) | 1; }

template <int NWC, int ND, int STG = CST>
OZ_HD void add_shifted_digits(uint32_t (&cb)[NWC], const int32_t (&d)[ND], int off, uint32_t *st) {
  static_assert(ND % 2 == 0 && ND / 2 + 1 <= STG, "staging too small");
  const uint32_t fill = d[ND - 1] < 0 ? 0xffffffffu : 0u;
#pragma unroll
  for (int k = 0; k < ND / 2; ++k)
    st[k] = ((uint32_t)d[2 * k] & 0xffffu) | ((uint32_t)d[2 * k + 1] << 16);
#pragma unroll
  for (int k = ND / 2; k < STG; ++k) st[k] = fill;
  const int q0 = off >> 5, b0 = off & 31;
  uint32_t carry = 0;
#pragma unroll
  for (int k = 0; k < NWC; ++k) {
    const int s = k - q0;
    uint32_t cur = s >= 0 ? st[s < STG ? s : STG - 1] : 0u;
    uint32_t prv = s - 1 >= 0 ? st[s - 1 < STG ? s - 1 : STG - 1] : 0u;
    uint32_t v = b0 ? ((cur << b0) | (prv >> (32 - b0))) : cur;
    uint64_t tt = (uint64_t)cb[k] + v + carry;
    cb[k] = (uint32_t)tt;
    carry = (uint32_t)(tt >> 32);
  }
}

// ---------------------------------------------------------------------------
// Consumer, one element: CRT of every retained digit group, exact sum
// cbar = sum_gi Sbar_{g0+gi} 2^(w gi), greedy rounding to NC components of
// cbar 2^eps.  tptr(gi) points at t_0 of group gi; consecutive moduli are
// pstride bytes apart.  st: CST words of thread-private scratch.
// ---------------------------------------------------------------------------
template <int NC, int NWC, int ND, class TT, class TPtr>
OZ_HD void consume_element(TPtr tptr, int64_t pstride, const DevPlan *pl, uint32_t *st, bool zero,
                           int eps, double (&c)[NC]) {
  static_assert(ND % 2 == 0 && ND <= NDCRT, "digits");
  const int w = pl->w, ng = pl->ng;
  uint32_t cb[NWC];
#pragma unroll
  for (int k = 0; k < NWC; ++k) cb[k] = 0u;
  for (int gi = 0; gi < ng; ++gi) {
    int32_t d[ND];
    crt_digits<ND, TT>(tptr(gi), pstride, pl, d);
    add_shifted_digits<NWC, ND>(cb, d, w * gi, st);
  }
  if (zero) {
#pragma unroll
    for (int q = 0; q < NC; ++q) c[q] = 0.0;
  } else {
    round_out_n<NWC, NC>(cb, eps, c);
  }
}

}  // namespace ozk
