// Device helpers of the byte back-ends shared by the expansion and limb
// producers: the residues of Sec. 3.2 slices for every modulus (moduli <=
// 256), written four elements per dword into the residue planes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ozii_elem.hpp"

namespace ozk {

// OCP FP8 E4M3 byte of an integer |d| <= 8 (sign, exponent bias 7, 3-bit
// fraction): d = 2^e (1 + f/8) with e = floor(log2 |d|).
__device__ __forceinline__ uint8_t e4m3_small(int32_t d) {
  const uint32_t a = (uint32_t)(d < 0 ? -d : d);
  const uint32_t sign = d < 0 ? 0x80u : 0u;
  if (a == 0) return (uint8_t)sign;
  const uint32_t e = 31u - (uint32_t)__builtin_clz(a);
  const uint32_t f = ((a << 3) >> e) & 7u;
  return (uint8_t)(sign | ((e + 7u) << 3) | f);
}

// v_mul_u32_u24 (full rate; the compiler selects the quarter-rate 32-bit
// multiply for operands it cannot prove to be 24-bit)
__device__ __forceinline__ uint32_t mul_u24(uint32_t a, uint32_t b) {
  uint32_t r;
  asm("v_mul_u32_u24 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// Residues of slice t of four elements (EPT = 4) for the moduli l0 .. l1-1
// (pp at the plane of modulus l0), stored as one dword (four consecutive
// bytes of a plane) per modulus; EPT = 1: one element, one byte.  F: the slice words
// (NWM 32-bit words, zero above the slice), sel: whether the (-2^W) mod m
// term applies (centring flag, or the sign of the top slice), base: REC_HW
// or REC_HT.  The residue of modulus m is
//   (sum_b byte_b (2^(8b) mod m) + [sel] ((-2^W) mod m)) mod m,
// the byte sum a chain of v_dot4_u32_u8 with the table words (scalar
// registers).  With h = floor(m/2) added first, the centred residue is
// acc - floor(acc/m) m - h, and floor(acc/m) is exact as the high word of
// (acc << k) * ceil(2^(32-k)/m): acc < 2^(32-k)/m and (acc << k) < 2^24 for
// slices of at most 10 words.  FP8: the balanced base-17 digits of Eq.
// (fp8digits) as E4M3 bytes, d0 then d1 plane.
template <int NWM, bool FP8, int EPT = 4>
__device__ __forceinline__ void emit_byte_residues(const uint32_t (&F)[EPT][NWM],
                                                   const uint32_t (&sel)[EPT], int base,
                                                   const DevPlan *__restrict__ pl, int l0, int l1,
                                                   uint8_t *pp, int64_t plane_elems,
                                                   uint32_t offb) {
  static_assert(EPT == 4 || EPT == 1, "four elements per dword, or one byte");
  for (int l = l0; l < l1; ++l, pp += (FP8 ? 2 : 1) * plane_elems) {
    const uint32_t *R = pl->rec[l];
    const uint32_t m = R[REC_M], h = R[REC_H], magic = R[REC_MAGIC], ks = R[REC_K];
    const uint32_t hs = R[base];
    int32_t c[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      uint32_t acc = sel[e] ? hs : h;
#pragma unroll
      for (int j = 0; j < NWM; ++j) acc = __builtin_amdgcn_udot4(F[e][j], R[j], acc, false);
      const uint32_t qq =
          (uint32_t)(((uint64_t)((acc << ks) & 0xffffffu) * (uint64_t)(magic & 0xffffffu)) >> 32);
      c[e] = (int32_t)(acc - mul_u24(qq, m) - h);
    }
    if (!FP8) {
      if constexpr (EPT == 4) {
        const uint32_t word = (uint32_t)(c[0] & 0xff) | ((uint32_t)(c[1] & 0xff) << 8) |
                              ((uint32_t)(c[2] & 0xff) << 16) | ((uint32_t)c[3] << 24);
        *(uint32_t *)(pp + offb) = word;
      } else {
        pp[offb] = (uint8_t)c[0];
      }
    } else {
      // d1 = round(c/17) (never a tie), d0 = c - 17 d1; floor((c+144)/17)
      // as a multiply-high, exact for |c| <= 128
      uint32_t w0 = 0, w1 = 0;
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int32_t d1 = (int32_t)(((uint32_t)(c[e] + 144) * 3856u) >> 16) - 8;
        const int32_t d0 = c[e] - 17 * d1;
        w0 |= (uint32_t)e4m3_small(d0) << (8 * e);
        w1 |= (uint32_t)e4m3_small(d1) << (8 * e);
      }
      if constexpr (EPT == 4) {
        *(uint32_t *)(pp + offb) = w0;
        *(uint32_t *)(pp + plane_elems + offb) = w1;
      } else {
        pp[offb] = (uint8_t)w0;
        pp[plane_elems + offb] = (uint8_t)w1;
      }
    }
  }
}

// CRT of one digit group (Eq. crt) for t-values below 256, as ND = NB/2
// two's-complement 16-bit digits (the top one signed).  tp points at t_0 of
// the element, consecutive moduli ps bytes apart.  sum_l t_l M_l is formed
// in NB byte columns with v_dot4_u32_u8, four moduli per instruction (their
// t-bytes packed into one word against the packed bytes of their M_l, table
// words in scalar registers); each column stays below 2^22.  F = sum_l t_l /
// m_l comes from the same instruction with f_l = round(2^16 / m_l): its error
// is below 54 * 255 / 2^17 < 0.11, and F lies within 2^-7 of an integer (the
// plan keeps |Sbar| < P 2^-7), so round(F) is exact.  Then Sbar =
// sum_k (col_k - round(F) P_k) 2^(8k), carried into 16-bit digits.
template <int NB, int PRE = 0>
__device__ __forceinline__ void crt_group_bytes(const uint8_t *tp, int64_t ps, int nmod,
                                                const DevPlan *__restrict__ pl,
                                                int32_t (&d)[NB / 2]) {
  static_assert(NB % 4 == 0 && NB <= CRT4_NB, "byte columns");
  constexpr int ND = NB / 2;
  const int nch = (nmod + 3) >> 2;
  // moduli past nmod read the last plane again: their table bytes are zero.
  // PRE = 0: the bytes of the next four moduli are loaded one chunk ahead
  // and packed only when used (enough with many wavefronts per CU to cover
  // the latency); PRE > 0 (callers with few wavefronts per CU, nmod <= 4 PRE):
  // the bytes of all PRE chunks are requested before the first product.
  uint32_t col[NB], F0 = 0, F1 = 0;
#pragma unroll
  for (int k = 0; k < NB; ++k) col[k] = 0u;
  auto chunk = [&](int c, uint32_t tw) {
    const uint32_t *T = pl->crt4[c];
#pragma unroll
    for (int k = 0; k < NB; ++k) col[k] = __builtin_amdgcn_udot4(tw, T[k], col[k], false);
    F0 = __builtin_amdgcn_udot4(tw, T[CRT4_NB], F0, false);
    F1 = __builtin_amdgcn_udot4(tw, T[CRT4_NB + 1], F1, false);
  };
  if constexpr (PRE > 0) {
    uint32_t bt[PRE][4];
#pragma unroll
    for (int c = 0; c < PRE; ++c)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int l = 4 * c + e < nmod ? 4 * c + e : nmod - 1;
        bt[c][e] = tp[(int64_t)l * ps];
      }
#pragma unroll
    for (int c = 0; c < PRE; ++c)
      if (c < nch) chunk(c, bt[c][0] | (bt[c][1] << 8) | (bt[c][2] << 16) | (bt[c][3] << 24));
  } else {
    uint32_t bt[4];
    auto load4 = [&](int c) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int l = 4 * c + e < nmod ? 4 * c + e : nmod - 1;
        bt[e] = tp[(int64_t)l * ps];
      }
    };
    load4(0);
    for (int c = 0; c < nch; ++c) {
      const uint32_t tw = bt[0] | (bt[1] << 8) | (bt[2] << 16) | (bt[3] << 24);
      if (c + 1 < nch) load4(c + 1);
      chunk(c, tw);
    }
  }
  const int32_t q = (int32_t)((F0 + (F1 << 8) + 32768u) >> 16);
  int32_t carry = 0;
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    const int32_t lo = (int32_t)col[2 * k] - q * (pl->pbyte[2 * k] & 0xff);
    const int32_t hi = (int32_t)col[2 * k + 1] - q * (pl->pbyte[2 * k + 1] & 0xff);
    const int32_t v = lo + (int32_t)((uint32_t)hi << 8) + carry;
    d[k] = v & 0xffff;
    carry = v >> 16;  // arithmetic
  }
  // |Sbar| < P/2 fits the ND digits: the top one carries the sign
  d[ND - 1] = (int32_t)(int16_t)(uint16_t)d[ND - 1];
}

}  // namespace ozk
