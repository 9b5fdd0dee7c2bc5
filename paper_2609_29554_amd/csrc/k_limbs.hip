// Ozaki-II product on arbitrary-precision limb numbers (p = 64 nlimb bits,
// the MPFR-like input of Sec. 3.3 and the p-bit results of (S6)):
//   x = (-1)^sign * (sum_q limb_q 2^(64 q)) * 2^(exp - p),  mantissa normalised,
// stored as one plane per limb (limb q of element idx at limb[q*plane + idx]).
//
//   (S1) k_limb_row_exp / k_limb_col_exp: e = max exp over the non-zero
//        entries of a row of A / a column of B;
//   (S2)+(S3) k_producer_limbs: X = sgn(x) trunc(|x| 2^mu) is never formed;
//        every w-bit slice window is read straight from the limb planes
//        (negative values as the complement plus an incoming carry of one)
//        and reduced by the byte residue emitter shared with the expansion
//        producer, so the residue planes have the same layout;
//   (S4) the batched INT8 modular GEMM of the expansion path;
//   (S5) k_consumer_limbs: the byte CRT of every digit group, added at bit
//        w gi into the exact group sum cbar, kept as a column of 32-bit words
//        per element in workspace (word k of element e at cw[k*E + e]): the
//        groups arrive in increasing order, so each one rewrites only its own
//        window and the sign extension above it is carried as a small integer;
//   (S6) k_limb_round: c = RN_p(cbar 2^eps), ties to even; mode 1 then
//        k_limb_sub: C = RN_p(C - c), the exact difference on a grid with a
//        guard word and a sticky bit, rounded once.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "ozii_bytes.hpp"
#include "ozii_elem.hpp"
#include "ozii_kernels.hpp"

using namespace ozk;

namespace {

constexpr int LIMB_ROWEXP_CHUNK = 16;

// ---------------------------------------------------------------------------
// (S1)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_limb_row_exp(const uint64_t *__restrict__ limb,
                                                      const int32_t *__restrict__ lexp, int64_t ld,
                                                      int64_t plane, int nlimb, int64_t rows,
                                                      int64_t cols, int32_t *e) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= rows) return;
  const int64_t h0 = (int64_t)blockIdx.y * LIMB_ROWEXP_CHUNK;
  const int64_t h1 = h0 + LIMB_ROWEXP_CHUNK < cols ? h0 + LIMB_ROWEXP_CHUNK : cols;
  int32_t best = EXP_ZERO;
  for (int64_t h = h0; h < h1; ++h) {
    const int64_t idx = i + h * ld;
    if (limb[(int64_t)(nlimb - 1) * plane + idx] != 0) {
      const int32_t v = lexp[idx];
      best = v > best ? v : best;
    }
  }
  if (best != EXP_ZERO) atomicMax(e + i, best);
}

__global__ __launch_bounds__(256) void k_limb_col_exp(const uint64_t *__restrict__ limb,
                                                      const int32_t *__restrict__ lexp, int64_t ld,
                                                      int64_t plane, int nlimb, int64_t rows,
                                                      int64_t cols, int32_t *e) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= cols) return;
  int32_t best = EXP_ZERO;
  for (int64_t h = lane; h < rows; h += 64) {
    const int64_t idx = h + j * ld;
    if (limb[(int64_t)(nlimb - 1) * plane + idx] != 0) {
      const int32_t v = lexp[idx];
      best = v > best ? v : best;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const int32_t o = __shfl_xor(best, off, 64);
    best = o > best ? o : best;
  }
  if (lane == 0) e[j] = best;
}

// ---------------------------------------------------------------------------
// (S2)+(S3).  Block layout as the expansion producer: one workgroup fills
// one 1 KiB block (16 rows x 64 k) of every residue plane; thread T owns
// row (T/4)%16 and the four inner indices 16(T/64) + 4(T%4) + e.
// Element with mantissa m, exponent ex and shift s = ex - p + mu:
// |X| = trunc(m 2^s), so bit b of |X| is bit b - s of m.  The slice chain
// (carry c_t, centring flag) is that of the expansion producer; a negative
// X = ~|X| + 1 starts with c_0 = 1 and complemented windows.
// ---------------------------------------------------------------------------
// Binary64 moduli: the residues of slice t of the thread's four elements as
// doubles for the moduli l0 .. l1-1 (pp at the plane of modulus l0), in the
// binary64 GEMM's fragment order (1 KiB blocks of 16 rows x 8 k, lane l: row
// l%16, k l/16 and 4 + l/16; eight blocks per 64-k window; off: each
// element's offset in a plane).  F and sel as for the byte
// emitter: a lower slice has the value F - sel 2^w (F < 2^w), the top slice
// is the nwt-word two's complement F with sign sel; its magnitude is reduced
// and the residue negated.
template <int NWM>
__device__ __forceinline__ void emit_f64_residues(const uint32_t (&F)[4][NWM],
                                                  const uint32_t (&sel)[4], bool top, int nwt,
                                                  const DevPlan *__restrict__ pl, int l0, int l1,
                                                  double *pp, int64_t plane_elems,
                                                  const int64_t (&off)[4]) {
  constexpr int NH = 2 * NWM;
  static_assert(NH <= NHMAX, "slice digits");
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    uint32_t mag[NWM];
    const bool neg = top && sel[e] != 0;
    uint32_t c = 1;
#pragma unroll
    for (int k = 0; k < NWM; ++k) {
      if (top && k >= nwt) {
        mag[k] = 0u;
      } else if (neg) {
        const uint32_t v = ~F[e][k];
        mag[k] = v + c;
        c = (c && mag[k] == 0u) ? 1u : 0u;
      } else {
        mag[k] = F[e][k];
      }
    }
    uint32_t dig[NH];
#pragma unroll
    for (int k = 0; k < NH; ++k) dig[k] = (mag[k >> 1] >> (16 * (k & 1))) & 0xffffu;
    const bool flag = !top && sel[e] != 0;
    for (int l = l0; l < l1; ++l) {
      const uint32_t m = (uint32_t)pl->m[l];
      uint32_t r = digits_mod<NH, true>(dig, pl, l);
      if (flag) {
        r += m - pl->p2w[l];  // F - 2^w (mod m)
        r = r >= m ? r - m : r;
      } else if (neg) {
        r = r == 0u ? 0u : m - r;
      }
      pp[(int64_t)(l - l0) * plane_elems + off[e]] = (double)centre(r, (int32_t)m);
    }
  }
}

template <int NWM, bool F64>
__global__ __launch_bounds__(256) void k_producer_limbs(
    const uint64_t *__restrict__ limb, const int32_t *__restrict__ lexp,
    const uint8_t *__restrict__ lsign, int64_t ld, int64_t plane, int nlimb, int rowwise,
    int64_t nout, int64_t K, int64_t KB, const int32_t *__restrict__ exps,
    const DevPlan *__restrict__ pl, uint8_t *__restrict__ planes, int64_t plane_elems) {
  constexpr int NLL = (NWM + 3) / 2;  // limbs covering NWM + 2 words
  const int T = threadIdx.x;
  const int64_t kb = blockIdx.x, ob = blockIdx.y;
  const int64_t o = ob * 16 + ((T >> 2) & 15);
  const int64_t h0 = kb * 64 + 16 * (T >> 6) + 4 * (T & 3);
  const uint32_t offb = (uint32_t)((ob * KB + kb) * 1024 + 4 * T);  // < 2^31
  const int S = pl->S, w = pl->w, nmod = pl->nmod, Q = pl->Q, nwt = pl->nwt;
  const int p = 64 * nlimb;
  // blockIdx.z: a part of the moduli (small products run several parts)
  const int l0 = (int)blockIdx.z * nmod / (int)gridDim.z;
  const int l1 = ((int)blockIdx.z + 1) * nmod / (int)gridDim.z;

  int32_t ex = EXP_ZERO;
  if (o < nout) ex = exps[o];
  int64_t idx[4];
  int32_t sh[4];
  uint32_t neg[4], live[4], cin[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    idx[e] = 0;
    sh[e] = 0;
    neg[e] = 0;
    live[e] = 0;
    const int64_t h = h0 + e;
    if (ex != EXP_ZERO && h < K) {
      const int64_t id = rowwise ? o + h * ld : h + o * ld;
      if (limb[(int64_t)(nlimb - 1) * plane + id] != 0) {
        const int64_t s = (int64_t)lexp[id] - p + (Q - 1 - (int64_t)ex);
        // below -(p + 64) every bit of the value is truncated away
        if (s > -(int64_t)(p + 64)) {
          live[e] = 1;
          sh[e] = (int32_t)s;
          idx[e] = id;
          neg[e] = lsign[id] & 1u;
        }
      }
    }
    cin[e] = neg[e];
  }
  for (int t = 0; t < S; ++t) {
    const bool top = t == S - 1;
    const int wq = w >> 5, wb = w & 31;
    uint32_t F[4][NWM];
    uint32_t sel[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (live[e]) {
        const int32_t pos0 = t * w - sh[e];  // mantissa bit of the window's bit 0
        const int32_t q0 = pos0 >> 6, r0 = pos0 & 63;
        uint32_t u[2 * NLL];
#pragma unroll
        for (int k = 0; k < NLL; ++k) {
          const int32_t q = q0 + k;
          const uint64_t v = (q >= 0 && q < nlimb) ? limb[(int64_t)q * plane + idx[e]] : 0ull;
          u[2 * k] = (uint32_t)v;
          u[2 * k + 1] = (uint32_t)(v >> 32);
        }
        const bool hi = (r0 >> 5) != 0;
        const uint32_t rb = (uint32_t)(r0 & 31);
#pragma unroll
        for (int j = 0; j < NWM; ++j) {
          const uint32_t a = hi ? u[j + 1] : u[j];
          const uint32_t b = hi ? u[j + 2] : u[j + 1];
          const uint32_t v = __builtin_amdgcn_alignbit(b, a, rb);
          F[e][j] = neg[e] ? ~v : v;
        }
      } else {
#pragma unroll
        for (int j = 0; j < NWM; ++j) F[e][j] = 0u;
      }
      if (!top) {
#pragma unroll
        for (int j = 0; j < NWM; ++j)
          F[e][j] = j < wq ? F[e][j] : (j == wq ? F[e][j] & ((1u << wb) - 1u) : 0u);
      }
      uint32_t c = cin[e];
#pragma unroll
      for (int j = 0; j < NWM; ++j) {
        const uint32_t sum = F[e][j] + c;
        c = sum < c ? 1u : 0u;
        F[e][j] = sum;
      }
      if (!top) {
        uint32_t co = 0, fl = 0;
        const int fq = (w - 1) >> 5, fb = (w - 1) & 31;
#pragma unroll
        for (int j = 0; j < NWM; ++j) {
          if (j == wq) {
            co = (F[e][j] >> wb) & 1u;
            F[e][j] &= ~(1u << wb);
          }
        }
#pragma unroll
        for (int j = 0; j < NWM; ++j)
          if (j == fq) fl = (F[e][j] >> fb) & 1u;
        sel[e] = fl;
        cin[e] = co + fl;
      } else {
        uint32_t sg = 0;
#pragma unroll
        for (int j = 0; j < NWM; ++j)
          if (j == nwt - 1) sg = F[e][j] >> 31;
        sel[e] = sg;
      }
    }
    if constexpr (F64) {
      int64_t off[4];
      const int r = (T >> 2) & 15;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int kk = 16 * (T >> 6) + 4 * (T & 3) + e, k8 = kk & 7;
        off[e] = ((ob * KB + kb) * 8 + (kk >> 3)) * 128 + 2 * ((k8 & 3) * 16 + r) + (k8 >> 2);
      }
      emit_f64_residues<NWM>(F, sel, top, nwt, pl, l0, l1,
                             (double *)planes + ((int64_t)t * nmod + l0) * plane_elems,
                             plane_elems, off);
    } else {
      emit_byte_residues<NWM, false>(F, sel, top ? REC_HT : REC_HW, pl, l0, l1,
                                     planes + ((int64_t)t * nmod + l0) * plane_elems, plane_elems,
                                     offb);
    }
  }
}

// ---------------------------------------------------------------------------
// (S5): cbar = sum_gi Sbar_(g0+gi) 2^(w gi) per element, words in cw.
// Invariant after each group: cbar = sum_(k < hw) cw[k] 2^(32k) + pend 2^(32 hw)
// with hw uniform.  Group gi adds V = Sbar 2^(b0) (nvw words, sign-extended
// by fill) at word q0 = floor(w gi / 32).  After the last group the final
// pend (0 or -1, the sign) is stored at word hw.
// ---------------------------------------------------------------------------
template <int ND, class TT>
__global__ __launch_bounds__(256) void k_consumer_limbs(const TT *__restrict__ tpl,
                                                        int64_t Mp, int64_t Np, int64_t M,
                                                        int64_t N, const DevPlan *__restrict__ pl,
                                                        int nvw, uint32_t *__restrict__ cw,
                                                        int64_t E) {
  constexpr int NV = ND / 2 + 1;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i >= M || j >= N) return;
  const int64_t e = i + j * M;
  const int nmod = pl->nmod, w = pl->w, ng = pl->ng;
  const int64_t ps = Np * Mp;
  uint32_t *col = cw + e;
  auto AT = [&](int k) -> uint32_t & { return col[(int64_t)k * E]; };
  int hw = 0;
  int32_t pend = 0;
  for (int gi = 0; gi < ng; ++gi) {
    int32_t d[ND];
    const TT *tg = tpl + ((int64_t)gi * nmod * Np + j) * Mp + i;
    if constexpr (sizeof(TT) == 1)
      crt_group_bytes<2 * ND>(tg, ps, nmod, pl, d);  // byte back-ends
    else
      crt_digits<ND, TT>(tg, ps, pl, d);              // binary64 moduli
    const uint32_t fill = d[ND - 1] < 0 ? 0xffffffffu : 0u;
    uint32_t st[ND / 2];
#pragma unroll
    for (int k = 0; k < ND / 2; ++k)
      st[k] = ((uint32_t)d[2 * k] & 0xffffu) | ((uint32_t)d[2 * k + 1] << 16);
    const int off = w * gi, q0 = off >> 5, b0 = off & 31;
    const uint32_t pext = pend < 0 ? 0xffffffffu : 0u;
    // a gap below the window holds the old value's extension
    for (int k = hw; k < q0; ++k) AT(k) = k == hw ? (uint32_t)pend : pext;
    if (q0 > hw) {
      hw = q0;
      pend = pend < 0 ? -1 : 0;
    }
    const uint32_t ext = pend < 0 ? 0xffffffffu : 0u;
    uint32_t carry = 0;
#pragma unroll
    for (int r = 0; r < NV; ++r) {
      if (r < nvw) {
        const int k = q0 + r;
        const uint32_t cur = r < ND / 2 ? st[r] : fill;
        const uint32_t prv = r == 0 ? 0u : (r - 1 < ND / 2 ? st[r - 1] : fill);
        const uint32_t v = b0 ? ((cur << b0) | (prv >> (32 - b0))) : cur;
        const uint32_t old = k < hw ? AT(k) : (k == hw ? (uint32_t)pend : ext);
        const uint64_t s = (uint64_t)old + v + carry;
        AT(k) = (uint32_t)s;
        carry = (uint32_t)(s >> 32);
      }
    }
    // old words above the window still take the extension of V
    for (int k = q0 + nvw; k <= hw; ++k) {
      const uint32_t old = k < hw ? AT(k) : (uint32_t)pend;
      const uint64_t s = (uint64_t)old + fill + carry;
      AT(k) = (uint32_t)s;
      carry = (uint32_t)(s >> 32);
    }
    const int kend = q0 + nvw > hw + 1 ? q0 + nvw : hw + 1;
    pend = (int32_t)carry + (pend < 0 ? -1 : 0) + (fill ? -1 : 0);
    hw = kend;
  }
  AT(hw) = (uint32_t)pend;
}

// ---------------------------------------------------------------------------
// RN_p of a non-negative integer given word by word (MAG(k), zero outside
// [0, nw)) times 2^escale, with an extra sticky bit below everything; writes
// limbs, exponent and sign of the p-bit result (zero for a zero magnitude).
// ---------------------------------------------------------------------------
template <class MagF>
__device__ __forceinline__ void round_to_limbs(MagF MAG, int nw, bool sticky_in, int nlimb,
                                               int64_t escale, uint32_t sign, uint64_t *olimb,
                                               int64_t oplane, int64_t oi, int32_t *oexp,
                                               uint8_t *osign) {
  const int p = 64 * nlimb, pw = 2 * nlimb;
  int tw = -1;
  for (int k = nw - 1; k >= 0; --k) {
    if (MAG(k) != 0u) {
      tw = k;
      break;
    }
  }
  if (tw < 0) {
    for (int q = 0; q < nlimb; ++q) olimb[(int64_t)q * oplane + oi] = 0ull;
    oexp[oi] = EXP_ZERO;
    osign[oi] = 0;
    return;
  }
  const int L = 32 * tw + 32 - __builtin_clz(MAG(tw));
  const int sh = L - p;
  auto BITS = [&](int pos) -> uint32_t {  // bits [pos, pos + 32) of the magnitude
    const int q = pos >> 5, r = pos & 31;
    const uint32_t lo = MAG(q);
    return r ? (lo >> r) | (MAG(q + 1) << (32 - r)) : lo;
  };
  bool up = false;
  if (sh > 0) {
    const int rp = sh - 1;  // round bit position
    const uint32_t rb = (MAG(rp >> 5) >> (rp & 31)) & 1u;
    bool sticky = sticky_in || (MAG(rp >> 5) & ((1u << (rp & 31)) - 1u)) != 0u;
    for (int k = 0; k < (rp >> 5) && !sticky; ++k) sticky = MAG(k) != 0u;
    up = rb && (sticky || (BITS(sh) & 1u));
  }
  // an increment carries through the low mantissa words equal to all ones
  int f = 0;
  bool over = false;
  if (up) {
    f = -1;
    for (int m = 0; m < pw; ++m) {
      if (BITS(sh + 32 * m) != 0xffffffffu) {
        f = m;
        break;
      }
    }
    over = f < 0;
  }
  auto WORD = [&](int m) -> uint32_t {
    if (over) return m == pw - 1 ? 0x80000000u : 0u;
    const uint32_t raw = BITS(sh + 32 * m);
    if (!up || m > f) return raw;
    return m < f ? 0u : raw + 1u;
  };
  for (int q = 0; q < nlimb; ++q)
    olimb[(int64_t)q * oplane + oi] = ((uint64_t)WORD(2 * q + 1) << 32) | WORD(2 * q);
  oexp[oi] = (int32_t)(L + (over ? 1 : 0) + escale);
  osign[oi] = (uint8_t)sign;
}

// ---------------------------------------------------------------------------
// (S6): c = RN_p(cbar 2^eps), eps = w g0 - mu_i - nu_j, written as a limb
// matrix (ldo, planeo).  cbar is the two's complement column of nwords words
// (the top one the sign); its magnitude is read on demand: for a negative
// cbar, word k of -cbar is 0 below the lowest non-zero word z, -c_z at z and
// ~c_k above.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_limb_round(const uint32_t *__restrict__ cw, int64_t E,
                                                    int nwords, int64_t M, int64_t N,
                                                    const int32_t *__restrict__ ea,
                                                    const int32_t *__restrict__ eb, int w, int g0,
                                                    int Q, int nlimb, uint64_t *__restrict__ olimb,
                                                    int32_t *__restrict__ oexp,
                                                    uint8_t *__restrict__ osign, int64_t ldo,
                                                    int64_t planeo) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i >= M || j >= N) return;
  const int64_t oi = i + j * ldo;
  const int32_t ei = ea[i], ej = eb[j];
  const uint32_t *col = cw + (i + j * M);
  auto C = [&](int k) -> uint32_t { return col[(int64_t)k * E]; };
  if (ei == EXP_ZERO || ej == EXP_ZERO) {
    round_to_limbs([](int) { return 0u; }, 0, false, nlimb, 0, 0, olimb, planeo, oi, oexp, osign);
    return;
  }
  const uint32_t neg = C(nwords - 1) >> 31;
  int z = nwords;
  if (neg) {
    for (int k = 0; k < nwords; ++k) {
      if (C(k) != 0u) {
        z = k;
        break;
      }
    }
  }
  auto MAG = [&](int k) -> uint32_t {
    if (k < 0 || k >= nwords) return 0u;
    const uint32_t v = C(k);
    if (!neg) return v;
    return k < z ? 0u : (k == z ? 0u - v : ~v);
  };
  const int64_t eps = (int64_t)w * g0 - (Q - 1 - (int64_t)ei) - (Q - 1 - (int64_t)ej);
  round_to_limbs(MAG, nwords, false, nlimb, eps, neg, olimb, planeo, oi, oexp, osign);
}

// ---------------------------------------------------------------------------
// Update: C = RN_p(C - T) for p-bit limb matrices C (ldc, planec) and T
// (M x N, ld M, plane M N).  With X the operand of larger magnitude and Y
// the other, the difference is formed on the grid of X's mantissa shifted up
// by one guard word: D_m = X_(m-1) +- (bits 32(m-1) + d .. of Y), d =
// exp(X) - exp(Y); bits of Y below the grid only set a sticky bit (for a
// subtraction they lower D by one unit first, so D + sticky brackets the
// exact value).  D (pw + 2 words per element) is written to dw, then
// rounded once.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_limb_sub(uint64_t *__restrict__ climb,
                                                  int32_t *__restrict__ cexp,
                                                  uint8_t *__restrict__ csign, int64_t ldc,
                                                  int64_t planec, const uint64_t *__restrict__ tlimb,
                                                  const int32_t *__restrict__ texp,
                                                  const uint8_t *__restrict__ tsign, int nlimb,
                                                  int64_t M, int64_t N, uint32_t *__restrict__ dw,
                                                  int64_t E) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i >= M || j >= N) return;
  const int p = 64 * nlimb, pw = 2 * nlimb, nwd = pw + 2;
  const int64_t ci = i + j * ldc, ti = i + j * M, planet = M * N;
  const bool tz = tlimb[(int64_t)(nlimb - 1) * planet + ti] == 0ull;
  if (tz) return;  // C - 0 = C exactly
  const bool az = climb[(int64_t)(nlimb - 1) * planec + ci] == 0ull;
  const uint32_t sa = csign[ci] & 1u, sc = (tsign[ti] & 1u) ^ 1u;  // C + (-T)
  if (az) {
    for (int q = 0; q < nlimb; ++q)
      climb[(int64_t)q * planec + ci] = tlimb[(int64_t)q * planet + ti];
    cexp[ci] = texp[ti];
    csign[ci] = (uint8_t)sc;
    return;
  }
  auto CW = [&](int m) -> uint32_t {  // mantissa word m of C
    const uint64_t v = climb[(int64_t)(m >> 1) * planec + ci];
    return (m & 1) ? (uint32_t)(v >> 32) : (uint32_t)v;
  };
  auto TW = [&](int m) -> uint32_t {
    const uint64_t v = tlimb[(int64_t)(m >> 1) * planet + ti];
    return (m & 1) ? (uint32_t)(v >> 32) : (uint32_t)v;
  };
  const int32_t xa = cexp[ci], xt = texp[ti];
  bool cx = xa > xt;  // C is X
  if (xa == xt) {
    cx = true;
    for (int m = pw - 1; m >= 0; --m) {
      const uint32_t a = CW(m), b = TW(m);
      if (a != b) {
        cx = a > b;
        break;
      }
    }
  }
  const int64_t d = cx ? (int64_t)xa - xt : (int64_t)xt - xa;
  const uint32_t sx = cx ? sa : sc, sy = cx ? sc : sa;
  const bool sub = sx != sy;
  auto XW = [&](int m) -> uint32_t { return cx ? CW(m) : TW(m); };
  auto YW = [&](int m) -> uint32_t {
    if (m < 0 || m >= pw) return 0u;
    return cx ? TW(m) : CW(m);
  };
  auto YB = [&](int64_t pos) -> uint32_t {  // bits [pos, pos + 32) of Y's mantissa
    if (pos >= p || pos <= -32) return 0u;
    const int q = (int)(pos >> 5), r = (int)(pos & 31);
    const uint32_t lo = YW(q);
    return r ? (lo >> r) | (YW(q + 1) << (32 - r)) : lo;
  };
  // bits of Y below position d - 32 fall below the grid
  bool sticky = false;
  if (d > 32) {
    const int64_t nb = d - 32 < p ? d - 32 : p;
    const int full = (int)(nb >> 5), part = (int)(nb & 31);
    for (int k = 0; k < full && !sticky; ++k) sticky = YW(k) != 0u;
    if (!sticky && part) sticky = (YW(full) & ((1u << part) - 1u)) != 0u;
  }
  uint32_t *dcol = dw + ti;
  auto DAT = [&](int k) -> uint32_t & { return dcol[(int64_t)k * E]; };
  uint32_t cb = sub && sticky ? 1u : 0u;  // carry (add) or borrow (sub)
  for (int m = 0; m < nwd; ++m) {
    const uint32_t xg = (m >= 1 && m <= pw) ? XW(m - 1) : 0u;
    const uint32_t yg = YB((int64_t)32 * (m - 1) + d);
    if (!sub) {
      const uint64_t s = (uint64_t)xg + yg + cb;
      DAT(m) = (uint32_t)s;
      cb = (uint32_t)(s >> 32);
    } else {
      const uint64_t s = (uint64_t)xg - yg - cb;
      DAT(m) = (uint32_t)s;
      cb = (uint32_t)((s >> 63) & 1u);
    }
  }
  auto DM = [&](int k) -> uint32_t { return (k < 0 || k >= nwd) ? 0u : DAT(k); };
  const int32_t ex = cx ? xa : xt;
  round_to_limbs(DM, nwd, sticky, nlimb, (int64_t)ex - p - 32, sx, climb, planec, ci, cexp, csign);
}

__global__ void k_limb_zero(uint64_t *limb, int32_t *lexp, uint8_t *lsign, int64_t ld,
                            int64_t plane, int nlimb, int64_t M, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i >= M || j >= N) return;
  const int64_t idx = i + j * ld;
  for (int q = 0; q < nlimb; ++q) limb[(int64_t)q * plane + idx] = 0ull;
  lexp[idx] = EXP_ZERO;
  lsign[idx] = 0;
}

}  // namespace

namespace ozl {

hipError_t launch_limb_exponents(const uint64_t *limb, const int32_t *lexp, int64_t ld,
                                 int64_t plane, int nlimb, int64_t rows, int64_t cols,
                                 int rowwise, int32_t *e, hipStream_t s) {
  if (rowwise) {
    if (rows <= 0) return hipSuccess;
    hipError_t err = launch_fill_int(e, EXP_ZERO, rows, s);
    if (err != hipSuccess || cols <= 0) return err;
    dim3 g((unsigned)((rows + 255) / 256),
           (unsigned)((cols + LIMB_ROWEXP_CHUNK - 1) / LIMB_ROWEXP_CHUNK));
    hipLaunchKernelGGL(k_limb_row_exp, g, dim3(256), 0, s, limb, lexp, ld, plane, nlimb, rows,
                       cols, e);
  } else {
    if (cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_limb_col_exp, dim3((unsigned)((cols + 3) / 4)), dim3(256), 0, s, limb,
                       lexp, ld, plane, nlimb, rows, cols, e);
  }
  return hipGetLastError();
}

template <bool F64>
static void producer_limbs_nw(int nwt, dim3 g, hipStream_t s, const uint64_t *limb,
                              const int32_t *lexp, const uint8_t *lsign, int64_t ld,
                              int64_t plane, int nlimb, int rowwise, int64_t nout, int64_t K,
                              int64_t KB, const int32_t *exps, const DevPlan *pl, uint8_t *planes,
                              int64_t plane_elems) {
  if (nwt <= 4)
    hipLaunchKernelGGL((k_producer_limbs<4, F64>), g, dim3(256), 0, s, limb, lexp, lsign, ld,
                       plane, nlimb, rowwise, nout, K, KB, exps, pl, planes, plane_elems);
  else if (nwt <= 6)
    hipLaunchKernelGGL((k_producer_limbs<6, F64>), g, dim3(256), 0, s, limb, lexp, lsign, ld,
                       plane, nlimb, rowwise, nout, K, KB, exps, pl, planes, plane_elems);
  else
    hipLaunchKernelGGL((k_producer_limbs<REC_PWMAX, F64>), g, dim3(256), 0, s, limb, lexp, lsign,
                       ld, plane, nlimb, rowwise, nout, K, KB, exps, pl, planes, plane_elems);
}

hipError_t launch_producer_limbs(const uint64_t *limb, const int32_t *lexp, const uint8_t *lsign,
                                 int64_t ld, int64_t plane, int nlimb, int rowwise, int64_t nout,
                                 int64_t noutp, int64_t K, int64_t Kp, const int32_t *exps,
                                 const DevPlan *pl, int nmod, int nwt, int kind, void *planes,
                                 int64_t plane_elems, hipStream_t s) {
  const int64_t KB = Kp / 64, OB = noutp / 16;
  if (KB <= 0 || OB <= 0) return hipSuccess;
  if (plane_elems >= ((int64_t)1 << 31) || nwt > REC_PWMAX) return hipErrorInvalidValue;
  if (kind != PLANES_I8 && kind != PLANES_F64) return hipErrorInvalidValue;
  // split the moduli over up to 8 parts while the blocks alone give fewer
  // than 4096 wavefronts (four per SIMD)
  dim3 g((unsigned)KB, (unsigned)OB,
         (unsigned)std::max<int64_t>(1, std::min<int64_t>({8, (int64_t)nmod,
                                                            (4096 + 4 * KB * OB - 1) / (4 * KB * OB)})));
  if (kind == PLANES_F64)
    producer_limbs_nw<true>(nwt, g, s, limb, lexp, lsign, ld, plane, nlimb, rowwise, nout, K, KB,
                            exps, pl, (uint8_t *)planes, plane_elems);
  else
    producer_limbs_nw<false>(nwt, g, s, limb, lexp, lsign, ld, plane, nlimb, rowwise, nout, K, KB,
                             exps, pl, (uint8_t *)planes, plane_elems);
  return hipGetLastError();
}

hipError_t launch_consumer_limbs(const void *tpl, int tbytes, int64_t Mp, int64_t Np, int64_t M,
                                 int64_t N, const DevPlan *pl, int nd, int nvw, uint32_t *cw,
                                 hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 g((unsigned)((M + 255) / 256), (unsigned)N);
  const int ndc = nd <= 18 ? 18 : (nd <= 24 ? 24 : 32);
  if (nd > 32 || (tbytes == 1 && nd > 24) || (tbytes != 1 && tbytes != 4) ||
      nvw > ndc / 2 + 1)
    return hipErrorInvalidValue;
#define OZ_CONSL(ND_, TT_)                                                                       \
  hipLaunchKernelGGL((k_consumer_limbs<ND_, TT_>), g, dim3(256), 0, s, (const TT_ *)tpl, Mp, Np, \
                     M, N, pl, nvw, cw, M * N)
  if (tbytes == 1) {
    if (ndc == 18) OZ_CONSL(18, uint8_t);
    else OZ_CONSL(24, uint8_t);
  } else {
    if (ndc == 18) OZ_CONSL(18, uint32_t);
    else OZ_CONSL(32, uint32_t);
  }
#undef OZ_CONSL
  return hipGetLastError();
}

hipError_t launch_limb_round(const uint32_t *cw, int nwords, int64_t M, int64_t N,
                             const int32_t *ea, const int32_t *eb, int w, int g0, int Q, int nlimb,
                             uint64_t *olimb, int32_t *oexp, uint8_t *osign, int64_t ldo,
                             int64_t planeo, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 g((unsigned)((M + 255) / 256), (unsigned)N);
  hipLaunchKernelGGL(k_limb_round, g, dim3(256), 0, s, cw, M * N, nwords, M, N, ea, eb, w, g0, Q,
                     nlimb, olimb, oexp, osign, ldo, planeo);
  return hipGetLastError();
}

hipError_t launch_limb_sub(uint64_t *climb, int32_t *cexp, uint8_t *csign, int64_t ldc,
                           int64_t planec, const uint64_t *tlimb, const int32_t *texp,
                           const uint8_t *tsign, int nlimb, int64_t M, int64_t N, uint32_t *dw,
                           hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 g((unsigned)((M + 255) / 256), (unsigned)N);
  hipLaunchKernelGGL(k_limb_sub, g, dim3(256), 0, s, climb, cexp, csign, ldc, planec, tlimb, texp,
                     tsign, nlimb, M, N, dw, M * N);
  return hipGetLastError();
}

hipError_t launch_limb_zero(uint64_t *limb, int32_t *lexp, uint8_t *lsign, int64_t ld,
                            int64_t plane, int nlimb, int64_t M, int64_t N, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 g((unsigned)((M + 255) / 256), (unsigned)N);
  hipLaunchKernelGGL(k_limb_zero, g, dim3(256), 0, s, limb, lexp, lsign, ld, plane, nlimb, M, N);
  return hipGetLastError();
}

}  // namespace ozl
