// Per-element stages of the byte back-ends, shared by the grid kernels of
// one Ozaki-II product and by the batched LU, which runs the same stages
// inside one workgroup per system:
//   produce_block_b   (S2)+(S3): one 16-row x 64-k block of every residue
//                     plane, from expansions (Eq. direct, Sec. 3.2 slicing);
//   mod_times_y       (S4) epilogue: t = ((C mod m) y) mod m, Eq. (crt);
//   consume_element_b (S5)+(S6): CRT of every retained digit group, exact
//                     group sum, one greedy rounding.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ozii_bytes.hpp"
#include "ozii_elem.hpp"

namespace ozk {

// Plane encodings of the three back-ends of (S3)/(S4).
enum { PL_I8 = 0, PL_F8 = 1, PL_F64 = 2 };

// Producer of the byte back-ends (INT8 residues, FP8 base-17 digits): the
// caller's threads fill block (ob, kb) -- rows 16 ob .. 16 ob + 15, inner
// indices 64 kb .. 64 kb + 63 -- of every plane.  EPT = 4: 256 threads,
// thread T owns the four consecutive bytes 4T .. 4T+3 of the block, i.e. row
// (T/4)%16 and inner indices 16(T/64) + 4(T%4) + e, e = 0..3, so each
// residue plane receives one dword store per thread; EPT = 1 (for small
// products: a quarter of the conversion and slicing per thread): 1024
// threads, thread T owns byte T (of the moduli l0 ..
// l1-1: small products split the moduli over several workgroups).  Rows at
// or past nout and inner indices at or past K are zero.
template <int NWX>
__device__ __forceinline__ uint32_t word_or_fill(const uint32_t (&X)[NWX], int k, uint32_t fill) {
  uint32_t r = fill;
#pragma unroll
  for (int i = 0; i < NWX; ++i) r = k == i ? X[i] : r;
  return r;
}

template <int NC, int NWX, int NWM, int PL, int EPT = 4>
__device__ __forceinline__ void produce_block_b(const double *__restrict__ X, int64_t ld,
                                                int rowwise, int64_t nout, int64_t K, int64_t KB,
                                                const int32_t *__restrict__ exps,
                                                const DevPlan *__restrict__ pl,
                                                uint8_t *__restrict__ planes,
                                                int64_t plane_elems, int64_t kb, int64_t ob,
                                                int T, int l0, int l1) {
  // block byte E0 .. E0 + EPT - 1: byte E is row (E/16)%16, inner index
  // 16(E/256) + 4((E/4)%4) + E%4 of the block
  const int E0 = EPT * T;
  const int64_t o = ob * 16 + ((E0 >> 4) & 15);
  const int64_t h0 = kb * 64 + 16 * (E0 >> 8) + 4 * ((E0 >> 2) & 3) + (E0 & 3);
  // index of this thread's bytes in every plane (planes hold fewer than
  // 2^31 elements)
  const uint32_t offb = (uint32_t)((ob * KB + kb) * 1024 + E0);  // < 2^31
  const int S = pl->S, w = pl->w, nmod = pl->nmod, Q = pl->Q, nwt = pl->nwt;

  uint32_t Xw[EPT][NWX];
  int32_t ex = EXP_ZERO;
  if (o < nout) ex = exps[o];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int64_t h = h0 + e;
    const double *src = nullptr;
    if (ex != EXP_ZERO && h < K) src = rowwise ? X + (o + h * ld) * NC : X + (h + o * ld) * NC;
    if (src) {
      to_fixed<NC, NWX>(src, Q - 1 - ex, Xw[e]);
    } else {
#pragma unroll
      for (int k = 0; k < NWX; ++k) Xw[e][k] = 0u;
    }
  }
  uint32_t cin[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) cin[e] = 0u;
  for (int t = 0; t < S; ++t) {
    const bool top = t == S - 1;
    const int bo = t * w, q = bo >> 5, b = bo & 31;
    const int wq = w >> 5, wb = w & 31;
    uint32_t F[EPT][NWM];
    uint32_t sel[EPT];  // 1: add the (-2^W) mod m term (flag or sign)
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const uint32_t fill = (Xw[e][NWX - 1] >> 31) ? 0xffffffffu : 0u;
      uint32_t prev = word_or_fill<NWX>(Xw[e], q, fill);
#pragma unroll
      for (int j = 0; j < NWM; ++j) {
        const uint32_t nxt = word_or_fill<NWX>(Xw[e], q + j + 1, fill);
        F[e][j] = __builtin_amdgcn_alignbit(nxt, prev, b);
        prev = nxt;
      }
      if (!top) {
        // keep the w-bit field
#pragma unroll
        for (int j = 0; j < NWM; ++j)
          F[e][j] = j < wq ? F[e][j] : (j == wq ? F[e][j] & ((1u << wb) - 1u) : 0u);
      }
      // add the incoming carry
      uint32_t c = cin[e];
#pragma unroll
      for (int j = 0; j < NWM; ++j) {
        const uint32_t sum = F[e][j] + c;
        c = sum < c ? 1u : 0u;
        F[e][j] = sum;
      }
      if (!top) {
        // carry out of the field (bit w, inside the window since 32 nwt > w)
        // and the centring flag (bit w-1)
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
    const int pstep = PL == PL_F8 ? 2 : 1;
    emit_byte_residues<NWM, PL == PL_F8, EPT>(F, sel, top ? REC_HT : REC_HW, pl, l0, l1,
                                         planes + ((int64_t)t * nmod + l0) * pstep * plane_elems,
                                         plane_elems, offb);
  }
}

// (S4) epilogue: t = ((c mod m) y) mod m in [0, m) for any int32 c, y < m
// <= 256.  x = c y is exact in binary64 (< 2^39); floor(x * RN(1/m)) is floor(x/m) unless x/m is an
// integer, when it may be one less (the rounding error, < 2^-17, is far
// below the 1/m distance of any other quotient to an integer), so the
// remainder is in [0, m] and the single wrap m -> 0 is an unsigned min.
__device__ __forceinline__ uint32_t mod_times_y(int32_t c, double md, double yd, double im,
                                                uint32_t m) {
  const double x = (double)c * yd;
  const double q = __builtin_floor(x * im);
  const uint32_t r = (uint32_t)__builtin_fma(-q, md, x);
  const uint32_t rm = r - m;
  return r < rm ? r : rm;
}

// Consumer of the byte back-ends, one element: per digit group gi the CRT of
// crt_group_bytes over the t-bytes at tbase + (gi nmod + l) ps (modulus l),
// the group added at bit w gi to the exact group sum, which is rounded once
// to NC components of value sum 2^eps (zero: all components 0).  st: STG
// words of thread-private scratch; PRE: see crt_group_bytes.
template <int NC, int NWC, int NB, int PRE = 0, int STG = CST>
__device__ __forceinline__ void consume_element_b(const uint8_t *tbase, int64_t ps,
                                                  const DevPlan *__restrict__ pl, uint32_t *st,
                                                  bool zero, int eps, double (&c)[NC]) {
  static_assert(NB % 4 == 0 && NB <= CRT4_NB, "byte columns");
  constexpr int ND = NB / 2;
  const int nmod = pl->nmod, w = pl->w, ng = pl->ng;
  uint32_t cb[NWC];
#pragma unroll
  for (int k = 0; k < NWC; ++k) cb[k] = 0u;
  for (int gi = 0; gi < ng; ++gi) {
    int32_t d[ND];
    crt_group_bytes<NB, PRE>(tbase + (int64_t)gi * nmod * ps, ps, nmod, pl, d);
    add_shifted_digits<NWC, ND, STG>(cb, d, w * gi, st);
  }
  if (zero) {
#pragma unroll
    for (int qq = 0; qq < NC; ++qq) c[qq] = 0.0;
  } else {
    round_out_n<NWC, NC>(cb, eps, c);
  }
}

// ---------------------------------------------------------------------------
// (S5)+(S6) consumer of the byte back-ends with the CRT's column sums on the
// matrix cores.  One wavefront (a workgroup of its own) takes 64 consecutive
// elements of a column.  Per digit group the t-bytes of its elements go to
// LDS one element row at a time (t - 128 as signed bytes); four 16-element
// blocks of them are the B operands of v_mfma_i32_16x16x64_i8 against the
// plan's column table (DevPlan::crtm, three A operands held in registers:
// f_l and the 46 bytes that M_l < 2^363 can have), which gives
// sum_l (t_l - 128) b_jl for every table column j.  Through LDS, 32 elements
// at a time, each lane collects its own element's columns, adds crtc, and
// forms the 16-bit digits of Sbar as crt_group_bytes does (the same exact
// integer, so the same digits).  The group shift, rounding and update are
// those of consume_element_b.  6.5 KiB of LDS per wavefront.  WAVE: the
// wavefront works on its own buffer inside a larger workgroup (the batched
// LU), so its steps are ordered by a wavefront barrier instead of the
// workgroup's.
// ---------------------------------------------------------------------------
typedef int mxv4 __attribute__((ext_vector_type(4)));
constexpr int MX_TBS = 80;   // bytes per element row of the t-bytes (conflict-free reads)
constexpr int MX_BLK = 3;    // 16-column blocks of the table: f_l, then bytes 0..45 of M_l
constexpr int MX_CBS = 16 * MX_BLK + 4;  // ints per element row of the column sums
static_assert(2 + 46 == 16 * MX_BLK, "table columns");

template <bool WAVE>
__device__ __forceinline__ void mx_sync() {
  if (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// The 16-bit digits of group gi's Sbar for the wavefront's 64 elements
// (lane L: element i0 + L) by the matrix-core route; tg: t-value of modulus 0
// of element i0 in group gi, moduli ps bytes apart.  Called by all 64 lanes
// of a one-wavefront workgroup (or, WAVE, of one wavefront on its own buf);
// buf (32 MX_CBS ints of LDS) is free again when it returns.
template <int NB, bool WAVE = false>
__device__ __forceinline__ void crt_group_mx(const uint8_t *tg, int64_t ps, int nmod,
                                             const DevPlan *__restrict__ pl,
                                             const mxv4 (&tab)[MX_BLK], int32_t *buf, int lane,
                                             int32_t (&d)[NB / 2]) {
  constexpr int ND = NB / 2;
  uint8_t *tb = (uint8_t *)buf;
  const int nch = (nmod + 3) >> 2;
  const int e4 = 4 * (lane & 15), lq = lane >> 4;
  // lane: moduli 4c + lq, elements e4 .. e4 + 3 (one dword of a plane);
  // moduli past nmod read the last plane again, their table columns are 0
  const uint8_t *src = tg + e4 + (int64_t)lq * ps, *last = tg + e4 + (int64_t)(nmod - 1) * ps;
  for (int c = 0; c < nch; ++c, src += 4 * ps) {
    const int l = 4 * c + lq;
    const uint32_t v = *(const uint32_t *)(l < nmod ? src : last) ^ 0x80808080u;
#pragma unroll
    for (int r = 0; r < 4; ++r) tb[(e4 + r) * MX_TBS + l] = (uint8_t)(v >> (8 * r));
  }
  mx_sync<WAVE>();
  mxv4 bf[4];
#pragma unroll
  for (int e = 0; e < 4; ++e)
    bf[e] = *(const mxv4 *)(tb + (16 * e + (lane & 15)) * MX_TBS + 16 * lq);
  mx_sync<WAVE>();
  int32_t col[52];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int e = 2 * h; e < 2 * h + 2; ++e)
#pragma unroll
      for (int b = 0; b < MX_BLK; ++b) {
        const mxv4 acc =
            __builtin_amdgcn_mfma_i32_16x16x64_i8(tab[b], bf[e], mxv4{0, 0, 0, 0}, 0, 0, 0);
        *(mxv4 *)(buf + (16 * (e - 2 * h) + (lane & 15)) * MX_CBS + 16 * b + 4 * lq) = acc;
      }
    mx_sync<WAVE>();
    if ((lane >> 5) == h) {
#pragma unroll
      for (int q = 0; q < 4 * MX_BLK; ++q) {
        const mxv4 v = *(const mxv4 *)(buf + (lane & 31) * MX_CBS + 4 * q);
#pragma unroll
        for (int r = 0; r < 4; ++r) col[4 * q + r] = v[r] + pl->crtc[4 * q + r];
      }
    }
    mx_sync<WAVE>();
  }
#pragma unroll
  for (int k = 16 * MX_BLK; k < 52; ++k) col[k] = 0;  // bytes 46, 47 of every M_l are 0
  // F = (sum_l t_l f_l) / 2^16 from columns 0, 1; then as crt_group_bytes
  const int32_t qf = (col[0] + col[1] * 256 + 32768) >> 16;
  int32_t carry = 0;
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    const int32_t lo = col[2 + 2 * k] - qf * (pl->pbyte[2 * k] & 0xff);
    const int32_t hi = col[3 + 2 * k] - qf * (pl->pbyte[2 * k + 1] & 0xff);
    const int32_t v = lo + (int32_t)((uint32_t)hi << 8) + carry;
    d[k] = v & 0xffff;
    carry = v >> 16;  // arithmetic
  }
  d[ND - 1] = (int32_t)(int16_t)(uint16_t)d[ND - 1];
}

}  // namespace ozk
