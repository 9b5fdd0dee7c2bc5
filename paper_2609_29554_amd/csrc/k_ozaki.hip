// Ozaki-II product kernels for gfx950 (Sec. 3.1-3.3 of the paper):
//   (S1) row / column exponents,
//   (S2)+(S3) producer: expansion -> fixed point -> balanced slices ->
//        centred int8 residues, written in MFMA-fragment order,
//   (S4) one batched INT8 MFMA launch over every (digit group, modulus, tile)
//        with the t_l = ((C mod m) y) mod m epilogue of Eq. (crt),
//   (S5)+(S6) consumer: CRT per digit group, exact accumulation of the
//        groups, one greedy rounding, and the update C -= A B.
//
// Residue plane layout ("fragment order"): a plane is a grid of 16 x 64-byte
// blocks; block (ob, kb) of a plane holds rows ob*16 .. ob*16+15 and inner
// indices kb*64 .. kb*64+63; inside a block, lane l of a wavefront owns the
// 16 contiguous bytes at l*16: row l%16, inner indices 16*(l/16) .. +15.
// One 16-byte load per lane therefore fetches a whole MFMA operand fragment.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "expansion.hpp"
#include "ozii_elem.hpp"
#include "ozii_bytes.hpp"
#include "ozii_kernels.hpp"
#include "ozii_stage.hpp"

using namespace ozk;

typedef int v4i __attribute__((ext_vector_type(4)));

namespace {

// ---------------------------------------------------------------------------
// (S1) exponents
// ---------------------------------------------------------------------------
// Row maxima: a 2-D grid, each thread scans a chunk of one row and the chunk
// maxima meet in e[i] through an atomic max (e pre-filled with EXP_ZERO).
constexpr int ROWEXP_CHUNK = 16;
template <int NC>
__global__ __launch_bounds__(256) void k_row_exponents(const double *A, int64_t lda, int64_t rows,
                                                       int64_t cols, int32_t *e) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= rows) return;
  const int64_t h0 = (int64_t)blockIdx.y * ROWEXP_CHUNK;
  const int64_t h1 = h0 + ROWEXP_CHUNK < cols ? h0 + ROWEXP_CHUNK : cols;
  int32_t best = EXP_ZERO;
  for (int64_t h = h0; h < h1; ++h) {
    int32_t v = exponent_of<NC>(A + (i + h * lda) * NC);
    best = v > best ? v : best;
  }
  if (best != EXP_ZERO) atomicMax(e + i, best);
}

// C = 0 for an M x N matrix of nc-component expansions (leading dimension
// ldc), one double per thread
__global__ __launch_bounds__(256) void k_zero_expansions(double *C, int64_t ldc, int64_t rows,
                                                         int64_t cols, int nc) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t per = rows * nc;
  if (t >= per * cols) return;
  const int64_t j = t / per, r = t - j * per;
  C[j * ldc * nc + r] = 0.0;
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t cnt) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < cnt) p[t] = v;
}

template <int NC>
__global__ __launch_bounds__(256) void k_col_exponents(const double *B, int64_t ldb, int64_t rows,
                                                       int64_t cols, int32_t *e) {
  const int lane = threadIdx.x & 63;
  int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= cols) return;
  int32_t best = EXP_ZERO;
  for (int64_t h = lane; h < rows; h += 64) {
    int32_t v = exponent_of<NC>(B + (h + j * ldb) * NC);
    best = v > best ? v : best;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    int32_t o = __shfl_xor(best, off, 64);
    best = o > best ? o : best;
  }
  if (lane == 0) e[j] = best;
}

// ---------------------------------------------------------------------------
// (S2)+(S3) producer
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// Producer of the byte back-ends (INT8 residues, FP8 base-17 digits).  One
// workgroup fills one 1 KiB block (16 rows x 64 k) of every plane; thread T
// owns the four consecutive bytes 4T .. 4T+3 of the block, i.e. row
// (T/4)%16 and inner indices 16(T/64) + 4(T%4) + e, e = 0..3, so each
// residue plane receives one dword store per thread.
//
// Per element: X = sum_c sgn(x_c) floor(|x_c| 2^mu) (Eq. direct) in NWX
// words; slice t of the balanced split (Sec. 3.2) is read straight from X as
// the w-bit field at bit t w plus the incoming carry c_t:
//   s = field + c_t;  carry = s >> w;  s mod= 2^w;  f = bit w-1 of s;
//   v_t = s - f 2^w;  c_{t+1} = carry + f,
// and the top slice is v = (X >> (S-1) w) + c_{S-1}, taken as a two's
// complement number of nwt words.  Its residue for modulus m is
//   (sum_b byte_b (2^(8b) mod m) + [f or sign] ((-2^W) mod m)) mod m,
// W = w or 32 nwt, where the byte sum is v_dot4_u32_u8 of the slice words
// with the table words (operands in scalar registers).  With h = floor(m/2)
// added first, the centred residue is acc - floor(acc/m) m - h, and
// floor(acc/m) is exact as the high word of (acc << k) * ceil(2^(32-k)/m):
// acc < 2^(32-k)/m and (acc << k) < 2^24 hold for w <= 300.
// ---------------------------------------------------------------------------
template <int NC, int NWX, int NWM, int PL, int EPT>
__global__ __launch_bounds__(256) void k_producer_b(const double *__restrict__ X, int64_t ld,
                                                    int rowwise, int64_t nout, int64_t K,
                                                    int64_t KB, const int32_t *__restrict__ exps,
                                                    const DevPlan *__restrict__ pl,
                                                    uint8_t *__restrict__ planes,
                                                    int64_t plane_elems) {
  // blockIdx.z: a part of the moduli (small products run several parts to
  // fill the chip; each part repeats the conversion and slicing).  EPT = 1:
  // four workgroups per block, blockIdx.x = 4 kb + quarter.
  const int nmod = pl->nmod, np = (int)gridDim.z, part = (int)blockIdx.z;
  const int64_t kb = EPT == 4 ? (int64_t)blockIdx.x : (int64_t)(blockIdx.x >> 2);
  const int T = EPT == 4 ? (int)threadIdx.x : (int)(((blockIdx.x & 3u) << 8) + threadIdx.x);
  produce_block_b<NC, NWX, NWM, PL, EPT>(X, ld, rowwise, nout, K, KB, exps, pl, planes,
                                         plane_elems, kb, blockIdx.y, T, part * nmod / np,
                                         (part + 1) * nmod / np);
}

// Producer: one workgroup fills one 16-row x 64-k window of every plane.
//   PL_I8 : int8 residues, 1 KiB blocks of 16 rows x 64 k (lane l: row l%16,
//           k 16(l/16) .. +16);
//   PL_F8 : the balanced base-17 digits d0, d1 of every residue (Eq.
//           fp8digits) as E4M3 bytes, two planes per (slice, modulus), same
//           blocks;
//   PL_F64: residues as doubles, 1 KiB blocks of 16 rows x 8 k (lane l: row
//           l%16, k l/16 and 4 + l/16), eight blocks per window.
template <int NC, int NWX, int NH, int PL>
__global__ __launch_bounds__(256) void k_producer(const double *X, int64_t ld, int rowwise,
                                                  int64_t nout, int64_t K, int64_t KB,
                                                  const int32_t *exps, const DevPlan *pl,
                                                  void *planes, int64_t plane_elems) {
  __shared__ uint32_t stage[256 * STG];
  uint32_t *st = stage + threadIdx.x * STG;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t kb = blockIdx.x, ob = blockIdx.y;
  const int nmod = pl->nmod, Q = pl->Q;
  for (int q = 0; q < 4; ++q) {
    int64_t o, h, off;
    if (PL == PL_F64) {
      // output order: consecutive threads write consecutive doubles
      const int E = q * 256 + (int)threadIdx.x;
      const int fb = E >> 7, L = (E >> 1) & 63, slot = E & 1;
      o = ob * 16 + (L & 15);
      h = kb * 64 + fb * 8 + (L >> 4) + 4 * slot;
      off = ((ob * KB + kb) * 8 + fb) * 128 + (E & 127);
    } else {
      o = ob * 16 + 4 * q + (lane >> 4);
      h = kb * 64 + 16 * wv + (lane & 15);
      off = (ob * KB + kb) * 1024 + 64 * q + 256 * wv + lane;
    }
    const double *src = nullptr;
    int mu = 0;
    if (o < nout && h < K) {
      const int32_t ex = exps[o];
      if (ex != EXP_ZERO) {
        src = rowwise ? X + (o + h * ld) * NC : X + (h + o * ld) * NC;
        mu = Q - 1 - ex;
      }
    }
    produce_element<NC, NWX, NH, PL == PL_F64>(src, mu, pl, st, [&](int t, int l, int32_t r) {
      const int64_t pi = (int64_t)(t * nmod + l);
      if (PL == PL_I8) {
        ((int8_t *)planes)[pi * plane_elems + off] = (int8_t)r;
      } else if (PL == PL_F8) {
        const int32_t d1 = (int32_t)__builtin_rintf((float)r * (1.0f / 17.0f));
        const int32_t d0 = r - 17 * d1;
        ((uint8_t *)planes)[(2 * pi) * plane_elems + off] = e4m3_small(d0);
        ((uint8_t *)planes)[(2 * pi + 1) * plane_elems + off] = e4m3_small(d1);
      } else {
        ((double *)planes)[pi * plane_elems + off] = (double)r;
      }
    });
  }
}

// ---------------------------------------------------------------------------
// (S4) batched INT8 GEMM: one workgroup = one 128x128 tile of one
// (group, modulus) product; four wavefronts in 2x2, each 64x64 = 4x4 MFMA
// 16x16x64 fragments.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gemm_i8(const int8_t *__restrict__ pa,
                                                 const int8_t *__restrict__ pb,
                                                 uint8_t *__restrict__ tpl, const DevPlan *pl,
                                                 int64_t Mp, int64_t Np, int64_t KB,
                                                 int64_t planeA, int64_t planeB, int tilesM,
                                                 int tilesN) {
  constexpr int LDT = 144;  // bytes per column of the output staging tile
  __shared__ __attribute__((aligned(16))) uint8_t tile[128 * LDT];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  // XCD-aware remap: the hardware deals consecutive workgroups round-robin to
  // 8 XCDs; give each XCD a contiguous range of logical tiles so that the
  // tiles of one (group, modulus) product share an L2.
  const int nb = gridDim.x, pid = blockIdx.x;
  const int xcd = pid & 7, loc = pid >> 3;
  const int qd = nb >> 3, rm = nb & 7;
  const int lt = (xcd < rm ? xcd * (qd + 1) : rm * (qd + 1) + (xcd - rm) * qd) + loc;
  const int tn = lt % tilesN;
  const int tm = (lt / tilesN) % tilesM;
  const int pr = lt / (tilesN * tilesM);
  const int nmod = pl->nmod;
  // products in modulus-major order: neighbouring groups of one modulus share
  // most of their slice planes; gl is the product's t-plane
  const int gi = pr % pl->ng, l = pr / pl->ng;
  const int gl = gi * nmod + l;
  const int S = pl->S, g = pl->g0 + gi;
  const int ta0 = g - (S - 1) > 0 ? g - (S - 1) : 0;
  const int ta1 = g < S - 1 ? g : S - 1;

  v4i acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = v4i{0, 0, 0, 0};

  for (int ta = ta0; ta <= ta1; ++ta) {
    const int tb = g - ta;
    const int8_t *A0 = pa + (int64_t)(ta * nmod + l) * planeA +
                       ((int64_t)(tm * 8 + wm * 4) * KB) * 1024 + lane * 16;
    const int8_t *B0 = pb + (int64_t)(tb * nmod + l) * planeB +
                       ((int64_t)(tn * 8 + wn * 4) * KB) * 1024 + lane * 16;
    v4i af[4], bf[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) af[a] = *(const v4i *)(A0 + (int64_t)a * KB * 1024);
#pragma unroll
    for (int b = 0; b < 4; ++b) bf[b] = *(const v4i *)(B0 + (int64_t)b * KB * 1024);
    for (int64_t kb = 0; kb < KB; ++kb) {
      v4i an[4], bn[4];
      const bool more = kb + 1 < KB;
      if (more) {
#pragma unroll
        for (int a = 0; a < 4; ++a) an[a] = *(const v4i *)(A0 + ((int64_t)a * KB + kb + 1) * 1024);
#pragma unroll
        for (int b = 0; b < 4; ++b) bn[b] = *(const v4i *)(B0 + ((int64_t)b * KB + kb + 1) * 1024);
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[a], bf[b], acc[a][b], 0, 0, 0);
      if (more) {
#pragma unroll
        for (int a = 0; a < 4; ++a) af[a] = an[a];
#pragma unroll
        for (int b = 0; b < 4; ++b) bf[b] = bn[b];
      }
    }
  }
  // epilogue: t = ((C mod m) y) mod m, one byte, staged through LDS so that
  // the column-major t-plane is written with contiguous 64-byte runs
  const uint32_t m = (uint32_t)pl->m[l];
  const double md = (double)m, yd = (double)pl->y[l], im = pl->inv_m[l];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      uint32_t packed = 0;
#pragma unroll
      for (int r = 0; r < 4; ++r) packed |= mod_times_y(acc[a][b][r], md, yd, im, m) << (8 * r);
      const int row = wm * 64 + 16 * a + 4 * (lane >> 4);
      const int col = wn * 64 + 16 * b + (lane & 15);
      *(uint32_t *)(tile + col * LDT + row) = packed;
    }
  }
  __syncthreads();
  {
    const int col = threadIdx.x >> 1, half = threadIdx.x & 1;
    const uint4 *src = (const uint4 *)(tile + col * LDT + half * 64);
    uint4 *dst = (uint4 *)(tpl + ((int64_t)gl * Np + (int64_t)tn * 128 + col) * Mp +
                           (int64_t)tm * 128 + half * 64);
#pragma unroll
    for (int k = 0; k < 4; ++k) dst[k] = src[k];
  }
}

// ---------------------------------------------------------------------------
// (S4), pipelined large tiles: one workgroup = one (128 WMW) x (64 WNW)
// tile of one (group, modulus) product, WMW x WNW wavefronts of 128x64
// (8x4 MFMA 16x16x64 fragments each).  Operand blocks move from global
// memory straight into LDS (global_load_lds, 16 bytes per lane: a 1 KiB
// fragment block lands as one wavefront instruction, in the order the MFMA
// reads it), NS stages deep, so up to NS-1 inner steps of loads are in flight
// without holding registers.  Each wavefront reads its 12 fragments of the
// next step from LDS while its MFMAs run on the current ones.
// ---------------------------------------------------------------------------
namespace {
constexpr int GL_LDT = 272;  // output staging column stride (256 rows + pad)
constexpr int GL_GM = 4;     // tile rows per raster group

typedef __attribute__((address_space(3))) void lds_void;

__device__ __forceinline__ void gl_to_lds(const int8_t *g, uint8_t *l) {
  __builtin_amdgcn_global_load_lds((const void *)g, (lds_void *)l, 16, 0, 0);
}

// wait until at most n*LPW of this wavefront's global->LDS loads are pending
template <int LPW>
__device__ __forceinline__ void gl_wait_pending(int n) {
  // s_waitcnt immediate: vmcnt[3:0] | expcnt 7 << 4 | lgkmcnt 15 << 8 | vmcnt[5:4] << 14
#define OZ_VMCNT(N) ((((N) & 15) | (7 << 4) | (15 << 8) | (((N) >> 4) << 14)))
  switch (n) {
    case 0: __builtin_amdgcn_s_waitcnt(OZ_VMCNT(0)); break;
    case 1: __builtin_amdgcn_s_waitcnt(OZ_VMCNT(1 * LPW)); break;
    case 2: __builtin_amdgcn_s_waitcnt(OZ_VMCNT(2 * LPW)); break;
    case 3: __builtin_amdgcn_s_waitcnt(OZ_VMCNT(3 * LPW)); break;
    default: __builtin_amdgcn_s_waitcnt(OZ_VMCNT(4 * LPW)); break;
  }
#undef OZ_VMCNT
}

// Workgroup barrier for the operand pipeline: this wavefront's LDS reads have
// returned (a wait the compiler sees, so it adds none of its own before the
// next MFMAs), then s_barrier.  The memory clobber keeps the compiler from
// moving LDS accesses across it; the global->LDS loads are waited for
// explicitly (gl_wait_pending), not by a blanket vmcnt(0) at every barrier.
__device__ __forceinline__ void gl_barrier() {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0), vmcnt and expcnt unconstrained
  asm volatile("s_barrier" ::: "memory");
}

}  // namespace

template <int WMW, int WNW, int NS>
__global__ __launch_bounds__(64 * WMW * WNW) void k_gemm_i8_p(
    const int8_t *__restrict__ pa, const int8_t *__restrict__ pb, uint8_t *__restrict__ tpl,
    const DevPlan *pl, int64_t Mp, int64_t Np, int64_t KB, int64_t planeA, int64_t planeB,
    int tilesM, int tilesN) {
  constexpr int NW = WMW * WNW, NT = 64 * NW;
  constexpr int NAB = 8 * WMW, NBB = 4 * WNW;  // 1 KiB blocks of A, B per stage
  constexpr int STAGE = (NAB + NBB) * 1024;
  constexpr int LPW = (NAB + NBB) / NW;        // global->LDS loads per wavefront per stage
  constexpr int LPA = NAB / NW;                // of which A blocks
  constexpr int TR = 128 * WMW, TC = 64 * WNW; // tile rows, columns
  static_assert(NAB % NW == 0 && NBB % NW == 0, "blocks must split evenly over wavefronts");
  static_assert(TR + 16 <= GL_LDT, "staging column stride");
  static_assert(NS * STAGE >= TC * GL_LDT, "output staging must fit the operand buffers");
  static_assert(NS >= 3 && NS <= 6, "wait table covers 0..4 stages in flight");
  static_assert(NT == 2 * TC, "output copy: two threads per tile column");
  __shared__ __attribute__((aligned(1024))) uint8_t lds[NS * STAGE];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv / WNW, wn = wv % WNW;
  // XCD-aware remap (as in k_gemm_i8), then a grouped raster inside each
  // product: consecutive logical tiles sweep GL_GM tile rows before moving to
  // the next tile column, so the tiles running together on one XCD share
  // few A and B panels in its L2.
  const int nb = gridDim.x, pid = blockIdx.x;
  const int xcd = pid & 7, loc = pid >> 3;
  const int qd = nb >> 3, rm = nb & 7;
  const int lt = (xcd < rm ? xcd * (qd + 1) : rm * (qd + 1) + (xcd - rm) * qd) + loc;
  const int per = tilesM * tilesN;
  const int pr = lt / per, r = lt - pr * per;
  const int grp = r / (GL_GM * tilesN), r2 = r - grp * (GL_GM * tilesN);
  const int tm0 = grp * GL_GM;
  const int gh = tilesM - tm0 < GL_GM ? tilesM - tm0 : GL_GM;
  const int tm = tm0 + r2 % gh, tn = r2 / gh;
  const int nmod = pl->nmod;
  // products in modulus-major order: neighbouring groups of one modulus share
  // most of their slice planes; gl is the product's t-plane
  const int gi = pr % pl->ng, l = pr / pl->ng;
  const int gl = gi * nmod + l;
  const int S = pl->S, g = pl->g0 + gi;
  const int ta0 = g - (S - 1) > 0 ? g - (S - 1) : 0;
  const int ta1 = g < S - 1 ? g : S - 1;
  const int nst = (ta1 - ta0 + 1) * (int)KB;

  // Wavefront wv loads blocks c NW + wv (c < LPW) of a stage: A blocks first,
  // then B blocks; lane l moves bytes [16 l, 16 l + 16) of each.
  const int64_t lo16 = (int64_t)lane * 16;
  int64_t off[LPW];
#pragma unroll
  for (int c = 0; c < LPW; ++c) {
    const int bi = c * NW + wv;
    off[c] = c < LPA ? (int64_t)(tm * NAB + bi) * KB * 1024 + lo16
                     : (int64_t)(tn * NBB + bi - NAB) * KB * 1024 + lo16;
  }

  v4i acc[8][4];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = v4i{0, 0, 0, 0};

  const int KBi = (int)KB;
  int f_ta = ta0, f_kb = 0;  // position of the next stage to load
#define OZ_ISSUE(BUF)                                                                          \
  do {                                                                                         \
    const int8_t *A0_ = pa + (int64_t)(f_ta * nmod + l) * planeA + (int64_t)f_kb * 1024;       \
    const int8_t *B0_ = pb + (int64_t)((g - f_ta) * nmod + l) * planeB + (int64_t)f_kb * 1024; \
    uint8_t *D_ = lds + (BUF) * STAGE + wv * 1024;                                             \
    _Pragma("unroll") for (int c_ = 0; c_ < LPW; ++c_)                                         \
      gl_to_lds((c_ < LPA ? A0_ : B0_) + off[c_], D_ + c_ * NW * 1024);                        \
    if (++f_kb == KBi) {                                                                       \
      f_kb = 0;                                                                                \
      ++f_ta;                                                                                  \
    }                                                                                          \
  } while (0)
#define OZ_READ(BUF, AF, BF)                                                                   \
  do {                                                                                         \
    const uint8_t *S_ = lds + (BUF) * STAGE + lo16;                                            \
    _Pragma("unroll") for (int b_ = 0; b_ < 4; ++b_)                                           \
      BF[b_] = *(const v4i *)(S_ + (NAB + wn * 4 + b_) * 1024);                                \
    _Pragma("unroll") for (int a_ = 0; a_ < 8; ++a_)                                           \
      AF[a_] = *(const v4i *)(S_ + (wm * 8 + a_) * 1024);                                      \
  } while (0)
  // Step st computes from CA/CB (stage st, read during step st-1).  First it
  // waits for its own loads of stage st+1 and meets the other wavefronts at
  // the barrier: stage st+1 has then landed, and every wavefront has read
  // stage st out of LDS, so stage st+NS can go into that buffer.
#define OZ_STEP(ST, CA, CB, NA, NB)                                                            \
  do {                                                                                         \
    const int nxt_ = (ST) + 1;                                                                 \
    if (nxt_ < nst) {                                                                          \
      const int ahead_ = nst - 1 - nxt_;                                                       \
      gl_wait_pending<LPW>(ahead_ < NS - 2 ? ahead_ : NS - 2);                                 \
    }                                                                                          \
    gl_barrier();                                                                              \
    if ((ST) + NS < nst) OZ_ISSUE(buf);                                                        \
    buf = buf == NS - 1 ? 0 : buf + 1;                                                         \
    if (nxt_ < nst) OZ_READ(buf, NA, NB);                                                      \
    _Pragma("unroll") for (int a = 0; a < 8; ++a)                                              \
      _Pragma("unroll") for (int b = 0; b < 4; ++b)                                            \
        acc[a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(CA[a], CB[b], acc[a][b], 0, 0, 0);   \
  } while (0)

  const int pro = nst < NS ? nst : NS;
  for (int s = 0; s < pro; ++s) OZ_ISSUE(s);
  gl_wait_pending<LPW>(pro - 1);
  gl_barrier();
  int buf = 0;  // buffer of the stage being computed
  v4i xa[8], xb[4], ya[8], yb[4];
  OZ_READ(0, xa, xb);
  // pairs of steps that both have a following stage, then one or two steps
  // with the fragments of the last one in xa/xb
  int st = 0;
  for (; st + 2 < nst; st += 2) {
    OZ_STEP(st, xa, xb, ya, yb);
    OZ_STEP(st + 1, ya, yb, xa, xb);
  }
  if (st + 1 < nst) {
    OZ_STEP(st, xa, xb, ya, yb);
#pragma unroll
    for (int a = 0; a < 8; ++a) xa[a] = ya[a];
#pragma unroll
    for (int b = 0; b < 4; ++b) xb[b] = yb[b];
  }
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
      acc[a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(xa[a], xb[b], acc[a][b], 0, 0, 0);
#undef OZ_STEP
#undef OZ_ISSUE
#undef OZ_READ
  gl_barrier();  // operand buffers are reused for the output staging tile
  // epilogue: t = ((C mod m) y) mod m staged through LDS as a TC-column x
  // TR-row byte tile, then written as 128-byte runs of the t-plane
  const uint32_t m = (uint32_t)pl->m[l];
  const double md = (double)m, yd = (double)pl->y[l], im = pl->inv_m[l];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      uint32_t packed = 0;
#pragma unroll
      for (int r = 0; r < 4; ++r) packed |= mod_times_y(acc[a][b][r], md, yd, im, m) << (8 * r);
      const int row = wm * 128 + 16 * a + 4 * (lane >> 4);
      const int col = wn * 64 + 16 * b + (lane & 15);
      *(uint32_t *)(lds + col * GL_LDT + row) = packed;
    }
  }
  __syncthreads();
  {
    constexpr int RUNS = TR / 2 / 16;  // uint4 per thread: half a column
    const int col = tid >> 1, half = tid & 1;
    const uint4 *src = (const uint4 *)(lds + col * GL_LDT + half * (TR / 2));
    uint4 *dst = (uint4 *)(tpl + ((int64_t)gl * Np + (int64_t)tn * TC + col) * Mp +
                           (int64_t)tm * TR + half * (TR / 2));
#pragma unroll
    for (int k = 0; k < RUNS; ++k) dst[k] = src[k];
  }
}

// ---------------------------------------------------------------------------
// (S4), FP8 E4M3 back-end (balanced base-17 digits, Eq. fp8digits): for every
// slice pair and modulus r r' = d0 d0' + 17 (d0 d1' + d1 d0') + 289 d1 d1',
// so three FP32 accumulators per output (the two cross products share one).
// Every partial sum is an integer below 2 K S 64 < 2^24, exact in FP32 under
// the plan's bound.  One workgroup = one 128x128 tile, eight wavefronts of
// 32x64 (2x4 fragments of v_mfma_f32_16x16x128_f8f6f4).  A 128-wide inner
// step takes two consecutive 1 KiB blocks per operand; both operands use the
// same byte-to-k assignment, so the products pair up as the dot product
// needs.
// ---------------------------------------------------------------------------
namespace {
typedef int v8i_t __attribute__((ext_vector_type(8)));
typedef float v4f_t __attribute__((ext_vector_type(4)));
typedef double v2d_t __attribute__((ext_vector_type(2)));
typedef double v4d_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v8i_t load_pair(const uint8_t *p) {
  const v4i lo = *(const v4i *)p, hi = *(const v4i *)(p + 1024);
  return v8i_t{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
}

// t = ((C mod m) y) mod m for an integer C held exactly in a double with
// |C y| < 2^44: floor(C y RN(1/m)) is off only for exact multiples (see
// mod_times_y), so the remainder lies in [0, m].
__device__ __forceinline__ uint32_t mod_times_y_d(double c, double md, double yd, double im,
                                                  uint32_t m) {
  const double x = c * yd;
  const double q = __builtin_floor(x * im);
  const uint32_t r = (uint32_t)__builtin_fma(-q, md, x);
  const uint32_t rm = r - m;
  return r < rm ? r : rm;
}
}  // namespace

// (S4) on the FP16 engine (the FP16 back-end: the INT8 moduli, one product
// per modulus, FP32 accumulation).  The operands are the INT8 residue planes:
// each lane's 16 residues of a 64-k block become two 8-element f16 vectors
// in registers (byte u = r + 128 placed under the exponent of 1024, then
// 1152 subtracted: exact), fed to v_mfma_f32_16x16x32_f16 -- the k order
// inside a block only has to agree between A and B.  Every FP32 partial sum
// covers at most 1024 products of residues |r| <= 128, so it stays within
// 2^24 and exact; it is folded into int32 accumulators every 16 blocks and
// at the end of each slice pair.  Tile and epilogue as k_gemm_i8.
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef _Float16 v2h __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t i8pair_to_f16(uint32_t u, uint32_t sel) {
  v2h h = __builtin_bit_cast(v2h, __builtin_amdgcn_perm(0x64646464u, u, sel));
  h = h - (v2h){(_Float16)1152.0f, (_Float16)1152.0f};
  return __builtin_bit_cast(uint32_t, h);
}

__device__ __forceinline__ void i8_to_f16(v4i f, v8h &lo, v8h &hi) {
  uint32_t o[8];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const uint32_t u = (uint32_t)f[d] ^ 0x80808080u;  // r + 128 per byte
    o[2 * d] = i8pair_to_f16(u, 0x04010400u);         // bytes 0, 1 under 0x64
    o[2 * d + 1] = i8pair_to_f16(u, 0x04030402u);     // bytes 2, 3
  }
  const v4i a = {(int)o[0], (int)o[1], (int)o[2], (int)o[3]};
  const v4i b = {(int)o[4], (int)o[5], (int)o[6], (int)o[7]};
  lo = __builtin_bit_cast(v8h, a);
  hi = __builtin_bit_cast(v8h, b);
}

__global__ __launch_bounds__(256) void k_gemm_f16(const int8_t *__restrict__ pa,
                                                  const int8_t *__restrict__ pb,
                                                  uint8_t *__restrict__ tpl, const DevPlan *pl,
                                                  int64_t Mp, int64_t Np, int64_t KB,
                                                  int64_t planeA, int64_t planeB, int tilesM,
                                                  int tilesN) {
  constexpr int LDT = 144;
  __shared__ __attribute__((aligned(16))) uint8_t tile[128 * LDT];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const int nb = gridDim.x, pid = blockIdx.x;
  const int xcd = pid & 7, loc = pid >> 3;
  const int qd = nb >> 3, rm = nb & 7;
  const int lt = (xcd < rm ? xcd * (qd + 1) : rm * (qd + 1) + (xcd - rm) * qd) + loc;
  const int tn = lt % tilesN;
  const int tm = (lt / tilesN) % tilesM;
  const int pr = lt / (tilesN * tilesM);
  const int nmod = pl->nmod;
  // products in modulus-major order: neighbouring groups of one modulus share
  // most of their slice planes; gl is the product's t-plane
  const int gi = pr % pl->ng, l = pr / pl->ng;
  const int gl = gi * nmod + l;
  const int S = pl->S, g = pl->g0 + gi;
  const int ta0 = g - (S - 1) > 0 ? g - (S - 1) : 0;
  const int ta1 = g < S - 1 ? g : S - 1;

  v4i acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = v4i{0, 0, 0, 0};

  for (int ta = ta0; ta <= ta1; ++ta) {
    const int tb = g - ta;
    const int8_t *A0 = pa + (int64_t)(ta * nmod + l) * planeA +
                       ((int64_t)(tm * 8 + wm * 4) * KB) * 1024 + lane * 16;
    const int8_t *B0 = pb + (int64_t)(tb * nmod + l) * planeB +
                       ((int64_t)(tn * 8 + wn * 4) * KB) * 1024 + lane * 16;
    v4f facc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) facc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int64_t kb = 0; kb < KB; ++kb) {
      v8h al[4], ah[4], bl[4], bh[4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
        i8_to_f16(*(const v4i *)(A0 + ((int64_t)a * KB + kb) * 1024), al[a], ah[a]);
#pragma unroll
      for (int b = 0; b < 4; ++b)
        i8_to_f16(*(const v4i *)(B0 + ((int64_t)b * KB + kb) * 1024), bl[b], bh[b]);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          facc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[a], bl[b], facc[a][b], 0, 0, 0);
          facc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[a], bh[b], facc[a][b], 0, 0, 0);
        }
      if ((kb & 15) == 15 || kb + 1 == KB) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) {
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[a][b][r] += (int)facc[a][b][r];
            facc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
          }
      }
    }
  }
  const uint32_t m = (uint32_t)pl->m[l];
  const double md = (double)m, yd = (double)pl->y[l], im = pl->inv_m[l];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      uint32_t packed = 0;
#pragma unroll
      for (int r = 0; r < 4; ++r) packed |= mod_times_y(acc[a][b][r], md, yd, im, m) << (8 * r);
      const int row = wm * 64 + 16 * a + 4 * (lane >> 4);
      const int col = wn * 64 + 16 * b + (lane & 15);
      *(uint32_t *)(tile + col * LDT + row) = packed;
    }
  }
  __syncthreads();
  {
    const int col = threadIdx.x >> 1, half = threadIdx.x & 1;
    const uint4 *src = (const uint4 *)(tile + col * LDT + half * 64);
    uint4 *dst = (uint4 *)(tpl + ((int64_t)gl * Np + (int64_t)tn * 128 + col) * Mp +
                           (int64_t)tm * 128 + half * 64);
#pragma unroll
    for (int k = 0; k < 4; ++k) dst[k] = src[k];
  }
}


__global__ __launch_bounds__(512) void k_gemm_f8(const uint8_t *__restrict__ pa,
                                                 const uint8_t *__restrict__ pb,
                                                 uint8_t *__restrict__ tpl, const DevPlan *pl,
                                                 int64_t Mp, int64_t Np, int64_t KB,
                                                 int64_t planeA, int64_t planeB, int tilesM,
                                                 int tilesN) {
  constexpr int LDT = 144;
  __shared__ __attribute__((aligned(16))) uint8_t tile[128 * LDT];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wm = wv >> 1, wn = wv & 1;  // 4 x 2 wavefronts of 32 x 64
  const int nb = gridDim.x, pid = blockIdx.x;
  const int xcd = pid & 7, loc = pid >> 3;
  const int qd = nb >> 3, rm = nb & 7;
  const int lt = (xcd < rm ? xcd * (qd + 1) : rm * (qd + 1) + (xcd - rm) * qd) + loc;
  const int tn = lt % tilesN;
  const int tm = (lt / tilesN) % tilesM;
  const int pr = lt / (tilesN * tilesM);
  const int nmod = pl->nmod;
  // products in modulus-major order: neighbouring groups of one modulus share
  // most of their slice planes; gl is the product's t-plane
  const int gi = pr % pl->ng, l = pr / pl->ng;
  const int gl = gi * nmod + l;
  const int S = pl->S, g = pl->g0 + gi;
  const int ta0 = g - (S - 1) > 0 ? g - (S - 1) : 0;
  const int ta1 = g < S - 1 ? g : S - 1;

  v4f_t c0[2][4], c1[2][4], c2[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      c0[a][b] = v4f_t{0.f, 0.f, 0.f, 0.f};
      c1[a][b] = c0[a][b];
      c2[a][b] = c0[a][b];
    }
  for (int ta = ta0; ta <= ta1; ++ta) {
    const int tb = g - ta;
    const uint8_t *A0 = pa + (int64_t)(2 * (ta * nmod + l)) * planeA +
                        ((int64_t)(tm * 8 + wm * 2) * KB) * 1024 + lane * 16;
    const uint8_t *B0 = pb + (int64_t)(2 * (tb * nmod + l)) * planeB +
                        ((int64_t)(tn * 8 + wn * 4) * KB) * 1024 + lane * 16;
    for (int64_t kb = 0; kb < KB; kb += 2) {
      v8i_t a0[2], a1[2], b0[4], b1[4];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const uint8_t *p = A0 + ((int64_t)a * KB + kb) * 1024;
        a0[a] = load_pair(p);
        a1[a] = load_pair(p + planeA);
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const uint8_t *p = B0 + ((int64_t)b * KB + kb) * 1024;
        b0[b] = load_pair(p);
        b1[b] = load_pair(p + planeB);
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          c0[a][b] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a0[a], b0[b], c0[a][b], 0, 0,
                                                                      0, 0, 0, 0);
          c1[a][b] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a0[a], b1[b], c1[a][b], 0, 0,
                                                                      0, 0, 0, 0);
          c1[a][b] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a1[a], b0[b], c1[a][b], 0, 0,
                                                                      0, 0, 0, 0);
          c2[a][b] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a1[a], b1[b], c2[a][b], 0, 0,
                                                                      0, 0, 0, 0);
        }
    }
  }
  const uint32_t m = (uint32_t)pl->m[l];
  const double md = (double)m, yd = (double)pl->y[l], im = pl->inv_m[l];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      uint32_t packed = 0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double cc = (double)c0[a][b][r] + 17.0 * (double)c1[a][b][r] +
                          289.0 * (double)c2[a][b][r];  // exact: |cc| < 2^33
        packed |= mod_times_y_d(cc, md, yd, im, m) << (8 * r);
      }
      const int row = wm * 32 + 16 * a + 4 * (lane >> 4);
      const int col = wn * 64 + 16 * b + (lane & 15);
      *(uint32_t *)(tile + col * LDT + row) = packed;
    }
  }
  __syncthreads();
  {
    const int col = threadIdx.x >> 2, qtr = threadIdx.x & 3;
    const uint4 *src = (const uint4 *)(tile + col * LDT + qtr * 32);
    uint4 *dst = (uint4 *)(tpl + ((int64_t)gl * Np + (int64_t)tn * 128 + col) * Mp +
                           (int64_t)tm * 128 + qtr * 32);
    dst[0] = src[0];
    dst[1] = src[1];
  }
}

// ---------------------------------------------------------------------------
// (S4), binary64-moduli back-end (Eq. fp64mod): residues of ~22-bit primes as
// doubles, one FP64 MFMA product per (group, modulus); every partial sum is
// an integer below K S m^2 < 2^53, so the accumulation is exact.  One
// workgroup = one 128x128 tile, four wavefronts of 64x64 (4x4 fragments of
// v_mfma_f64_16x16x4_f64); a 1 KiB block holds 16 rows x 8 k (lane l: row
// l%16, k l/16 and 4 + l/16), i.e. two MFMA steps.  t-values are uint32.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gemm_f64(const double *__restrict__ pa,
                                                  const double *__restrict__ pb,
                                                  uint32_t *__restrict__ tpl, const DevPlan *pl,
                                                  int64_t Mp, int64_t Np, int64_t KB8,
                                                  int64_t planeA, int64_t planeB, int tilesM,
                                                  int tilesN) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const int nb = gridDim.x, pid = blockIdx.x;
  const int xcd = pid & 7, loc = pid >> 3;
  const int qd = nb >> 3, rm = nb & 7;
  const int lt = (xcd < rm ? xcd * (qd + 1) : rm * (qd + 1) + (xcd - rm) * qd) + loc;
  const int tn = lt % tilesN;
  const int tm = (lt / tilesN) % tilesM;
  const int pr = lt / (tilesN * tilesM);
  const int nmod = pl->nmod;
  // products in modulus-major order: neighbouring groups of one modulus share
  // most of their slice planes; gl is the product's t-plane
  const int gi = pr % pl->ng, l = pr / pl->ng;
  const int gl = gi * nmod + l;
  const int S = pl->S, g = pl->g0 + gi;
  const int ta0 = g - (S - 1) > 0 ? g - (S - 1) : 0;
  const int ta1 = g < S - 1 ? g : S - 1;

  v4d_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = v4d_t{0.0, 0.0, 0.0, 0.0};
  for (int ta = ta0; ta <= ta1; ++ta) {
    const int tb = g - ta;
    const double *A0 = pa + (int64_t)(ta * nmod + l) * planeA +
                       ((int64_t)(tm * 8 + wm * 4) * KB8) * 128 + lane * 2;
    const double *B0 = pb + (int64_t)(tb * nmod + l) * planeB +
                       ((int64_t)(tn * 8 + wn * 4) * KB8) * 128 + lane * 2;
    v2d_t af[4], bf[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) af[a] = *(const v2d_t *)(A0 + (int64_t)a * KB8 * 128);
#pragma unroll
    for (int b = 0; b < 4; ++b) bf[b] = *(const v2d_t *)(B0 + (int64_t)b * KB8 * 128);
    for (int64_t kb = 0; kb < KB8; ++kb) {
      v2d_t an[4], bn[4];
      const bool more = kb + 1 < KB8;
      if (more) {
#pragma unroll
        for (int a = 0; a < 4; ++a) an[a] = *(const v2d_t *)(A0 + ((int64_t)a * KB8 + kb + 1) * 128);
#pragma unroll
        for (int b = 0; b < 4; ++b) bn[b] = *(const v2d_t *)(B0 + ((int64_t)b * KB8 + kb + 1) * 128);
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a][0], bf[b][0], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a][1], bf[b][1], acc[a][b], 0, 0, 0);
        }
      if (more) {
#pragma unroll
        for (int a = 0; a < 4; ++a) af[a] = an[a];
#pragma unroll
        for (int b = 0; b < 4; ++b) bf[b] = bn[b];
      }
    }
  }
  // t = ((C mod m) y) mod m.  |C| < 2^53: floor(C RN(1/m)) is within one of
  // floor(C/m) either way, so C - q m lies in [-m, 2m) and is corrected once;
  // then (c y) < 2^46 is reduced like the small back-ends.
  const uint32_t m = (uint32_t)pl->m[l];
  const double md = (double)m, yd = (double)pl->y[l], im = pl->inv_m[l];
  // The FP64 MFMA's result rows are interleaved: value r of lane l is row
  // l/16 + 4 r, column l%16, of the 16x16 fragment.
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t row0 = (int64_t)tm * 128 + wm * 64 + 16 * a + (lane >> 4);
      const int64_t col = (int64_t)tn * 128 + wn * 64 + 16 * b + (lane & 15);
      uint32_t *dst = tpl + ((int64_t)gl * Np + col) * Mp + row0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double C = acc[a][b][r];
        const double q = __builtin_floor(C * im);
        double c = __builtin_fma(-q, md, C);
        c = c < 0.0 ? c + md : c;
        c = c >= md ? c - md : c;
        dst[4 * r] = mod_times_y_d(c, md, yd, im, m);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// (S5)+(S6) consumer
// ---------------------------------------------------------------------------
template <int NC, int NWC, int ND, class TT>
__global__ __launch_bounds__(256) void k_consumer(const TT *__restrict__ tpl, int64_t Mp,
                                                  int64_t Np, double *C, int64_t ldc, int64_t M,
                                                  int64_t N, const int32_t *ea, const int32_t *eb,
                                                  const DevPlan *pl, int mode) {
  __shared__ uint32_t stage[256 * CST];
  uint32_t *st = stage + threadIdx.x * CST;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i >= M || j >= N) return;
  const int nmod = pl->nmod, Q = pl->Q;
  const int32_t ei = ea[i], ej = eb[j];
  const bool zero = ei == EXP_ZERO || ej == EXP_ZERO;
  const int eps = zero ? 0 : pl->w * pl->g0 - (Q - 1 - ei) - (Q - 1 - ej);
  double c[NC];
  consume_element<NC, NWC, ND, TT>(
      [&](int gi) { return tpl + ((int64_t)gi * nmod * Np + j) * Mp + i; }, Np * Mp, pl, st, zero,
      eps, c);
  double *dst = C + (i + j * ldc) * NC;
  if (mode == 0) {
    ozx::store<NC>(dst, c);
  } else {
    double a[NC], nc_[NC], r[NC];
    ozx::load<NC>(dst, a);
#pragma unroll
    for (int q = 0; q < NC; ++q) nc_[q] = -c[q];
    ozx::add<NC>(a, nc_, r);
    ozx::store<NC>(dst, r);
  }
}


// Block (x, y) of a 2-D grid in an XCD-aware order: workgroups are dispatched
// to the 8 XCDs in turn, so each XCD is given a contiguous range of logical
// blocks; neighbouring 64-element blocks of a column then share an L2 and
// each 128-byte line of a t-plane row is fetched from HBM once.
__device__ __forceinline__ void xcd_block(int64_t &bx, int64_t &by) {
  const int64_t gx = gridDim.x, nb = gx * gridDim.y;
  const int64_t pid = blockIdx.x + gx * blockIdx.y;
  const int64_t xcd = pid & 7, loc = pid >> 3, qd = nb >> 3, rm = nb & 7;
  const int64_t lt = (xcd < rm ? xcd * (qd + 1) : rm * (qd + 1) + (xcd - rm) * qd) + loc;
  bx = lt % gx;
  by = lt / gx;
}

template <int NC, int NWC, int NB>
__global__ __launch_bounds__(64) void k_consumer_mx(const uint8_t *__restrict__ tpl, int64_t Mp,
                                                    int64_t Np, double *__restrict__ C,
                                                    int64_t ldc, int64_t M, int64_t N,
                                                    const int32_t *__restrict__ ea,
                                                    const int32_t *__restrict__ eb,
                                                    const DevPlan *__restrict__ pl, int mode) {
  constexpr int ND = NB / 2, STG = stage_words<ND>();
  static_assert(64 * MX_TBS <= 32 * MX_CBS * 4 && 64 * STG <= 32 * MX_CBS, "LDS reuse");
  // the t-byte rows, then the column sums of 32 elements, then the digit
  // staging of add_shifted_digits share one buffer
  __shared__ __attribute__((aligned(16))) int32_t buf[32 * MX_CBS];
  const int lane = (int)threadIdx.x;
  int64_t bx, j;
  xcd_block(bx, j);
  const int64_t i0 = bx * 64, i = i0 + lane;
  const int nmod = pl->nmod, w = pl->w, ng = pl->ng, Q = pl->Q;
  v4i tab[MX_BLK];
#pragma unroll
  for (int b = 0; b < MX_BLK; ++b) tab[b] = *(const v4i *)&pl->crtm[b][lane][0];
  const bool valid = i < M;
  const int32_t ej = eb[j], ei = valid ? ea[i] : EXP_ZERO;
  const bool zero = ei == EXP_ZERO || ej == EXP_ZERO;
  const int eps = zero ? 0 : w * pl->g0 - (Q - 1 - ei) - (Q - 1 - ej);
  const int64_t ps = Np * Mp;
  uint32_t *st = (uint32_t *)buf + lane * STG;
  uint32_t cb[NWC];
#pragma unroll
  for (int k = 0; k < NWC; ++k) cb[k] = 0u;
  for (int gi = 0; gi < ng; ++gi) {
    int32_t d[ND];
    crt_group_mx<NB>(tpl + (int64_t)gi * nmod * ps + j * Mp + i0, ps, nmod, pl, tab, buf, lane, d);
    add_shifted_digits<NWC, ND, STG>(cb, d, w * gi, st);
    __syncthreads();  // the buffer takes the next group's t-bytes
  }
  if (!valid) return;
  double c[NC];
  if (zero) {
#pragma unroll
    for (int q = 0; q < NC; ++q) c[q] = 0.0;
  } else {
    round_out_n<NWC, NC>(cb, eps, c);
  }
  double *dst = C + (i + j * ldc) * NC;
  if (mode == 0) {
    ozx::store<NC>(dst, c);
  } else {
    double a[NC], nc_[NC], r[NC];
    ozx::load<NC>(dst, a);
#pragma unroll
    for (int qq = 0; qq < NC; ++qq) nc_[qq] = -c[qq];
    ozx::add<NC>(a, nc_, r);
    ozx::store<NC>(dst, r);
  }
}

// Fused (S4)+(S5)+(S6) on the INT8 back-end: one workgroup per 32 x 32
// output tile keeps every (digit group, modulus) t-value of its tile in LDS
// instead of writing t-planes to HBM.  Eight wavefronts: wavefront w owns
// the 16 x 16 block (w & 1, (w >> 1) & 1) of the tile and the products gl
// of parity w >> 2, each the batched modular product of k_gemm_i8 on
// fragments read straight from the residue planes (the next product's
// fragments in flight while the current one multiplies), then the t
// epilogue into LDS ([gl][column][row], 1 KiB per product).  After one
// barrier every thread takes two elements through the consumer's CRT,
// rounding and update (consume_element_b reading its bytes from LDS), so
// the results equal those of k_gemm_i8 + k_consumer_mx bit for bit.
constexpr int FUSE_T = 32;        // tile edge
constexpr int FUSE_MAXPROD = 120;  // (group, modulus) products whose t-bytes fit in LDS
constexpr int FUSE_LDS_MAX = 160 * 1024;
// per-thread staging words of the consumer phase (NB byte columns)
template <int NB>
constexpr int fuse_stage_words() { return stage_words<NB / 2>(); }
static_assert(FUSE_MAXPROD * 1024 + 512 * fuse_stage_words<48>() * 4 <= FUSE_LDS_MAX,
              "t-bytes and staging of the largest plan fit in LDS");
template <int NC, int NWC, int NB>
__global__ __launch_bounds__(512) void k_fused_b(const int8_t *__restrict__ pa,
                                                 const int8_t *__restrict__ pb,
                                                 const DevPlan *__restrict__ pl, int64_t KB,
                                                 int64_t planeA, int64_t planeB, double *C,
                                                 int64_t ldc, int64_t M, int64_t N,
                                                 const int32_t *__restrict__ ea,
                                                 const int32_t *__restrict__ eb, int mode,
                                                 int tilesM) {
  extern __shared__ __attribute__((aligned(16))) uint8_t fsm[];
  const int nmod = pl->nmod, ng = pl->ng, S = pl->S, g0 = pl->g0;
  const int npr = ng * nmod;
  uint8_t *tl = fsm;
  uint32_t *stage = (uint32_t *)(fsm + (size_t)npr * 1024);
  const int tm = (int)(blockIdx.x % (unsigned)tilesM), tn = (int)(blockIdx.x / (unsigned)tilesM);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int bm = wv & 1, bn = (wv >> 1) & 1, par = wv >> 2;
  const int64_t arow = (int64_t)(tm * 2 + bm) * KB * 1024 + lane * 16;
  const int64_t bcol = (int64_t)(tn * 2 + bn) * KB * 1024 + lane * 16;
  // fragments of one product: (pairs <= S) x KB blocks of A and of B
  auto pairs_of = [&](int gl, int &l, int &ta0, int &ta1, int &g) {
    l = gl % nmod;
    g = g0 + gl / nmod;
    ta0 = g - (S - 1) > 0 ? g - (S - 1) : 0;
    ta1 = g < S - 1 ? g : S - 1;
  };
  for (int gl = par; gl < npr; gl += 2) {
    int l, ta0, ta1, g;
    pairs_of(gl, l, ta0, ta1, g);
    v4i acc = {0, 0, 0, 0};
    for (int ta = ta0; ta <= ta1; ++ta) {
      const int8_t *A0 = pa + (int64_t)(ta * nmod + l) * planeA + arow;
      const int8_t *B0 = pb + (int64_t)((g - ta) * nmod + l) * planeB + bcol;
      v4i af = *(const v4i *)A0, bf = *(const v4i *)B0;
      for (int64_t kb = 0; kb < KB; ++kb) {
        v4i an = af, bnx = bf;
        if (kb + 1 < KB) {
          an = *(const v4i *)(A0 + (kb + 1) * 1024);
          bnx = *(const v4i *)(B0 + (kb + 1) * 1024);
        }
        acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(af, bf, acc, 0, 0, 0);
        af = an;
        bf = bnx;
      }
    }
    const uint32_t m = (uint32_t)pl->m[l];
    const double md = (double)m, yd = (double)pl->y[l], im = pl->inv_m[l];
    uint32_t packed = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) packed |= mod_times_y(acc[r], md, yd, im, m) << (8 * r);
    const int row = bm * 16 + 4 * (lane >> 4), col = bn * 16 + (lane & 15);
    *(uint32_t *)(tl + (size_t)gl * 1024 + col * FUSE_T + row) = packed;
  }
  __syncthreads();
  constexpr int STG = fuse_stage_words<NB>();
  uint32_t *st = stage + threadIdx.x * STG;
  const int Q = pl->Q;
  for (int e = threadIdx.x; e < FUSE_T * FUSE_T; e += 512) {
    const int r = e & (FUSE_T - 1), cc = e / FUSE_T;
    const int64_t i = (int64_t)tm * FUSE_T + r, j = (int64_t)tn * FUSE_T + cc;
    if (i >= M || j >= N) continue;
    const int32_t ei = ea[i], ej = eb[j];
    const bool zero = ei == EXP_ZERO || ej == EXP_ZERO;
    const int eps = zero ? 0 : pl->w * g0 - (Q - 1 - ei) - (Q - 1 - ej);
    double c[NC];
    consume_element_b<NC, NWC, NB, 0, STG>(tl + cc * FUSE_T + r, 1024, pl, st, zero, eps, c);
    double *dst = C + (i + j * ldc) * NC;
    if (mode == 0) {
      ozx::store<NC>(dst, c);
    } else {
      double a[NC], nc_[NC], rr[NC];
      ozx::load<NC>(dst, a);
#pragma unroll
      for (int q = 0; q < NC; ++q) nc_[q] = -c[q];
      ozx::add<NC>(a, nc_, rr);
      ozx::store<NC>(dst, rr);
    }
  }
}

// Export of the group sums (parity hook): Sbar as 64-bit limbs (two's
// complement), layout [gi][j][i][limb], nlimb limbs, from the ND 16-bit
// digits of a CRT routine.
template <int ND>
__device__ __forceinline__ void store_sbar_limbs(const int32_t (&d)[ND], uint64_t *o, int nlimb) {
  const uint64_t fill = d[ND - 1] < 0 ? ~0ull : 0ull;
  for (int q = 0; q < nlimb; ++q) {
    uint64_t v = 0;
    if (4 * q + 3 < ND) {
      for (int k = 0; k < 4; ++k) v |= ((uint64_t)((uint32_t)d[4 * q + k] & 0xffffu)) << (16 * k);
    } else {
      for (int k = 0; k < 4; ++k) {
        const uint64_t dig = 4 * q + k < ND ? (uint64_t)((uint32_t)d[4 * q + k] & 0xffffu)
                                            : (fill & 0xffffu);
        v |= dig << (16 * k);
      }
    }
    o[q] = v;
  }
}

// binary64 moduli: the group sums of crt_digits, the CRT of k_consumer
template <class TT>
__global__ __launch_bounds__(256) void k_crt_export(const TT *__restrict__ tpl, int64_t Mp,
                                                    int64_t Np, int64_t M, int64_t N,
                                                    const DevPlan *pl, uint64_t *out, int nlimb) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i >= M || j >= N) return;
  const int nmod = pl->nmod;
  for (int gi = 0; gi < pl->ng; ++gi) {
    int32_t d[NDCRT];
    crt_digits<NDCRT, TT>(tpl + ((int64_t)gi * nmod * Np + j) * Mp + i, Np * Mp, pl, d);
    store_sbar_limbs<NDCRT>(d, out + (((int64_t)gi * N + j) * M + i) * nlimb, nlimb);
  }
}

// byte back-ends (INT8, FP8): the group sums of crt_group_bytes<NB>, the
// CRT that k_consumer_limbs and the fused kernel run (k_consumer_mx forms
// the same digits on the matrix cores), with the same NB
template <int NB>
__global__ __launch_bounds__(256) void k_crt_export_b(const uint8_t *__restrict__ tpl, int64_t Mp,
                                                      int64_t Np, int64_t M, int64_t N,
                                                      const DevPlan *__restrict__ pl,
                                                      uint64_t *out, int nlimb) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i >= M || j >= N) return;
  const int nmod = pl->nmod;
  for (int gi = 0; gi < pl->ng; ++gi) {
    int32_t d[NB / 2];
    crt_group_bytes<NB>(tpl + ((int64_t)gi * nmod * Np + j) * Mp + i, Np * Mp, nmod, pl, d);
    store_sbar_limbs<NB / 2>(d, out + (((int64_t)gi * N + j) * M + i) * nlimb, nlimb);
  }
}

// The group sums of k_consumer_mx's own route, exported like k_crt_export_b.
template <int NB>
__global__ __launch_bounds__(64) void k_crt_export_mx(const uint8_t *__restrict__ tpl, int64_t Mp,
                                                      int64_t Np, int64_t M, int64_t N,
                                                      const DevPlan *__restrict__ pl,
                                                      uint64_t *out, int nlimb) {
  __shared__ __attribute__((aligned(16))) int32_t buf[32 * MX_CBS];
  const int lane = (int)threadIdx.x;
  int64_t bx, j;
  xcd_block(bx, j);
  const int64_t i0 = bx * 64, i = i0 + lane;
  const int nmod = pl->nmod;
  const int64_t ps = Np * Mp;
  v4i tab[MX_BLK];
#pragma unroll
  for (int b = 0; b < MX_BLK; ++b) tab[b] = *(const v4i *)&pl->crtm[b][lane][0];
  for (int gi = 0; gi < pl->ng; ++gi) {
    int32_t d[NB / 2];
    crt_group_mx<NB>(tpl + (int64_t)gi * nmod * ps + j * Mp + i0, ps, nmod, pl, tab, buf, lane, d);
    if (i < M) store_sbar_limbs<NB / 2>(d, out + (((int64_t)gi * N + j) * M + i) * nlimb, nlimb);
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
namespace ozl {

hipError_t launch_zero_expansions(int nc, double *C, int64_t ldc, int64_t M, int64_t N,
                                  hipStream_t s) {
  const int64_t total = M * N * nc;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_expansions, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, C,
                     ldc, M, N, nc);
  return hipGetLastError();
}

hipError_t launch_exponents(int nc, const double *X, int64_t ld, int64_t rows, int64_t cols,
                            int rowwise, int32_t *e, hipStream_t s) {
  if (rowwise) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, e,
                       EXP_ZERO, rows);
    if (cols <= 0) return hipGetLastError();
    dim3 g((unsigned)((rows + 255) / 256), (unsigned)((cols + ROWEXP_CHUNK - 1) / ROWEXP_CHUNK));
    if (nc == 2) hipLaunchKernelGGL(k_row_exponents<2>, g, dim3(256), 0, s, X, ld, rows, cols, e);
    else if (nc == 3) hipLaunchKernelGGL(k_row_exponents<3>, g, dim3(256), 0, s, X, ld, rows, cols, e);
    else hipLaunchKernelGGL(k_row_exponents<4>, g, dim3(256), 0, s, X, ld, rows, cols, e);
  } else {
    if (cols <= 0) return hipSuccess;
    dim3 g((unsigned)((cols + 3) / 4));
    if (nc == 2) hipLaunchKernelGGL(k_col_exponents<2>, g, dim3(256), 0, s, X, ld, rows, cols, e);
    else if (nc == 3) hipLaunchKernelGGL(k_col_exponents<3>, g, dim3(256), 0, s, X, ld, rows, cols, e);
    else hipLaunchKernelGGL(k_col_exponents<4>, g, dim3(256), 0, s, X, ld, rows, cols, e);
  }
  return hipGetLastError();
}

template <int NC, int NWX, int PL>
static void producer_nh(int nh, dim3 g, hipStream_t s, const double *X, int64_t ld, int rowwise,
                        int64_t nout, int64_t K, int64_t KB, const int32_t *exps,
                        const DevPlan *pl, void *planes, int64_t plane_elems) {
  if (nh <= 8)
    hipLaunchKernelGGL((k_producer<NC, NWX, 8, PL>), g, dim3(256), 0, s, X, ld, rowwise, nout, K,
                       KB, exps, pl, planes, plane_elems);
  else if (nh <= 12)
    hipLaunchKernelGGL((k_producer<NC, NWX, 12, PL>), g, dim3(256), 0, s, X, ld, rowwise, nout, K,
                       KB, exps, pl, planes, plane_elems);
  else
    hipLaunchKernelGGL((k_producer<NC, NWX, NHMAX, PL>), g, dim3(256), 0, s, X, ld, rowwise, nout,
                       K, KB, exps, pl, planes, plane_elems);
}

template <int NC, int NWX, int PL, int EPT>
static void producer_b_ept(int nwt, dim3 g, hipStream_t s, const double *X, int64_t ld,
                           int rowwise, int64_t nout, int64_t K, int64_t KB, const int32_t *exps,
                           const DevPlan *pl, uint8_t *P, int64_t plane_elems) {
  if (nwt <= 4)
    hipLaunchKernelGGL((k_producer_b<NC, NWX, 4, PL, EPT>), g, dim3(256), 0, s, X, ld, rowwise,
                       nout, K, KB, exps, pl, P, plane_elems);
  else if (nwt <= 6)
    hipLaunchKernelGGL((k_producer_b<NC, NWX, 6, PL, EPT>), g, dim3(256), 0, s, X, ld, rowwise,
                       nout, K, KB, exps, pl, P, plane_elems);
  else
    hipLaunchKernelGGL((k_producer_b<NC, NWX, REC_PWMAX, PL, EPT>), g, dim3(256), 0, s, X, ld,
                       rowwise, nout, K, KB, exps, pl, P, plane_elems);
}

// g: (KB, OB, moduli parts); fine: one element per thread (four workgroups
// per block) for products too small to fill the chip otherwise
template <int NC, int NWX, int PL>
static void producer_b_nw(int nwt, bool fine, dim3 g, hipStream_t s, const double *X, int64_t ld,
                          int rowwise, int64_t nout, int64_t K, int64_t KB, const int32_t *exps,
                          const DevPlan *pl, void *planes, int64_t plane_elems) {
  uint8_t *P = (uint8_t *)planes;
  if (fine) {
    g.x *= 4;
    producer_b_ept<NC, NWX, PL, 1>(nwt, g, s, X, ld, rowwise, nout, K, KB, exps, pl, P, plane_elems);
  } else {
    producer_b_ept<NC, NWX, PL, 4>(nwt, g, s, X, ld, rowwise, nout, K, KB, exps, pl, P, plane_elems);
  }
}

template <int PL>
static void producer_b(int nc, int nwx, int nwt, bool fine, dim3 g, hipStream_t s, const double *X,
                       int64_t ld, int rowwise, int64_t nout, int64_t K, int64_t KB,
                       const int32_t *exps, const DevPlan *pl, void *planes,
                       int64_t plane_elems) {
#define OZ_PRODB(NC_, NWX_)                                                                     \
  producer_b_nw<NC_, NWX_, PL>(nwt, fine, g, s, X, ld, rowwise, nout, K, KB, exps, pl, planes, \
                               plane_elems)
  if (nc == 2) { if (nwx <= 8) OZ_PRODB(2, 8); else OZ_PRODB(2, 12); }
  else if (nc == 3) { if (nwx <= 8) OZ_PRODB(3, 8); else OZ_PRODB(3, 12); }
  else { if (nwx <= 8) OZ_PRODB(4, 8); else OZ_PRODB(4, 12); }
#undef OZ_PRODB
}

template <int PL>
static void producer_pl(int nc, int nwx, int nh, dim3 g, hipStream_t s, const double *X,
                        int64_t ld, int rowwise, int64_t nout, int64_t K, int64_t KB,
                        const int32_t *exps, const DevPlan *pl, void *planes,
                        int64_t plane_elems) {
#define OZ_PROD(NC_, NWX_) \
  producer_nh<NC_, NWX_, PL>(nh, g, s, X, ld, rowwise, nout, K, KB, exps, pl, planes, plane_elems)
  if (nc == 2) { if (nwx <= 8) OZ_PROD(2, 8); else OZ_PROD(2, 12); }
  else if (nc == 3) { if (nwx <= 8) OZ_PROD(3, 8); else OZ_PROD(3, 12); }
  else { if (nwx <= 8) OZ_PROD(4, 8); else OZ_PROD(4, 12); }
#undef OZ_PROD
}

hipError_t launch_producer(int nc, int nwx, int nh, int nwt, const double *X, int64_t ld, int rowwise,
                           int64_t nout, int64_t noutp, int64_t K, int64_t Kp,
                           const int32_t *exps, const DevPlan *pl, int nmod, int backend,
                           void *planes,
                           int64_t plane_elems, hipStream_t s) {
  const int64_t KB = Kp / 64, OB = noutp / 16;
  if (KB <= 0 || OB <= 0) return hipSuccess;
  // the byte producer addresses a plane with 32-bit offsets
  if (backend != PLANES_F64 && plane_elems >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  dim3 g((unsigned)KB, (unsigned)OB);
  // byte back-ends on products too small to give 4096 wavefronts (four per
  // SIMD): one element per thread, then the moduli split over up to 8 parts
  const bool fine = KB * OB * 4 < 4096;
  const int64_t waves = KB * OB * (fine ? 16 : 4);
  dim3 gb = g;
  gb.z = (unsigned)std::max<int64_t>(1, std::min<int64_t>({8, nmod, (4096 + waves - 1) / waves}));
  if (backend == PLANES_F8)
    producer_b<PL_F8>(nc, nwx, nwt, fine, gb, s, X, ld, rowwise, nout, K, KB, exps, pl, planes,
                      plane_elems);
  else if (backend == PLANES_F64)
    producer_pl<PL_F64>(nc, nwx, nh, g, s, X, ld, rowwise, nout, K, KB, exps, pl, planes, plane_elems);
  else
    producer_b<PL_I8>(nc, nwx, nwt, fine, gb, s, X, ld, rowwise, nout, K, KB, exps, pl, planes,
                      plane_elems);
  return hipGetLastError();
}

hipError_t launch_gemm_f8(const uint8_t *pa, const uint8_t *pb, uint8_t *tpl, const DevPlan *pl,
                          int ng, int nmod, int64_t Mp, int64_t Np, int64_t Kp, int64_t planeA,
                          int64_t planeB, hipStream_t s) {
  const int64_t prods = (int64_t)ng * nmod;
  if (prods <= 0 || Mp <= 0 || Np <= 0) return hipSuccess;
  if (Mp % 128 || Np % 128 || Kp % 128) return hipErrorInvalidValue;
  const int tilesM = (int)(Mp / 128), tilesN = (int)(Np / 128);
  hipLaunchKernelGGL(k_gemm_f8, dim3((unsigned)(prods * tilesM * tilesN)), dim3(512), 0, s, pa, pb,
                     tpl, pl, Mp, Np, Kp / 64, planeA, planeB, tilesM, tilesN);
  return hipGetLastError();
}

hipError_t launch_gemm_f16(const int8_t *pa, const int8_t *pb, uint8_t *tpl, const DevPlan *pl,
                           int ng, int nmod, int64_t Mp, int64_t Np, int64_t Kp, int64_t planeA,
                           int64_t planeB, hipStream_t s) {
  const int64_t prods = (int64_t)ng * nmod;
  if (prods <= 0 || Mp <= 0 || Np <= 0) return hipSuccess;
  if (Mp % 128 || Np % 128 || Kp % 64) return hipErrorInvalidValue;
  const int tilesM = (int)(Mp / 128), tilesN = (int)(Np / 128);
  hipLaunchKernelGGL(k_gemm_f16, dim3((unsigned)(prods * tilesM * tilesN)), dim3(256), 0, s, pa,
                     pb, tpl, pl, Mp, Np, Kp / 64, planeA, planeB, tilesM, tilesN);
  return hipGetLastError();
}

hipError_t launch_gemm_f64(const double *pa, const double *pb, uint32_t *tpl, const DevPlan *pl,
                           int ng, int nmod, int64_t Mp, int64_t Np, int64_t Kp, int64_t planeA,
                           int64_t planeB, hipStream_t s) {
  const int64_t prods = (int64_t)ng * nmod;
  if (prods <= 0 || Mp <= 0 || Np <= 0) return hipSuccess;
  if (Mp % 128 || Np % 128 || Kp % 64) return hipErrorInvalidValue;
  const int tilesM = (int)(Mp / 128), tilesN = (int)(Np / 128);
  hipLaunchKernelGGL(k_gemm_f64, dim3((unsigned)(prods * tilesM * tilesN)), dim3(256), 0, s, pa,
                     pb, tpl, pl, Mp, Np, Kp / 8, planeA, planeB, tilesM, tilesN);
  return hipGetLastError();
}

hipError_t launch_gemm_i8(const int8_t *pa, const int8_t *pb, uint8_t *tpl, const DevPlan *pl,
                          int ng, int nmod, int64_t Mp, int64_t Np, int64_t Kp, int64_t planeA,
                          int64_t planeB, int tile, hipStream_t s) {
  const int64_t prods = (int64_t)ng * nmod;
  if (prods <= 0 || Mp <= 0 || Np <= 0) return hipSuccess;
  if (tile == GEMM_TILE_AUTO) tile = gemm_tile_auto(prods, Mp, Np);
  if (tile < GEMM_TILE_AUTO || tile > GEMM_TILE_256x256 || !gemm_tile_fits(tile, Mp, Np))
    return hipErrorInvalidValue;
  const int64_t KB = Kp / 64;
  if (tile == GEMM_TILE_256x256) {
    const int tilesM = (int)(Mp / 256), tilesN = (int)(Np / 256);
    hipLaunchKernelGGL((k_gemm_i8_p<2, 4, 3>), dim3((unsigned)(prods * tilesM * tilesN)),
                       dim3(512), 0, s, pa, pb, tpl, pl, Mp, Np, KB, planeA, planeB, tilesM,
                       tilesN);
  } else if (tile == GEMM_TILE_256x128) {
    const int tilesM = (int)(Mp / 256), tilesN = (int)(Np / 128);
    hipLaunchKernelGGL((k_gemm_i8_p<2, 2, 3>), dim3((unsigned)(prods * tilesM * tilesN)),
                       dim3(256), 0, s, pa, pb, tpl, pl, Mp, Np, KB, planeA, planeB, tilesM,
                       tilesN);
  } else {
    const int tilesM = (int)(Mp / 128), tilesN = (int)(Np / 128);
    hipLaunchKernelGGL(k_gemm_i8, dim3((unsigned)(prods * tilesM * tilesN)), dim3(256), 0, s, pa,
                       pb, tpl, pl, Mp, Np, KB, planeA, planeB, tilesM, tilesN);
  }
  return hipGetLastError();
}

hipError_t launch_consumer(int nc, int nwc, int nd, const void *tpl, int tbytes, int64_t Mp,
                           int64_t Np, double *C, int64_t ldc, int64_t M, int64_t N,
                           const int32_t *ea, const int32_t *eb, const DevPlan *pl, int mode,
                           hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 g((unsigned)((M + 255) / 256), (unsigned)N);
#define OZ_CONS(NC_, NWC_, ND_, TT_)                                                            \
  hipLaunchKernelGGL((k_consumer<NC_, NWC_, ND_, TT_>), g, dim3(256), 0, s, (const TT_ *)tpl, Mp, \
                     Np, C, ldc, M, N, ea, eb, pl, mode)
#define OZ_CONS_ND(NC_, NWC_)                            \
  do {                                                  \
    if (nd <= 18) OZ_CONS(NC_, NWC_, 18, uint32_t);     \
    else OZ_CONS(NC_, NWC_, 32, uint32_t);              \
  } while (0)
  if ((tbytes == 1 && nd > 24) || nd > 32) return hipErrorInvalidValue;
  if (tbytes == 1) {
    // the matrix-core CRT: 64-element wavefronts read whole plane rows
    if ((M + 63) / 64 * 64 > Mp) return hipErrorInvalidValue;
    dim3 gx((unsigned)((M + 63) / 64), (unsigned)N);
#define OZ_CONSX(NC_, NWC_, NB_)                                                                \
  hipLaunchKernelGGL((k_consumer_mx<NC_, NWC_, NB_>), gx, dim3(64), 0, s, (const uint8_t *)tpl, \
                     Mp, Np, C, ldc, M, N, ea, eb, pl, mode)
#define OZ_CONSX_ND(NC_, NWC_)                 \
  do {                                        \
    if (nd <= 18) OZ_CONSX(NC_, NWC_, 36);    \
    else OZ_CONSX(NC_, NWC_, 48);             \
  } while (0)
    if (nc == 2) { if (nwc <= 12) OZ_CONSX_ND(2, 12); else OZ_CONSX_ND(2, 16); }
    else if (nc == 3) { if (nwc <= 12) OZ_CONSX_ND(3, 12); else OZ_CONSX_ND(3, 16); }
    else { if (nwc <= 12) OZ_CONSX_ND(4, 12); else OZ_CONSX_ND(4, 16); }
#undef OZ_CONSX_ND
#undef OZ_CONSX
    return hipGetLastError();
  }
  if (nc == 2) { if (nwc <= 12) OZ_CONS_ND(2, 12); else OZ_CONS_ND(2, 16); }
  else if (nc == 3) { if (nwc <= 12) OZ_CONS_ND(3, 12); else OZ_CONS_ND(3, 16); }
  else { if (nwc <= 12) OZ_CONS_ND(4, 12); else OZ_CONS_ND(4, 16); }
#undef OZ_CONS_ND
#undef OZ_CONS
  return hipGetLastError();
}

int fused_max_products() { return FUSE_MAXPROD; }

hipError_t launch_fused_b(int nc, int nwc, int nd, const int8_t *pa, const int8_t *pb,
                          const DevPlan *pl, int ng, int nmod, int64_t Kp, int64_t planeA,
                          int64_t planeB, double *C, int64_t ldc, int64_t M, int64_t N,
                          const int32_t *ea, const int32_t *eb, int mode, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (ng * nmod > FUSE_MAXPROD || nd > 24) return hipErrorInvalidValue;
  const int tilesM = (int)((M + FUSE_T - 1) / FUSE_T), tilesN = (int)((N + FUSE_T - 1) / FUSE_T);
  hipError_t e = hipSuccess;
#define OZ_FUSED(NC_, NWC_, NB_)                                                                  \
  do {                                                                                            \
    const size_t lds = (size_t)ng * nmod * 1024 + 512 * fuse_stage_words<NB_>() * 4;            \
    e = hipFuncSetAttribute((const void *)k_fused_b<NC_, NWC_, NB_>,                             \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                \
    if (e != hipSuccess) return e;                                                                \
    hipLaunchKernelGGL((k_fused_b<NC_, NWC_, NB_>), dim3((unsigned)(tilesM * tilesN)), dim3(512), \
                       lds, s, pa, pb, pl, Kp / 64, planeA, planeB, C, ldc, M, N, ea, eb, mode,    \
                       tilesM);                                                                   \
  } while (0)
#define OZ_FUSED_ND(NC_, NWC_)              \
  do {                                     \
    if (nd <= 18) OZ_FUSED(NC_, NWC_, 36); \
    else OZ_FUSED(NC_, NWC_, 48);          \
  } while (0)
  if (nc == 2) { if (nwc <= 12) OZ_FUSED_ND(2, 12); else OZ_FUSED_ND(2, 16); }
  else if (nc == 3) { if (nwc <= 12) OZ_FUSED_ND(3, 12); else OZ_FUSED_ND(3, 16); }
  else { if (nwc <= 12) OZ_FUSED_ND(4, 12); else OZ_FUSED_ND(4, 16); }
#undef OZ_FUSED_ND
#undef OZ_FUSED
  return hipGetLastError();
}

hipError_t launch_crt_export(const void *tpl, int tbytes, int nd, int64_t Mp, int64_t Np,
                             int64_t M, int64_t N, const DevPlan *pl, uint64_t *out, int nlimb,
                             int mx, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 g((unsigned)((M + 255) / 256), (unsigned)N);
  if (tbytes == 1 && mx) {
    // the route of k_consumer_mx (expansion products)
    if (nd > 24 || (M + 63) / 64 * 64 > Mp) return hipErrorInvalidValue;
    dim3 gx((unsigned)((M + 63) / 64), (unsigned)N);
    if (nd <= 18)
      hipLaunchKernelGGL(k_crt_export_mx<36>, gx, dim3(64), 0, s, (const uint8_t *)tpl, Mp, Np, M,
                         N, pl, out, nlimb);
    else
      hipLaunchKernelGGL(k_crt_export_mx<48>, gx, dim3(64), 0, s, (const uint8_t *)tpl, Mp, Np, M,
                         N, pl, out, nlimb);
    return hipGetLastError();
  }
  if (tbytes == 1) {
    // the byte-column count of the consumers (launch_consumer, the limb
    // consumer): 36 up to 18 digits, else 48
    if (nd > 24) return hipErrorInvalidValue;
    if (nd <= 18)
      hipLaunchKernelGGL(k_crt_export_b<36>, g, dim3(256), 0, s, (const uint8_t *)tpl, Mp, Np, M,
                         N, pl, out, nlimb);
    else
      hipLaunchKernelGGL(k_crt_export_b<48>, g, dim3(256), 0, s, (const uint8_t *)tpl, Mp, Np, M,
                         N, pl, out, nlimb);
  } else {
    hipLaunchKernelGGL(k_crt_export<uint32_t>, g, dim3(256), 0, s, (const uint32_t *)tpl, Mp, Np,
                       M, N, pl, out, nlimb);
  }
  return hipGetLastError();
}

}  // namespace ozl
