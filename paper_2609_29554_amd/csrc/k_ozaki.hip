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

#include "expansion.hpp"
#include "ozii_elem.hpp"
#include "ozii_kernels.hpp"

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
template <int NC, int NWX, int NH>
__global__ __launch_bounds__(256) void k_producer(const double *X, int64_t ld, int rowwise,
                                                  int64_t nout, int64_t K, int64_t KB,
                                                  const int32_t *exps, const DevPlan *pl,
                                                  int8_t *planes, int64_t plane_bytes) {
  __shared__ uint32_t stage[256 * STG];
  uint32_t *st = stage + threadIdx.x * STG;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t kb = blockIdx.x, ob = blockIdx.y;
  const int nmod = pl->nmod, Q = pl->Q;
  for (int q = 0; q < 4; ++q) {
    const int64_t o = ob * 16 + 4 * q + (lane >> 4);
    const int64_t h = kb * 64 + 16 * wv + (lane & 15);
    const int64_t off = (ob * KB + kb) * 1024 + 64 * q + 256 * wv + lane;
    const double *src = nullptr;
    int mu = 0;
    if (o < nout && h < K) {
      const int32_t ex = exps[o];
      if (ex != EXP_ZERO) {
        src = rowwise ? X + (o + h * ld) * NC : X + (h + o * ld) * NC;
        mu = Q - 1 - ex;
      }
    }
    produce_element<NC, NWX, NH>(src, mu, pl, st, [&](int t, int l, int8_t r) {
      planes[(int64_t)(t * nmod + l) * plane_bytes + off] = r;
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
  const int gl = lt / (tilesN * tilesM);
  const int nmod = pl->nmod;
  const int l = gl % nmod, gi = gl / nmod;
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
  const int32_t m = pl->m[l];
  const double md = (double)m, yd = (double)pl->y[l], im = pl->inv_m[l];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      uint32_t packed = 0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double x = (double)acc[a][b][r] * yd;
        double qq = __builtin_floor(x * im);
        double rr = __builtin_fma(-qq, md, x);
        rr = rr < 0.0 ? rr + md : rr;
        rr = rr >= md ? rr - md : rr;
        packed |= ((uint32_t)rr & 0xffu) << (8 * r);
      }
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
// (S5)+(S6) consumer
// ---------------------------------------------------------------------------
template <int NC, int NWC, int ND>
__global__ __launch_bounds__(256) void k_consumer(const uint8_t *__restrict__ tpl, int64_t Mp,
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
  consume_element<NC, NWC, ND>(
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

// Debug export of the group sums: Sbar as 64-bit limbs (two's complement),
// layout [gi][j][i][limb], nlimb limbs.
__global__ __launch_bounds__(256) void k_crt_export(const uint8_t *__restrict__ tpl, int64_t Mp,
                                                    int64_t Np, int64_t M, int64_t N,
                                                    const DevPlan *pl, uint64_t *out, int nlimb) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i >= M || j >= N) return;
  const int nmod = pl->nmod;
  for (int gi = 0; gi < pl->ng; ++gi) {
    int32_t d[NDCRT];
    crt_digits<NDCRT>(tpl + ((int64_t)gi * nmod * Np + j) * Mp + i, Np * Mp, pl, d);
    uint64_t *o = out + (((int64_t)gi * N + j) * M + i) * nlimb;
    const uint64_t fill = d[NDCRT - 1] < 0 ? ~0ull : 0ull;
    for (int q = 0; q < nlimb; ++q) {
      uint64_t v = 0;
      if (4 * q + 3 < NDCRT) {
        for (int k = 0; k < 4; ++k) v |= ((uint64_t)((uint32_t)d[4 * q + k] & 0xffffu)) << (16 * k);
      } else {
        v = fill;
      }
      o[q] = v;
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
namespace ozl {

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

template <int NC, int NWX>
static void producer_nh(int nh, dim3 g, hipStream_t s, const double *X, int64_t ld, int rowwise,
                        int64_t nout, int64_t K, int64_t KB, const int32_t *exps,
                        const DevPlan *pl, int8_t *planes, int64_t plane_bytes) {
  if (nh <= 8)
    hipLaunchKernelGGL((k_producer<NC, NWX, 8>), g, dim3(256), 0, s, X, ld, rowwise, nout, K, KB,
                       exps, pl, planes, plane_bytes);
  else if (nh <= 12)
    hipLaunchKernelGGL((k_producer<NC, NWX, 12>), g, dim3(256), 0, s, X, ld, rowwise, nout, K, KB,
                       exps, pl, planes, plane_bytes);
  else
    hipLaunchKernelGGL((k_producer<NC, NWX, NHMAX>), g, dim3(256), 0, s, X, ld, rowwise, nout, K,
                       KB, exps, pl, planes, plane_bytes);
}

hipError_t launch_producer(int nc, int nwx, int nh, const double *X, int64_t ld, int rowwise,
                           int64_t nout, int64_t noutp, int64_t K, int64_t Kp,
                           const int32_t *exps, const DevPlan *pl, int8_t *planes,
                           int64_t plane_bytes, hipStream_t s) {
  const int64_t KB = Kp / 64, OB = noutp / 16;
  if (KB <= 0 || OB <= 0) return hipSuccess;
  dim3 g((unsigned)KB, (unsigned)OB);
#define OZ_PROD(NC_, NWX_) producer_nh<NC_, NWX_>(nh, g, s, X, ld, rowwise, nout, K, KB, exps, pl, planes, plane_bytes)
  if (nc == 2) { if (nwx <= 8) OZ_PROD(2, 8); else OZ_PROD(2, 12); }
  else if (nc == 3) { if (nwx <= 8) OZ_PROD(3, 8); else OZ_PROD(3, 12); }
  else { if (nwx <= 8) OZ_PROD(4, 8); else OZ_PROD(4, 12); }
#undef OZ_PROD
  return hipGetLastError();
}

hipError_t launch_gemm_i8(const int8_t *pa, const int8_t *pb, uint8_t *tpl, const DevPlan *pl,
                          int ng, int nmod, int64_t Mp, int64_t Np, int64_t Kp, int64_t planeA,
                          int64_t planeB, hipStream_t s) {
  const int tilesM = (int)(Mp / 128), tilesN = (int)(Np / 128);
  const int64_t nblk = (int64_t)ng * nmod * tilesM * tilesN;
  if (nblk <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gemm_i8, dim3((unsigned)nblk), dim3(256), 0, s, pa, pb, tpl, pl, Mp, Np,
                     Kp / 64, planeA, planeB, tilesM, tilesN);
  return hipGetLastError();
}

hipError_t launch_consumer(int nc, int nwc, int nd, const uint8_t *tpl, int64_t Mp, int64_t Np,
                           double *C, int64_t ldc, int64_t M, int64_t N, const int32_t *ea,
                           const int32_t *eb, const DevPlan *pl, int mode, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 g((unsigned)((M + 255) / 256), (unsigned)N);
#define OZ_CONS(NC_, NWC_, ND_)                                                             \
  hipLaunchKernelGGL((k_consumer<NC_, NWC_, ND_>), g, dim3(256), 0, s, tpl, Mp, Np, C, ldc, M, \
                     N, ea, eb, pl, mode)
#define OZ_CONS_ND(NC_, NWC_) \
  do { if (nd <= 18) OZ_CONS(NC_, NWC_, 18); else OZ_CONS(NC_, NWC_, 24); } while (0)
  if (nc == 2) { if (nwc <= 12) OZ_CONS_ND(2, 12); else OZ_CONS_ND(2, 16); }
  else if (nc == 3) { if (nwc <= 12) OZ_CONS_ND(3, 12); else OZ_CONS_ND(3, 16); }
  else { if (nwc <= 12) OZ_CONS_ND(4, 12); else OZ_CONS_ND(4, 16); }
#undef OZ_CONS_ND
#undef OZ_CONS
  return hipGetLastError();
}

hipError_t launch_crt_export(const uint8_t *tpl, int64_t Mp, int64_t Np, int64_t M, int64_t N,
                             const DevPlan *pl, uint64_t *out, int nlimb, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 g((unsigned)((M + 255) / 256), (unsigned)N);
  hipLaunchKernelGGL(k_crt_export, g, dim3(256), 0, s, tpl, Mp, Np, M, N, pl, out, nlimb);
  return hipGetLastError();
}

}  // namespace ozl
