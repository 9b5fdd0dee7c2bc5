// Batched LU + solve of many small, uneven matrices in one persistent launch
// (the batched configuration: 256 independent DD / QD systems of order 64 to
// 512).  Every workgroup takes matrices from a device work queue -- the host
// orders the batch by decreasing cost (longest-processing-time first) -- and
// factors and solves each one alone with the expansion arithmetic of
// expansion.hpp: unblocked right-looking LU with partial pivoting (LAPACK's
// i?amax, whole-row interchanges), then the solve with the factors.  Per
// element the operations come in exactly the order of ozII_getrf with b = 1
// and the native update, followed by ozII_getrs, so results match those (and
// the oracle) bit for bit.  The launch allocates nothing and clears its queue
// with a kernel, so it can be captured in a hipGraph.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ozii.h"
#include "expansion.hpp"
#include "ozii_elem.hpp"
#include "ozii_stage.hpp"

using namespace ozk;

typedef int v4i __attribute__((ext_vector_type(4)));

namespace {

constexpr int BT = 1024;  // threads per workgroup (4 wavefronts per SIMD)
constexpr int BTZ = 512;  // the same for the Ozaki-II update
constexpr int BZ_PRE = 10; // t-byte chunks requested at once by its CRT (nmod <= 40)

// The elements idx = t, t + NT, t + 2 NT, ... of a rectangle with mr > 0 rows
// taken column by column, (i, c) = (idx % mr, idx / mr), with one division
// per thread instead of one per element.
template <int NT>
struct ColWalk {
  int32_t i, c, di, dc, mr;
  __device__ ColWalk(int32_t rows, int32_t t)
      : i(t % rows), c(t / rows), di(NT % rows), dc(NT / rows), mr(rows) {}
  __device__ void next() {
    i += di;
    c += dc;
    if (i >= mr) {
      i -= mr;
      ++c;
    }
  }
};

// largest |value| first, then the lower row index (a total order)
template <int NC>
__device__ __forceinline__ bool piv_better(const double (&kb_)[NC], int64_t ib,
                                           const double (&ka)[NC], int64_t ia) {
  if (ib < 0) return false;
  if (ia < 0) return true;
  if (ozx::abs_greater<NC>(kb_, ka)) return true;
  if (ozx::abs_greater<NC>(ka, kb_)) return false;
  return ib < ia;
}

// Column j of the LU: pivot search over rows j..n-1 (largest magnitude, then
// the lower row index), ipiv and info, the whole-row interchange and the
// division of the column below the pivot (nothing to divide after a zero
// pivot: the column below it is zero).  Ends with the workgroup in step and
// returns whether the pivot was exactly zero (the same in every thread).
template <int NC, int NT>
__device__ bool pivot_column(const ozII_batch_item &it, int64_t j, double (*rkey)[4],
                             int64_t *ridx, int *s_info) {
  const int tid = threadIdx.x;
  const int64_t n = it.n;
  double *A = it.A;
  auto E = [&](int64_t i, int64_t c) { return A + (i + c * n) * NC; };
  double bk[NC];
  int64_t bi = -1;
#pragma unroll
  for (int q = 0; q < NC; ++q) bk[q] = 0.0;
  for (int64_t i = j + tid; i < n; i += NT) {
    double x[NC];
    ozx::load<NC>(E(i, j), x);
    if (piv_better<NC>(x, i, bk, bi)) {
#pragma unroll
      for (int q = 0; q < NC; ++q) bk[q] = x[q];
      bi = i;
    }
  }
  // the order is total, so any reduction order gives the same winner: a
  // butterfly inside each wavefront, then thread 0 over the wavefront winners
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    double kv[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) kv[q] = __shfl_xor(bk[q], off, 64);
    const int64_t iv = __shfl_xor(bi, off, 64);
    if (piv_better<NC>(kv, iv, bk, bi)) {
#pragma unroll
      for (int q = 0; q < NC; ++q) bk[q] = kv[q];
      bi = iv;
    }
  }
  if ((tid & 63) == 0) {
#pragma unroll
    for (int q = 0; q < NC; ++q) rkey[tid >> 6][q] = bk[q];
    ridx[tid >> 6] = bi;
  }
  __syncthreads();
  if (tid == 0) {
    for (int wv = 1; wv < NT / 64; ++wv) {
      double ka[NC], kv[NC];
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        ka[q] = rkey[0][q];
        kv[q] = rkey[wv][q];
      }
      if (piv_better<NC>(kv, ridx[wv], ka, ridx[0])) {
#pragma unroll
        for (int q = 0; q < NC; ++q) rkey[0][q] = kv[q];
        ridx[0] = ridx[wv];
      }
    }
  }
  __syncthreads();
  const int64_t p = ridx[0];
  bool zero = true;
#pragma unroll
  for (int q = 0; q < NC; ++q) zero = zero && (rkey[0][q] == 0.0);
  __syncthreads();
  if (tid == 0) {
    it.ipiv[j] = p;
    if (zero && *s_info == 0) *s_info = (int)(j + 1);
  }
  if (!zero) {
    if (p != j) {  // whole-row interchange
      for (int64_t c = tid; c < n; c += NT) {
        double u[NC], v[NC];
        ozx::load<NC>(E(j, c), u);
        ozx::load<NC>(E(p, c), v);
        ozx::store<NC>(E(j, c), v);
        ozx::store<NC>(E(p, c), u);
      }
      __syncthreads();
    }
    double d[NC];
    ozx::load<NC>(E(j, j), d);
    for (int64_t i = j + 1 + tid; i < n; i += NT) {
      double a[NC], l[NC];
      ozx::load<NC>(E(i, j), a);
      ozx::div<NC>(a, d, l);
      ozx::store<NC>(E(i, j), l);
    }
    __syncthreads();
  }
  return zero;
}

template <int NC, int NT>
__device__ void solve_one(const ozII_batch_item &it);

template <int NC>
__device__ void lu_solve_one(const ozII_batch_item &it, double (*rkey)[4], int64_t *ridx,
                             int *s_info) {
  const int tid = threadIdx.x;
  const int64_t n = it.n;
  double *A = it.A;
  auto E = [&](int64_t i, int64_t c) { return A + (i + c * n) * NC; };
  if (tid == 0) *s_info = 0;
  __syncthreads();
  for (int64_t j = 0; j < n; ++j) {
    pivot_column<NC, BT>(it, j, rkey, ridx, s_info);
    // rank-1 update of the trailing matrix (also after a zero pivot, with the
    // unscaled -- all-zero -- column, as the blocked LU with b = 1 does)
    const int64_t m = n - j - 1;
    ColWalk<BT> wk((int32_t)(m > 0 ? m : 1), tid);
    for (int64_t idx = tid; idx < m * m; idx += BT, wk.next()) {
      const int64_t i = j + 1 + wk.i, c = j + 1 + wk.c;
      double a[NC], l[NC], u[NC], o[NC];
      ozx::load<NC>(E(i, c), a);
      ozx::load<NC>(E(i, j), l);
      ozx::load<NC>(E(j, c), u);
      ozx::fms<NC>(a, l, u, o);
      ozx::store<NC>(E(i, c), o);
    }
    __syncthreads();
  }
  if (tid == 0) *it.info = *s_info;
  solve_one<NC, BT>(it);
}

// The solve with the factors: interchanges in ipiv order, forward (unit L,
// ascending), backward (descending, each x_k divided by u_kk once its
// updates are in), as ozII_getrs does for one right-hand side.
template <int NC, int NT>
__device__ void solve_one(const ozII_batch_item &it) {
  if (!it.b) return;
  const int tid = threadIdx.x;
  const int64_t n = it.n;
  double *A = it.A;
  auto E = [&](int64_t i, int64_t c) { return A + (i + c * n) * NC; };
  double *x = it.b;
  if (tid == 0)
    for (int64_t j = 0; j < n; ++j) {
      const int64_t p = it.ipiv[j];
      if (p != j) {
        double u[NC], v[NC];
        ozx::load<NC>(x + j * NC, u);
        ozx::load<NC>(x + p * NC, v);
        ozx::store<NC>(x + j * NC, v);
        ozx::store<NC>(x + p * NC, u);
      }
    }
  __syncthreads();
  for (int64_t k = 0; k < n; ++k) {
    double xk[NC];
    ozx::load<NC>(x + k * NC, xk);
    for (int64_t i = k + 1 + tid; i < n; i += NT) {
      double a[NC], l[NC], o[NC];
      ozx::load<NC>(x + i * NC, a);
      ozx::load<NC>(E(i, k), l);
      ozx::fms<NC>(a, l, xk, o);
      ozx::store<NC>(x + i * NC, o);
    }
    __syncthreads();
  }
  for (int64_t k = n - 1; k >= 0; --k) {
    if (tid == 0) {
      double u[NC], xk[NC], o[NC];
      ozx::load<NC>(E(k, k), u);
      ozx::load<NC>(x + k * NC, xk);
      ozx::div<NC>(xk, u, o);
      ozx::store<NC>(x + k * NC, o);
    }
    __syncthreads();
    double xk[NC];
    ozx::load<NC>(x + k * NC, xk);
    for (int64_t i = tid; i < k; i += NT) {
      double a[NC], u[NC], o[NC];
      ozx::load<NC>(x + i * NC, a);
      ozx::load<NC>(E(i, k), u);
      ozx::fms<NC>(a, u, xk, o);
      ozx::store<NC>(x + i * NC, o);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Blocked LU with the Ozaki-II Schur update, one system per workgroup
// (Sec. 3.4, Eq. (schur), with the product of Sec. 3.1-3.3 at K = b).  Per
// block of b columns: the panel (pivot_column and the rank-1 updates of the
// panel's own columns, whole-row interchanges), U12 = L11^-1 A12 (for
// k = k0 .. : a_ic -= l_ik u_kc over the rows below k of the block), then
// A22 -= L21 U12 by the stages of ozII_gemm run inside the workgroup:
//   (S1) row / column exponents into the scratch;
//   (S2)+(S3) produce_block_b, the 256-thread quarters taking the 16-row x
//        64-k blocks of L21 and U12 in turn;
//   (S4) every wavefront takes 64 x 64 tiles of the (group, modulus)
//        products: 4 x 4 MFMA 16x16x64 fragments, operands straight from
//        the scratch planes, the t-bytes stored as 4-byte column runs;
//   (S5)+(S6) one element per thread: consume_element_b and the expansion
//        subtraction.
// Per element the operations are those of ozII_getrf with the same b and
// method = Ozaki-II on the INT8 back-end, so the factors agree bit for bit.
//
// Scratch of one workgroup (Mp = m2 and Kp = b rounded up to 64): ea, eb
// (Mp int32 each), S nmod planes of L21 residues and S nmod planes of U12
// residues (Mp x Kp bytes each), ng nmod t-planes (Mp x Mp bytes each).
// ---------------------------------------------------------------------------
template <int NC, int NWM, int NT>
__device__ __forceinline__ void oz_update(double *A, int64_t n, int64_t k0, int64_t k1, const DevPlan *pl,
                          uint8_t *ws, uint32_t *stage) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t K = k1 - k0, m2 = n - k1;
  const int64_t Mp = (m2 + 63) & ~(int64_t)63, Kp = (K + 63) & ~(int64_t)63, KB = Kp / 64;
  const int S = pl->S, nmod = pl->nmod, ng = pl->ng, g0 = pl->g0, Q = pl->Q, w = pl->w;
  int32_t *ea = (int32_t *)ws;
  int32_t *eb = ea + Mp;
  const int64_t plane = Mp * Kp;
  uint8_t *pa = (uint8_t *)(eb + Mp);
  uint8_t *pb = pa + (int64_t)S * nmod * plane;
  uint8_t *tpl = pb + (int64_t)S * nmod * plane;
  const double *L21 = A + (k1 + k0 * n) * NC;  // m2 x K, leading dimension n
  const double *U12 = A + (k0 + k1 * n) * NC;  // K x m2
  double *A22 = A + (k1 + k1 * n) * NC;

  // (S1)
  for (int64_t i = tid; i < Mp; i += NT) {
    int32_t be = EXP_ZERO, bf = EXP_ZERO;
    if (i < m2)
      for (int64_t h = 0; h < K; ++h) {
        const int32_t u = exponent_of<NC>(L21 + (i + h * n) * NC);
        const int32_t v = exponent_of<NC>(U12 + (h + i * n) * NC);
        be = u > be ? u : be;
        bf = v > bf ? v : bf;
      }
    ea[i] = be;
    eb[i] = bf;
  }
  __syncthreads();

  // (S2)+(S3)
  {
    const int T = tid & 255;
    const int64_t NBLK = Mp / 16 * KB;  // blocks per operand
    for (int64_t q = tid >> 8; q < 2 * NBLK; q += NT / 256) {
      const bool isA = q < NBLK;
      const int64_t r = isA ? q : q - NBLK;
      produce_block_b<NC, 8, NWM, PL_I8>(isA ? L21 : U12, n, isA ? 1 : 0, m2, K, KB,
                                         isA ? ea : eb, pl, isA ? pa : pb, plane, r % KB, r / KB,
                                         T, 0, pl->nmod);
    }
  }
  __syncthreads();

  // (S4)
  {
    const int64_t TM = Mp / 64;
    const int64_t items = (int64_t)ng * nmod * TM * TM;
    for (int64_t q = wv; q < items; q += NT / 64) {
      const int64_t tn = q % TM, tm = (q / TM) % TM;
      const int gl = (int)(q / (TM * TM));
      const int l = gl % nmod, g = g0 + gl / nmod;
      const int ta0 = g - (S - 1) > 0 ? g - (S - 1) : 0;
      const int ta1 = g < S - 1 ? g : S - 1;
      v4i acc[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = v4i{0, 0, 0, 0};
      for (int ta = ta0; ta <= ta1; ++ta) {
        const uint8_t *A0 = pa + (int64_t)(ta * nmod + l) * plane + tm * 4 * KB * 1024 + lane * 16;
        const uint8_t *B0 =
            pb + (int64_t)((g - ta) * nmod + l) * plane + tn * 4 * KB * 1024 + lane * 16;
        for (int64_t kb = 0; kb < KB; ++kb) {
          v4i af[4], bf[4];
#pragma unroll
          for (int a = 0; a < 4; ++a) af[a] = *(const v4i *)(A0 + (a * KB + kb) * 1024);
#pragma unroll
          for (int b = 0; b < 4; ++b) bf[b] = *(const v4i *)(B0 + (b * KB + kb) * 1024);
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
              acc[a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[a], bf[b], acc[a][b], 0, 0, 0);
        }
      }
      const uint32_t m = (uint32_t)pl->m[l];
      const double md = (double)m, yd = (double)pl->y[l], im = pl->inv_m[l];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          uint32_t packed = 0;
#pragma unroll
          for (int r = 0; r < 4; ++r) packed |= mod_times_y(acc[a][b][r], md, yd, im, m) << (8 * r);
          const int64_t row = tm * 64 + 16 * a + 4 * (lane >> 4);
          const int64_t col = tn * 64 + 16 * b + (lane & 15);
          *(uint32_t *)(tpl + ((int64_t)gl * Mp + col) * Mp + row) = packed;
        }
    }
  }
  __syncthreads();

  // (S5)+(S6) and A22 -= c: each wavefront takes 64 consecutive elements of
  // a column at a time through the matrix-core CRT, on its own slice of the
  // staging LDS (the route and results of k_consumer_mx)
  {
    constexpr int NB = 36, NWC = 12, ND = NB / 2, STG = stage_words<ND>();
    static_assert(64 * MX_TBS <= 32 * MX_CBS * 4 && 64 * STG <= 32 * MX_CBS, "LDS reuse");
    static_assert(NT / 64 * 32 * MX_CBS <= NT * CST, "one column-sum buffer per wavefront");
    int32_t *buf = (int32_t *)stage + wv * 32 * MX_CBS;
    uint32_t *st = (uint32_t *)buf + lane * STG;
    mxv4 tab[MX_BLK];
#pragma unroll
    for (int b = 0; b < MX_BLK; ++b) tab[b] = *(const mxv4 *)&pl->crtm[b][lane][0];
    const int64_t TMB = Mp / 64, ps = Mp * Mp;
    for (int64_t ch = wv; ch < m2 * TMB; ch += NT / 64) {
      const int64_t j = ch / TMB, i0 = (ch % TMB) * 64, i = i0 + lane;
      const bool valid = i < m2;
      const int32_t ej = eb[j], ei = valid ? ea[i] : EXP_ZERO;
      const bool zero = ei == EXP_ZERO || ej == EXP_ZERO;
      const int eps = zero ? 0 : w * g0 - (Q - 1 - ei) - (Q - 1 - ej);
      uint32_t cb[NWC];
#pragma unroll
      for (int k = 0; k < NWC; ++k) cb[k] = 0u;
      for (int gi = 0; gi < ng; ++gi) {
        int32_t d[ND];
        crt_group_mx<NB, true>(tpl + (int64_t)gi * nmod * ps + j * Mp + i0, ps, nmod, pl, tab, buf,
                               lane, d);
        add_shifted_digits<NWC, ND, STG>(cb, d, w * gi, st);
        mx_sync<true>();  // the buffer takes the next group's t-bytes
      }
      if (!valid) continue;
      double c[NC];
      if (zero) {
#pragma unroll
        for (int q = 0; q < NC; ++q) c[q] = 0.0;
      } else {
        round_out_n<NWC, NC>(cb, eps, c);
      }
      double *dst = A22 + (i + j * n) * NC;
      double a[NC], nc_[NC], r[NC];
      ozx::load<NC>(dst, a);
#pragma unroll
      for (int q = 0; q < NC; ++q) nc_[q] = -c[q];
      ozx::add<NC>(a, nc_, r);
      ozx::store<NC>(dst, r);
    }
  }
  __syncthreads();
}

// a <- a - l u for the elements idx = 0 .. total-1 of one step (where(idx)
// gives the three operands; a is updated in place), two elements per
// thread in flight: both elements' loads are issued before the first
// multiply-subtract, so one memory round trip serves two of them (the
// Ozaki-II workgroup has half the wavefronts of the native one).  Each
// element is updated once, so the order of its updates is the caller's.
template <int NC, int NT, typename W>
__device__ __forceinline__ void fms_sweep(int64_t total, W where) {
  for (int64_t idx = threadIdx.x; idx < total; idx += 2 * NT) {
    const bool two = idx + NT < total;
    double *pa0, *pa1 = nullptr;
    const double *pl0, *pu0, *pl1 = nullptr, *pu1 = nullptr;
    where(idx, pa0, pl0, pu0);
    if (two) where(idx + NT, pa1, pl1, pu1);
    double a0[NC], l0[NC], u0[NC], a1[NC] = {}, l1[NC] = {}, u1[NC] = {}, o[NC];
    ozx::load<NC>(pa0, a0);
    ozx::load<NC>(pl0, l0);
    ozx::load<NC>(pu0, u0);
    if (two) {
      ozx::load<NC>(pa1, a1);
      ozx::load<NC>(pl1, l1);
      ozx::load<NC>(pu1, u1);
    }
    ozx::fms<NC>(a0, l0, u0, o);
    ozx::store<NC>(pa0, o);
    if (two) {
      ozx::fms<NC>(a1, l1, u1, o);
      ozx::store<NC>(pa1, o);
    }
  }
}

template <int NC, int NWM, int NT>
__device__ __forceinline__ void lu_solve_oz(const ozII_batch_item &it, double (*rkey)[4], int64_t *ridx,
                            int *s_info, const DevPlan *pl, uint8_t *ws, int b,
                            uint32_t *stage) {
  const int tid = threadIdx.x;
  const int64_t n = it.n;
  double *A = it.A;
  auto E = [&](int64_t i, int64_t c) { return A + (i + c * n) * NC; };
  if (tid == 0) *s_info = 0;
  __syncthreads();
  for (int64_t k0 = 0; k0 < n; k0 += b) {
    const int64_t k1 = k0 + b < n ? k0 + b : n;
    for (int64_t j = k0; j < k1; ++j) {
      // rank-1 update of the panel's own columns j+1 .. k1-1; none after an
      // exactly zero pivot (the column is left as it is, as in LAPACK's
      // unblocked panel)
      const bool zero = pivot_column<NC, NT>(it, j, rkey, ridx, s_info);
      const int64_t mr = zero ? 0 : n - j - 1, mc = k1 - j - 1;
      fms_sweep<NC, NT>(mr * mc, [&](int64_t idx, double *&pa, const double *&pl,
                                     const double *&pu) {
        const int64_t i = j + 1 + idx % mr, c = j + 1 + idx / mr;
        pa = E(i, c);
        pl = E(i, j);
        pu = E(j, c);
      });
      __syncthreads();
    }
    if (k1 < n) {
      // U12 = L11^-1 A12, forward in k
      const int64_t ncol = n - k1;
      for (int64_t k = k0; k + 1 < k1; ++k) {
        const int64_t mr = k1 - k - 1;
        fms_sweep<NC, NT>(mr * ncol, [&](int64_t idx, double *&pa, const double *&pl,
                                         const double *&pu) {
          const int64_t i = k + 1 + idx % mr, c = k1 + idx / mr;
          pa = E(i, c);
          pl = E(i, k);
          pu = E(k, c);
        });
        __syncthreads();
      }
      oz_update<NC, NWM, NT>(A, n, k0, k1, pl, ws, stage);
    }
  }
  if (tid == 0) *it.info = *s_info;
  solve_one<NC, NT>(it);
}

// One workgroup of BTZ threads per CU (the update's stages need more than
// the 128 registers a 1024-thread workgroup leaves per thread); the
// consumer's per-thread staging shares the LDS with the pivot search (never
// live at the same time).
__global__ __launch_bounds__(BTZ) void k_batch_lu_oz(const ozII_batch_item *items, int count,
                                                    int *queue, uint64_t *times,
                                                    const DevPlan *pl2, const DevPlan *pl3,
                                                    const DevPlan *pl4, uint8_t *ws, int64_t slot,
                                                    int b) {
  __shared__ __attribute__((aligned(16))) uint32_t lds[BTZ * CST];
  static_assert(BTZ * CST * 4 >= BTZ * (32 + 8), "pivot search arrays fit the staging");
  double(*rkey)[4] = (double(*)[4])lds;
  int64_t *ridx = (int64_t *)(lds + BTZ * 8);
  __shared__ int s_item, s_info;
  uint8_t *myws = ws + (int64_t)blockIdx.x * slot;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(queue, 1);
    __syncthreads();
    const int q = s_item;
    __syncthreads();
    if (q >= count) break;  // every workgroup leaves once the queue is empty
    const ozII_batch_item it = items[q];
    if (times && threadIdx.x == 0) times[2 * it.reserved] = __builtin_amdgcn_s_memrealtime();
    if (it.nc == 2) lu_solve_oz<2, 6, BTZ>(it, rkey, ridx, &s_info, pl2, myws, b, lds);
    else if (it.nc == 3) lu_solve_oz<3, 4, BTZ>(it, rkey, ridx, &s_info, pl3, myws, b, lds);
    else lu_solve_oz<4, 4, BTZ>(it, rkey, ridx, &s_info, pl4, myws, b, lds);
    __syncthreads();
    if (times && threadIdx.x == 0) {
      __builtin_amdgcn_s_waitcnt(0x0F70);
      times[2 * it.reserved + 1] = __builtin_amdgcn_s_memrealtime();
    }
  }
}

__global__ __launch_bounds__(BT) void k_batch_lu(const ozII_batch_item *items, int count,
                                                 int *queue, uint64_t *times) {
  __shared__ double rkey[BT][4];
  __shared__ int64_t ridx[BT];
  __shared__ int s_item, s_info;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(queue, 1);
    __syncthreads();
    const int q = s_item;
    __syncthreads();
    if (q >= count) break;  // every workgroup leaves once the queue is empty
    const ozII_batch_item it = items[q];  // reserved = the item's index in the caller's order
    if (times && threadIdx.x == 0) times[2 * it.reserved] = __builtin_amdgcn_s_memrealtime();
    if (it.nc == 2) lu_solve_one<2>(it, rkey, ridx, &s_info);
    else if (it.nc == 3) lu_solve_one<3>(it, rkey, ridx, &s_info);
    else lu_solve_one<4>(it, rkey, ridx, &s_info);
    __syncthreads();
    if (times && threadIdx.x == 0) {
      // the item's global writes are complete before its end stamp
      __builtin_amdgcn_s_waitcnt(0x0F70);
      times[2 * it.reserved + 1] = __builtin_amdgcn_s_memrealtime();
    }
  }
}

__global__ void k_batch_clear(int *queue) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *queue = 0;
}

}  // namespace

namespace ozl {
hipError_t launch_batch(const ozII_batch_item *items, int count, int *queue, uint64_t *times,
                        int grid, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_clear, dim3(1), dim3(64), 0, s, queue);
  hipLaunchKernelGGL(k_batch_lu, dim3((unsigned)grid), dim3(BT), 0, s, items, count, queue, times);
  return hipGetLastError();
}
hipError_t launch_batch_oz(const ozII_batch_item *items, int count, int *queue, uint64_t *times,
                          int grid, const DevPlan *pl2, const DevPlan *pl3, const DevPlan *pl4,
                          uint8_t *ws, int64_t slot, int b, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (b < 1 || b > 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_batch_clear, dim3(1), dim3(64), 0, s, queue);
  hipLaunchKernelGGL(k_batch_lu_oz, dim3((unsigned)grid), dim3(BTZ), 0, s, items, count, queue,
                     times, pl2, pl3, pl4, ws, slot, b);
  return hipGetLastError();
}
}  // namespace ozl
