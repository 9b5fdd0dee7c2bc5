// The LU with partial pivoting on limb matrices outside the Ozaki-II
// product (Sec. 3.4; the solve of Sec. 4.3), in the p-bit arithmetic of
// limbfp.hpp: one wavefront per element operation, lane q handling limb q.
//
//   panel, per column j:  k_lpiv (per-workgroup candidates: largest exact
//     magnitude, lowest row on ties) -> k_lpiv_final (the pivot, ipiv, info,
//     the interchange inside the panel) -> k_ldiv (l = RN(a / pivot)) ->
//     k_lrank1 (RN(a - RN(l u)) on the panel's remaining columns);
//   k_llaswp: the panel's interchanges on the other columns, in order;
//   k_ltrsm:  B <- L^-1 B for a unit lower triangle (the U12 solve and the
//     leaves of its recursive form), one workgroup per column, k ascending;
//   k_lschur_naive: the native update RN(a - RN(l_ik u_kj)), k ascending, on
//     any block (the Schur update, or the inner updates of the recursion);
//   getrs: the interchanges, then blocks of LBLK rows: the diagonal block
//     by one workgroup per right-hand side, the rows below (forward) or
//     above (backward) by one wavefront each, every element taking its
//     multiply-subtracts in the order of column-oriented substitution and
//     x_k = RN(x_k / u_kk) once its updates are in.
// A zero pivot skips its column's division and update (LAPACK's panel).
// Every kernel hands work out per wavefront, so each wavefront stays
// converged through the cross-lane arithmetic.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lanes.hpp"
#include "limbfp.hpp"
#include "ozii_kernels.hpp"

using lfp::WF;
using ozl::LimbMat;

namespace {

constexpr int LBLK = 16;  // rows per diagonal block of the substitutions
constexpr int WPB = 4;    // wavefronts per 256-thread workgroup

__device__ __forceinline__ WF ld_el(const LimbMat &A, int64_t i, int64_t j, int nl) {
  const int l = lfp::lane_id();
  const int64_t idx = i + j * A.ld;
  uint64_t m = 0;
  if (l < nl) m = A.limb[(int64_t)l * A.plane + idx];
  const bool z = lfp::ballot(m != 0) == 0;
  WF x;
  x.m = m;
  x.e = z ? lfp::EXP_ZERO : A.exp[idx];
  x.s = z ? 0u : (uint32_t)(A.sign[idx] & 1u);
  return x;
}

__device__ __forceinline__ void st_el(const LimbMat &A, int64_t i, int64_t j, int nl,
                                      const WF &x) {
  const int l = lfp::lane_id();
  const int64_t idx = i + j * A.ld;
  if (l < nl) A.limb[(int64_t)l * A.plane + idx] = x.m;
  if (l == 0) {
    A.exp[idx] = x.e;
    A.sign[idx] = (uint8_t)x.s;
  }
}

__device__ __forceinline__ void swap_el(const LimbMat &A, int64_t i1, int64_t i2, int64_t j,
                                        int nl) {
  const int l = lfp::lane_id();
  const int64_t a = i1 + j * A.ld, b = i2 + j * A.ld;
  if (l < nl) {
    uint64_t *p = A.limb + (int64_t)l * A.plane;
    const uint64_t t = p[a];
    p[a] = p[b];
    p[b] = t;
  }
  if (l == 0) {
    const int32_t te = A.exp[a];
    A.exp[a] = A.exp[b];
    A.exp[b] = te;
    const uint8_t ts = A.sign[a];
    A.sign[a] = A.sign[b];
    A.sign[b] = ts;
  }
}

__device__ __forceinline__ int wave_in_block() { return (int)(threadIdx.x >> 6); }
__device__ __forceinline__ int waves_in_block() { return (int)(blockDim.x >> 6); }
__device__ __forceinline__ int64_t wave_global() {
  return (int64_t)blockIdx.x * waves_in_block() + wave_in_block();
}
__device__ __forceinline__ int64_t waves_total() { return (int64_t)gridDim.x * waves_in_block(); }

// keep (r, x) when |x| is larger, or equal with a lower row
__device__ __forceinline__ void take_max(int64_t &b, WF &v, int64_t r, const WF &x) {
  const int c = b < 0 ? 1 : lfp::cmp_abs(x, v);
  if (c > 0 || (c == 0 && r < b)) {
    b = r;
    v = x;
  }
}

__global__ __launch_bounds__(256) void k_lpiv(LimbMat A, int nl, int64_t j, int64_t n,
                                              int64_t *cand) {
  __shared__ int64_t srow[WPB];
  const int w = wave_in_block();
  int64_t best = -1;
  WF bv = lfp::wf_zero();
  for (int64_t r = j + wave_global(); r < n; r += waves_total()) take_max(best, bv, r, ld_el(A, r, j, nl));
  if (lfp::lane_id() == 0) srow[w] = best;
  __syncthreads();
  if (w == 0) {
    int64_t b = -1;
    WF v = lfp::wf_zero();
    for (int k = 0; k < WPB; ++k) {
      const int64_t r = srow[k];
      if (r >= 0) take_max(b, v, r, ld_el(A, r, j, nl));
    }
    if (lfp::lane_id() == 0) cand[blockIdx.x] = b;
  }
}

// The pivot among the per-workgroup candidates: 16 wavefronts take up to
// four candidates each, then a tournament through LDS (greatest |value|,
// lowest row on ties); ipiv, info, the zero flag and the interchange across
// the panel's columns [c0, c1).
constexpr int FIN_WAVES = 16;
constexpr int FIN_PER = ozl::LPIV_MAXGRID / FIN_WAVES;  // candidates per wavefront
__global__ __launch_bounds__(1024) void k_lpiv_final(LimbMat A, int nl, int64_t j,
                                                     const int64_t *cand, int ncand, int64_t c0,
                                                     int64_t c1, int64_t *ipiv, int32_t *info,
                                                     int32_t *zflag) {
  __shared__ uint64_t sm[FIN_WAVES][64];
  __shared__ int64_t srow[FIN_WAVES];
  __shared__ int32_t se[FIN_WAVES];
  __shared__ uint32_t ss[FIN_WAVES];
  const int w = wave_in_block(), l = lfp::lane_id();
  int64_t b = -1;
  WF v = lfp::wf_zero();
  // this wavefront's (up to FIN_PER) candidates: all loads issued first
  int64_t rr[FIN_PER];
  uint64_t mm[FIN_PER];
#pragma unroll
  for (int t = 0; t < FIN_PER; ++t) {
    const int k = w + t * FIN_WAVES;
    rr[t] = k < ncand ? cand[k] : -1;
  }
#pragma unroll
  for (int t = 0; t < FIN_PER; ++t)
    mm[t] = (rr[t] >= 0 && l < nl) ? A.limb[(int64_t)l * A.plane + rr[t] + j * A.ld] : 0ull;
#pragma unroll
  for (int t = 0; t < FIN_PER; ++t) {
    if (rr[t] < 0) continue;
    const int64_t idx = rr[t] + j * A.ld;
    WF x;
    x.m = mm[t];
    const bool z = lfp::ballot(x.m != 0) == 0;
    x.e = z ? lfp::EXP_ZERO : A.exp[idx];
    x.s = z ? 0u : (uint32_t)(A.sign[idx] & 1u);
    take_max(b, v, rr[t], x);
  }
  sm[w][l] = v.m;
  if (l == 0) {
    srow[w] = b;
    se[w] = v.e;
    ss[w] = v.s;
  }
  __syncthreads();
  for (int step = 1; step < FIN_WAVES; step *= 2) {
    if ((w & (2 * step - 1)) == 0) {
      const int o = w + step;
      const int64_t r = srow[o];
      if (r >= 0) {
        WF x;
        x.m = sm[o][l];
        x.e = se[o];
        x.s = ss[o];
        take_max(b, v, r, x);
      }
    }
    __syncthreads();
    if ((w & (2 * step - 1)) == 0) {
      sm[w][l] = v.m;
      if (l == 0) {
        srow[w] = b;
        se[w] = v.e;
        ss[w] = v.s;
      }
    }
    __syncthreads();
  }
  if (w == 0 && l == 0) {
    ipiv[j] = b;
    const int32_t z = lfp::is_zero(v) ? 1 : 0;
    zflag[0] = z;
    if (z && info[0] == 0) info[0] = (int32_t)(j + 1);
  }
  const int64_t r = srow[0];
  if (r != j)
    for (int64_t c = c0 + w; c < c1; c += FIN_WAVES) swap_el(A, j, r, c, nl);
}

// rows j <-> ipiv[j] on columns [s0, s1), one wavefront per column
__global__ __launch_bounds__(256) void k_lswap(LimbMat A, int nl, int64_t j, const int64_t *ipiv,
                                               int64_t s0, int64_t s1) {
  const int64_t r = ipiv[j];
  if (r == j) return;
  for (int64_t c = s0 + wave_global(); c < s1; c += waves_total()) swap_el(A, j, r, c, nl);
}

__global__ __launch_bounds__(256) void k_ldiv(LimbMat A, int nl, int64_t j, int64_t n,
                                              const int32_t *zflag) {
  if (*zflag) return;
  const WF pv = ld_el(A, j, j, nl);
  for (int64_t i = j + 1 + wave_global(); i < n; i += waves_total())
    st_el(A, i, j, nl, lfp::div(ld_el(A, i, j, nl), pv, nl));
}

__global__ __launch_bounds__(256) void k_lrank1(LimbMat A, int nl, int64_t j, int64_t n,
                                                int64_t c1, const int32_t *zflag) {
  if (*zflag) return;
  const int64_t rows = n - j - 1, cnt = rows * (c1 - j - 1);
  for (int64_t t = wave_global(); t < cnt; t += waves_total()) {
    const int64_t i = j + 1 + t % rows, c = j + 1 + t / rows;
    const WF a = ld_el(A, i, c, nl), lv = ld_el(A, i, j, nl), u = ld_el(A, j, c, nl);
    st_el(A, i, c, nl, lfp::fms(a, lv, u, nl));
  }
}

// rows jj <-> ipiv[jj] for jj = k0 .. k0+kb-1 in order, on columns
// [ca0, ca1) and [cb0, cb1); one wavefront per column
__global__ __launch_bounds__(256) void k_llaswp(LimbMat A, int nl, const int64_t *ipiv, int64_t k0,
                                                int64_t kb, int64_t ca0, int64_t ca1, int64_t cb0,
                                                int64_t cb1) {
  const int64_t na = ca1 - ca0, cnt = na + (cb1 - cb0);
  for (int64_t t = wave_global(); t < cnt; t += waves_total()) {
    const int64_t c = t < na ? ca0 + t : cb0 + (t - na);
    for (int64_t jj = k0; jj < k0 + kb; ++jj) {
      const int64_t r = ipiv[jj];
      if (r != jj) swap_el(A, jj, r, c, nl);
    }
  }
}

// B = A[r0:r0+h, b0:b1] <- L^-1 B for the unit lower triangle L at (r0, r0):
// one workgroup per column, k ascending, the rows below k over its waves
__global__ __launch_bounds__(1024) void k_ltrsm(LimbMat A, int nl, int64_t r0, int64_t h,
                                                int64_t b0, int64_t b1) {
  const int w = wave_in_block(), nw = waves_in_block();
  for (int64_t c = b0 + blockIdx.x; c < b1; c += gridDim.x) {
    for (int64_t k = 0; k + 1 < h; ++k) {
      const WF u = ld_el(A, r0 + k, c, nl);
      for (int64_t i = k + 1 + w; i < h; i += nw) {
        const WF a = ld_el(A, r0 + i, c, nl), lv = ld_el(A, r0 + i, r0 + k, nl);
        st_el(A, r0 + i, c, nl, lfp::fms(a, lv, u, nl));
      }
      __syncthreads();
    }
  }
}

// A[i0:i1, c0:c1] -= A[i0:i1, k0:k0+K] A[k0:k0+K, c0:c1] by multiply-subtracts,
// k ascending; one wavefront per element
__global__ __launch_bounds__(256) void k_lschur_naive(LimbMat A, int nl, int64_t i0, int64_t i1,
                                                      int64_t c0, int64_t c1, int64_t k0,
                                                      int64_t K) {
  const int64_t m = i1 - i0, cnt = m * (c1 - c0);
  for (int64_t t = wave_global(); t < cnt; t += waves_total()) {
    const int64_t i = i0 + t % m, c = c0 + t / m;
    WF a = ld_el(A, i, c, nl);
    for (int64_t k = k0; k < k0 + K; ++k)
      a = lfp::fms(a, ld_el(A, i, k, nl), ld_el(A, k, c, nl), nl);
    st_el(A, i, c, nl, a);
  }
}

// forward substitution, diagonal block [k0, k1); blockIdx.x = right-hand side
__global__ __launch_bounds__(1024) void k_lfwd_diag(LimbMat LU, LimbMat X, int nl, int64_t k0,
                                                    int64_t k1) {
  const int64_t r = blockIdx.x;
  const int w = wave_in_block(), nw = waves_in_block();
  for (int64_t k = k0; k + 1 < k1; ++k) {
    const WF xk = ld_el(X, k, r, nl);
    for (int64_t i = k + 1 + w; i < k1; i += nw)
      st_el(X, i, r, nl, lfp::fms(ld_el(X, i, r, nl), ld_el(LU, i, k, nl), xk, nl));
    __syncthreads();
  }
}

// forward substitution, rows [k1, n) after the block [k0, k1); blockIdx.y = rhs
__global__ __launch_bounds__(256) void k_lfwd_rest(LimbMat LU, LimbMat X, int nl, int64_t k0,
                                                   int64_t k1, int64_t n) {
  const int64_t r = blockIdx.y;
  for (int64_t i = k1 + wave_global(); i < n; i += waves_total()) {
    WF x = ld_el(X, i, r, nl);
    for (int64_t k = k0; k < k1; ++k) x = lfp::fms(x, ld_el(LU, i, k, nl), ld_el(X, k, r, nl), nl);
    st_el(X, i, r, nl, x);
  }
}

// backward substitution, diagonal block [k0, k1), k descending
__global__ __launch_bounds__(1024) void k_lbwd_diag(LimbMat LU, LimbMat X, int nl, int64_t k0,
                                                    int64_t k1) {
  const int64_t r = blockIdx.x;
  const int w = wave_in_block(), nw = waves_in_block();
  for (int64_t k = k1 - 1; k >= k0; --k) {
    if (w == 0) st_el(X, k, r, nl, lfp::div(ld_el(X, k, r, nl), ld_el(LU, k, k, nl), nl));
    __syncthreads();
    const WF xk = ld_el(X, k, r, nl);
    for (int64_t i = k0 + w; i < k; i += nw)
      st_el(X, i, r, nl, lfp::fms(ld_el(X, i, r, nl), ld_el(LU, i, k, nl), xk, nl));
    __syncthreads();
  }
}

// backward substitution, rows [0, k0) after the block [k0, k1)
__global__ __launch_bounds__(256) void k_lbwd_rest(LimbMat LU, LimbMat X, int nl, int64_t k0,
                                                   int64_t k1) {
  const int64_t r = blockIdx.y;
  for (int64_t i = wave_global(); i < k0; i += waves_total()) {
    WF x = ld_el(X, i, r, nl);
    for (int64_t k = k1 - 1; k >= k0; --k)
      x = lfp::fms(x, ld_el(LU, i, k, nl), ld_el(X, k, r, nl), nl);
    st_el(X, i, r, nl, x);
  }
}

// elementwise a op b on vectors (element t at index t): 0 add, 1 sub, 2 mul, 3 div
__global__ __launch_bounds__(256) void k_larith(int op, int nl, int64_t cnt, LimbMat A, LimbMat B,
                                                LimbMat C) {
  for (int64_t t = wave_global(); t < cnt; t += waves_total()) {
    const WF a = ld_el(A, t, 0, nl), b = ld_el(B, t, 0, nl);
    WF r;
    if (op == 0) r = lfp::add(a, b, 0u, nl);
    else if (op == 1) r = lfp::add(a, b, 1u, nl);
    else if (op == 2) r = lfp::mul(a, b, nl);
    else r = lfp::div(a, b, nl);
    st_el(C, t, 0, nl, r);
  }
}

__global__ void k_lfill_i32(int32_t *p, int32_t v, int count) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < count) p[i] = v;
}

// workgroups for `waves` independent wavefront tasks
int grid_for(int64_t waves, int64_t cap = 8192) {
  int64_t g = (waves + WPB - 1) / WPB;
  if (g < 1) g = 1;
  return (int)(g < cap ? g : cap);
}

}  // namespace

namespace ozl {

int lpiv_grid(int64_t rows) {
  int64_t g = (rows + 7) / 8;  // at least two rows per wavefront
  if (g < 1) g = 1;
  return (int)(g < LPIV_MAXGRID ? g : LPIV_MAXGRID);
}

hipError_t launch_lpanel_column(LimbMat A, int nl, int64_t j, int64_t n, int64_t s0, int64_t s1,
                                int64_t c1, int64_t *cand, int64_t *ipiv, int32_t *info,
                                int32_t *zflag, hipStream_t s) {
  const int g = lpiv_grid(n - j);
  hipLaunchKernelGGL(k_lpiv, dim3(g), dim3(256), 0, s, A, nl, j, n, cand);
  // a wide interchange runs on one wavefront per column after the reduction
  const bool wide = s1 - s0 > FIN_WAVES * 4;
  hipLaunchKernelGGL(k_lpiv_final, dim3(1), dim3(64 * FIN_WAVES), 0, s, A, nl, j,
                     (const int64_t *)cand, g, s0, wide ? s0 : s1, ipiv, info, zflag);
  if (wide)
    hipLaunchKernelGGL(k_lswap, dim3(grid_for(s1 - s0)), dim3(256), 0, s, A, nl, j,
                       (const int64_t *)ipiv, s0, s1);
  if (j + 1 < n) {
    hipLaunchKernelGGL(k_ldiv, dim3(grid_for(n - j - 1)), dim3(256), 0, s, A, nl, j, n,
                       (const int32_t *)zflag);
    if (j + 1 < c1)
      hipLaunchKernelGGL(k_lrank1, dim3(grid_for((n - j - 1) * (c1 - j - 1))), dim3(256), 0, s, A,
                         nl, j, n, c1, (const int32_t *)zflag);
  }
  return hipGetLastError();
}

hipError_t launch_llaswp(LimbMat A, int nl, const int64_t *ipiv, int64_t k0, int64_t kb,
                         int64_t ca0, int64_t ca1, int64_t cb0, int64_t cb1, hipStream_t s) {
  const int64_t cnt = (ca1 - ca0) + (cb1 - cb0);
  if (cnt <= 0 || kb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_llaswp, dim3(grid_for(cnt)), dim3(256), 0, s, A, nl, ipiv, k0, kb, ca0, ca1,
                     cb0, cb1);
  return hipGetLastError();
}

hipError_t launch_ltrsm(LimbMat A, int nl, int64_t r0, int64_t h, int64_t b0, int64_t b1,
                        hipStream_t s) {
  const int64_t cols = b1 - b0;
  if (cols <= 0 || h <= 1) return hipSuccess;
  hipLaunchKernelGGL(k_ltrsm, dim3((unsigned)(cols < 65535 ? cols : 65535)), dim3(1024), 0, s, A,
                     nl, r0, h, b0, b1);
  return hipGetLastError();
}

hipError_t launch_lschur_naive(LimbMat A, int nl, int64_t i0, int64_t i1, int64_t c0, int64_t c1,
                               int64_t k0, int64_t K, hipStream_t s) {
  const int64_t cnt = (i1 - i0) * (c1 - c0);
  if (i1 <= i0 || c1 <= c0 || K <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lschur_naive, dim3(grid_for(cnt)), dim3(256), 0, s, A, nl, i0, i1, c0, c1,
                     k0, K);
  return hipGetLastError();
}

hipError_t launch_lgetrs(LimbMat LU, int nl, int64_t n, const int64_t *ipiv, LimbMat X,
                         int64_t nrhs, hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_llaswp, dim3(grid_for(nrhs)), dim3(256), 0, s, X, nl, ipiv, (int64_t)0, n,
                     (int64_t)0, nrhs, (int64_t)0, (int64_t)0);
  for (int64_t k0 = 0; k0 < n; k0 += LBLK) {
    const int64_t k1 = k0 + LBLK < n ? k0 + LBLK : n;
    hipLaunchKernelGGL(k_lfwd_diag, dim3((unsigned)nrhs), dim3(1024), 0, s, LU, X, nl, k0, k1);
    if (k1 < n)
      hipLaunchKernelGGL(k_lfwd_rest, dim3(grid_for(n - k1, 2048), (unsigned)nrhs), dim3(256), 0, s,
                         LU, X, nl, k0, k1, n);
  }
  for (int64_t k1 = n; k1 > 0;) {
    const int64_t k0 = k1 - LBLK > 0 ? k1 - LBLK : 0;
    hipLaunchKernelGGL(k_lbwd_diag, dim3((unsigned)nrhs), dim3(1024), 0, s, LU, X, nl, k0, k1);
    if (k0 > 0)
      hipLaunchKernelGGL(k_lbwd_rest, dim3(grid_for(k0, 2048), (unsigned)nrhs), dim3(256), 0, s, LU,
                         X, nl, k0, k1);
    k1 = k0;
  }
  return hipGetLastError();
}

hipError_t launch_larith(int op, int nl, int64_t cnt, LimbMat A, LimbMat B, LimbMat C,
                         hipStream_t s) {
  if (cnt <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_larith, dim3(grid_for(cnt)), dim3(256), 0, s, op, nl, cnt, A, B, C);
  return hipGetLastError();
}

hipError_t launch_lfill_i32(int32_t *p, int32_t v, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lfill_i32, dim3((count + 255) / 256), dim3(256), 0, s, p, v, count);
  return hipGetLastError();
}

}  // namespace ozl
