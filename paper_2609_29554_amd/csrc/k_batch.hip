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

namespace {

constexpr int BT = 1024;  // threads per workgroup (4 wavefronts per SIMD)

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
    // pivot search in column j, rows j..n-1
    double bk[NC];
    int64_t bi = -1;
#pragma unroll
    for (int q = 0; q < NC; ++q) bk[q] = 0.0;
    for (int64_t i = j + tid; i < n; i += BT) {
      double x[NC];
      ozx::load<NC>(E(i, j), x);
      if (piv_better<NC>(x, i, bk, bi)) {
#pragma unroll
        for (int q = 0; q < NC; ++q) bk[q] = x[q];
        bi = i;
      }
    }
#pragma unroll
    for (int q = 0; q < NC; ++q) rkey[tid][q] = bk[q];
    ridx[tid] = bi;
    __syncthreads();
    for (int s = BT / 2; s > 0; s >>= 1) {
      if (tid < s) {
        double ka[NC], kv[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) {
          ka[q] = rkey[tid][q];
          kv[q] = rkey[tid + s][q];
        }
        if (piv_better<NC>(kv, ridx[tid + s], ka, ridx[tid])) {
#pragma unroll
          for (int q = 0; q < NC; ++q) rkey[tid][q] = kv[q];
          ridx[tid] = ridx[tid + s];
        }
      }
      __syncthreads();
    }
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
        for (int64_t c = tid; c < n; c += BT) {
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
      for (int64_t i = j + 1 + tid; i < n; i += BT) {
        double a[NC], l[NC];
        ozx::load<NC>(E(i, j), a);
        ozx::div<NC>(a, d, l);
        ozx::store<NC>(E(i, j), l);
      }
      __syncthreads();
    }
    // rank-1 update of the trailing matrix (also after a zero pivot, with the
    // unscaled -- all-zero -- column, as the blocked LU with b = 1 does)
    const int64_t m = n - j - 1;
    for (int64_t idx = tid; idx < m * m; idx += BT) {
      const int64_t i = j + 1 + idx % m, c = j + 1 + idx / m;
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
  if (!it.b) return;
  // solve: interchanges in ipiv order, forward (unit L, ascending), backward
  // with the reciprocals 1 / u_kk (descending)
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
    for (int64_t i = k + 1 + tid; i < n; i += BT) {
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
      double one[NC], u[NC], r[NC], xk[NC], o[NC];
#pragma unroll
      for (int q = 0; q < NC; ++q) one[q] = q == 0 ? 1.0 : 0.0;
      ozx::load<NC>(E(k, k), u);
      ozx::div<NC>(one, u, r);
      ozx::load<NC>(x + k * NC, xk);
      ozx::mul<NC>(xk, r, o);
      ozx::store<NC>(x + k * NC, o);
    }
    __syncthreads();
    double xk[NC];
    ozx::load<NC>(x + k * NC, xk);
    for (int64_t i = tid; i < k; i += BT) {
      double a[NC], u[NC], o[NC];
      ozx::load<NC>(x + i * NC, a);
      ozx::load<NC>(E(i, k), u);
      ozx::fms<NC>(a, u, xk, o);
      ozx::store<NC>(x + i * NC, o);
    }
    __syncthreads();
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
}  // namespace ozl
