// LU kernels for gfx950 around the Ozaki-II update (Sec. 3.4 of the paper):
//   (P1) panel factorisation with partial pivoting,
//   (P2) row interchanges (laswp),
//   (P3) U12 = L11^{-1} A12,
//   the native expansion product C -= A B (blocked-naive comparator and the
//   triangular-solve updates), and the pieces of the solve (getrs).
// All multiple-precision arithmetic here is the expansion arithmetic of
// expansion.hpp; every element sees its multiply-subtracts in the order the
// specification fixes (ascending inner index, descending in the backward
// substitution).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "expansion.hpp"
#include "ozii_kernels.hpp"

namespace {

// ---------------------------------------------------------------------------
// Exchange between the workgroups of the cooperative panel kernel.
//
// Each workgroup owns two 128-byte candidate lines (one per parity of the
// pivot column): word 0 holds an arrival epoch, the rest the workgroup's
// pivot candidate for that column -- its row position and physical row, its
// value in the pivot column and in the next column -- and a buffer crow holds
// the rest of that row.  A workgroup writes the payload with device-coherent
// stores, waits for them to complete and then stores the epoch (no release
// fence, which would write back the whole L2 every column; see
// cand_arrive).  Readers poll the epochs and read every payload and crow
// with device-coherent loads, which go past the non-coherent caches, so no
// cache invalidation is needed on the reading side; they are issued only
// after the epochs were seen (the wait ends in a workgroup barrier).  Waits
// are bounded: a timeout raises the sticky error flag, after which every
// later wait returns at once, so a broken invariant ends the kernel quickly.
// ---------------------------------------------------------------------------
constexpr int CAND_WORDS = 32;  // uint32 per candidate line
constexpr int CAND_KEY = 4;     // first payload word of the key doubles

__device__ __forceinline__ uint32_t ld_dev_u32(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_dev_f64(const double *p) {
  const uint64_t v = __hip_atomic_load((const uint64_t *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  double d;
  __builtin_memcpy(&d, &v, 8);
  return d;
}

__device__ __forceinline__ void st_dev_u32(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev_f64(double *p, double v) {
  uint64_t u;
  __builtin_memcpy(&u, &v, 8);
  __hip_atomic_store((uint64_t *)p, u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Publish the epoch in this workgroup's candidate line.  Everything the
// other workgroups read of it (the line's payload, the candidate row) is
// written with device-coherent stores, so it only has to have completed
// before the epoch is stored: every wave waits for its own stores
// (s_waitcnt vmcnt(0)), then the workgroup barrier, then the epoch -- no
// write-back of the XCD's L2, which a release fence would do every column.
__device__ __forceinline__ void cand_arrive(uint32_t *line, uint32_t epoch) {
  __builtin_amdgcn_s_waitcnt(0x0F70);
  __syncthreads();
  if (threadIdx.x == 0) st_dev_u32(line, epoch);
}

// Wait until the lines of all G workgroups (buffer b) carry an epoch of at
// least `epoch`.  Returns false when the wait failed (timeout now or
// earlier); the caller must then stop using data published by others.
__device__ __forceinline__ bool cand_wait(const uint32_t *lines, int G, int b, uint32_t epoch,
                                          int *err) {
  __shared__ int s_fail;
  if ((int)threadIdx.x < G) {
    // bounded by the 100 MHz real-time counter: about one second
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    uint32_t spins = 0;
    const uint32_t *f = lines + ((size_t)b * G + threadIdx.x) * CAND_WORDS;
    // epochs only grow: a workgroup that already arrived for a later epoch
    // has also arrived for this one
    while ((int32_t)(ld_dev_u32(f) - epoch) < 0) {
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
      if ((++spins & 63u) == 0 && __builtin_amdgcn_s_memrealtime() - t0 > 100000000ull) {
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0)
    s_fail = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
  __syncthreads();
  return !s_fail;
}

// Candidate order of the pivot search: larger |value| first, then the lower
// row position.  A total order on (key, position) pairs, so any reduction
// tree picks the same winner.
template <int NC>
__device__ __forceinline__ bool cand_better(const double (&kb_)[NC], int pb, int ib,
                                            const double (&ka)[NC], int pa, int ia) {
  if (ib < 0) return false;
  if (ia < 0) return true;
  if (ozx::abs_greater<NC>(kb_, ka)) return true;
  if (ozx::abs_greater<NC>(ka, kb_)) return false;
  return pb < pa;
}

// Partner value of a 64-bit / 32-bit word under a DPP lane pattern (CTRL:
// quad_perm or row mirror, never out of range); every lane of the
// wavefront must call it.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  uint64_t u;
  __builtin_memcpy(&u, &x, 8);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xf, 0xf, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, false);
  const uint64_t v = ((uint64_t)hi << 32) | lo;
  double d;
  __builtin_memcpy(&d, &v, 8);
  return d;
}
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xf, 0xf, false);
}

// The best candidate of the wavefront in every lane (cand_better is a total
// order, so any pairing network that meets every lane gives the same one):
// lanes 32 and 16 apart through the LDS crossbar, then within each row of 16
// by DPP (mirror, half mirror, quad swaps), which needs no LDS round trip.
// All 64 lanes must call it.
template <int NC>
__device__ __forceinline__ void cand_allreduce(double (&k)[NC], int &pos, int &idx) {
  auto take = [&](const double (&ok)[NC], int op, int oi) {
    if (cand_better<NC>(ok, op, oi, k, pos, idx)) {
#pragma unroll
      for (int q = 0; q < NC; ++q) k[q] = ok[q];
      pos = op;
      idx = oi;
    }
  };
#pragma unroll
  for (int off = 32; off >= 16; off >>= 1) {
    double ok[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) ok[q] = __shfl_xor(k[q], off, 64);
    take(ok, __shfl_xor(pos, off, 64), __shfl_xor(idx, off, 64));
  }
#define OZ_DPP_STEP(CTRL)                                         \
  do {                                                            \
    double ok[NC];                                                \
    _Pragma("unroll") for (int q = 0; q < NC; ++q) ok[q] = dpp_f64<CTRL>(k[q]); \
    take(ok, dpp_i32<CTRL>(pos), dpp_i32<CTRL>(idx));              \
  } while (0)
  OZ_DPP_STEP(0x140);  // row_mirror: lane i <-> 15 - i of its row
  OZ_DPP_STEP(0x141);  // row_half_mirror: i <-> 7 - i of its half row
  OZ_DPP_STEP(0x4E);   // quad_perm [2, 3, 0, 1]
  OZ_DPP_STEP(0xB1);   // quad_perm [1, 0, 3, 2]
#undef OZ_DPP_STEP
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  uint64_t u;
  __builtin_memcpy(&u, &v, 8);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
  const uint64_t w = ((uint64_t)hi << 32) | lo;
  double d;
  __builtin_memcpy(&d, &w, 8);
  return d;
}

__device__ __forceinline__ double wave_max_f64(double v) {
  v = fmax(v, __shfl_xor(v, 32, 64));
  v = fmax(v, __shfl_xor(v, 16, 64));
  v = fmax(v, dpp_f64<0x140>(v));
  v = fmax(v, dpp_f64<0x141>(v));
  v = fmax(v, dpp_f64<0x4E>(v));
  v = fmax(v, dpp_f64<0xB1>(v));
  return v;
}

// Leading-magnitude shortcut of the candidate order.  Each lane of a
// wavefront has reduced its own candidates to lead = the largest |k[0]|
// among them (-1 for none, NaN if one is NaN) and nlead = how many reach
// it.  The order compares |k[0]| first, so when the largest leading
// magnitude belongs to exactly one candidate, that one wins whatever its
// other components and position: returns 1 and its lane in w.  Returns 0
// when no lane has a candidate, 2 when the full order has to decide (equal
// leading magnitudes, NaN).  All 64 lanes must call it; the result is
// uniform.
__device__ __forceinline__ int lead_winner(double lead, int nlead, int &w) {
  const double M = wave_max_f64(lead);
  const uint64_t hit = __ballot(lead == M);
  const uint64_t odd = __ballot(lead != lead || (lead == M && nlead > 1));
  if (odd != 0) return 2;
  if (M < 0.0) return 0;
  if (__popcll(hit) != 1) return 2;
  w = __ffsll((unsigned long long)hit) - 1;
  return 1;
}

constexpr int PANEL_NT = 512;  // threads per panel workgroup

// ---------------------------------------------------------------------------
// (P1) panel.  Panel rows [k, n), columns [k, k+kb).  Workgroup w owns the
// physical rows k + w*R .. k + w*R + R - 1 and keeps them in LDS for the
// whole panel.  Rows are never moved during the panel: the row permutation
// is tracked in LDS (position -> physical row and back, every workgroup
// keeping an identical copy) and applied once afterwards.  Per column j:
//   1. wait for every workgroup's candidate for column j (largest |value| in
//      its active rows, ties to the lowest position) and reduce the table
//      identically everywhere: the winner is LAPACK's i?amax on the permuted
//      column;
//   2. wavefront 0 divides the active rows by the pivot and updates column
//      j+1 (the candidate line carries the pivot row's value there) while
//      the other wavefronts fetch the rest of the pivot row;
//   3. pick the local candidate for column j+1, finish that row's update and
//      publish it (the critical path), then arrive;
//   4. update the remaining columns of the other active rows while the other
//      workgroups arrive.
// Every element still receives its multiply-subtracts in column order.
// ---------------------------------------------------------------------------
template <int NC>
__global__ __launch_bounds__(PANEL_NT) void k_panel(double *A, int64_t lda, int64_t n, int64_t k,
                                                    int kb, int R, int64_t *ipiv, int32_t *info,
                                                    uint32_t *lines, int *err, double *crow,
                                                    int *perm_out, int *moved, int *nmoved) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  // the panel is the critical path of the factorisation, and with
  // look-ahead the previous step's Schur update runs beside it on the same
  // CUs: its wavefronts take the SIMDs' issue slots first
  __builtin_amdgcn_s_setprio(3);
  const int nr = (int)(n - k);
  const int G = gridDim.x, wg = blockIdx.x, tid = threadIdx.x;
  double *rows = (double *)smem_raw;                 // R * kb * NC
  double *piv = rows + (size_t)R * kb * NC;          // kb * NC
  int *sperm = (int *)(piv + (size_t)kb * NC);       // nr
  int *sinv = sperm + nr;                            // nr
  __shared__ double tkey[256][NC], tnxt[256][NC];
  __shared__ int tpos[256], tidx[256], tphys[256];
  __shared__ uint32_t active;
  __shared__ int s_info, s_wi, s_ppos, s_pphys, s_zero, s_best;

  const int r0 = wg * R;
  const int cnt = r0 < nr ? (nr - r0 < R ? nr - r0 : R) : 0;
  auto RW = [&](int r, int c) { return rows + ((size_t)r * kb + c) * NC; };
  auto LINE = [&](int b, int w) { return lines + ((size_t)b * G + w) * CAND_WORDS; };
  auto CROW = [&](int b, int w) { return crow + ((size_t)b * G + w) * kb * NC; };

  for (int idx = tid; idx < cnt * kb; idx += PANEL_NT) {
    const int r = idx % cnt, c = idx / cnt;
    const double *src = A + ((k + r0 + r) + (k + c) * lda) * NC;
#pragma unroll
    for (int q = 0; q < NC; ++q) RW(r, c)[q] = src[q];
  }
  for (int p = tid; p < nr; p += PANEL_NT) {
    sperm[p] = p;
    sinv[p] = p;
  }
  if (tid == 0) {
    active = cnt >= 32 ? 0xffffffffu : ((1u << cnt) - 1u);
    s_info = 0;
  }
  __syncthreads();

  // local candidate for column c among the active rows (thread 0), result in
  // s_best (local row or -1)
  auto pick = [&](int c) {
    if (tid == 0) {
      int best = -1;
      double bk[NC];
      for (int r = 0; r < cnt; ++r) {
        if (!((active >> r) & 1u)) continue;
        double x[NC];
        ozx::load<NC>(RW(r, c), x);
        bool take = best < 0;
        if (!take) {
          if (ozx::abs_greater<NC>(x, bk)) take = true;
          else if (!ozx::abs_greater<NC>(bk, x) && sinv[r0 + r] < sinv[r0 + best]) take = true;
        }
        if (take) {
          best = r;
#pragma unroll
          for (int q = 0; q < NC; ++q) bk[q] = x[q];
        }
      }
      s_best = best;
    }
    __syncthreads();
  };
  // publish the candidate of column c (row s_best) into buffer b: the line
  // payload (position, physical row, values in columns c and c+1) and the
  // row's columns c+2 .. kb-1 in crow
  auto publish = [&](int c, int b) {
    const int best = s_best;
    uint32_t *ln = LINE(b, wg);
    if (tid == 0) {
      double *kv = (double *)(ln + CAND_KEY);
      if (best >= 0) {
        st_dev_u32(ln + 1, (uint32_t)sinv[r0 + best]);
        st_dev_u32(ln + 2, (uint32_t)(r0 + best));
#pragma unroll
        for (int q = 0; q < NC; ++q) {
          st_dev_f64(kv + q, RW(best, c)[q]);
          st_dev_f64(kv + NC + q, c + 1 < kb ? RW(best, c + 1)[q] : 0.0);
        }
      } else {
        st_dev_u32(ln + 1, 0x7fffffffu);
        st_dev_u32(ln + 2, 0xffffffffu);
      }
    }
    if (best >= 0) {
      double *cr = CROW(b, wg);
      for (int idx = tid; idx < (kb - c - 2) * NC; idx += PANEL_NT)
        st_dev_f64(cr + (size_t)(c + 2) * NC + idx, RW(best, c + 2)[idx]);
    }
  };

  pick(0);
  publish(0, 0);
  cand_arrive(LINE(0, wg), 1u);

  for (int j = 0; j < kb; ++j) {
    const int buf = j & 1;
    if (!cand_wait(lines, G, buf, (uint32_t)(j + 1), err)) return;
    // read the candidate table (one line per thread, device-coherent) and
    // reduce it identically in every workgroup: four entries per lane of the
    // first wavefront, then a butterfly
    if (tid < G) {
      // every device-coherent load first, then the LDS stores: the compiler
      // keeps atomic loads in program order, so a store between two of them
      // would make each load wait for the previous one's round trip
      const uint32_t *ln = LINE(buf, tid);
      const double *kv = (const double *)(ln + CAND_KEY);
      const int ph = (int)ld_dev_u32(ln + 2);
      const int pos = (int)ld_dev_u32(ln + 1);
      double kk[NC], kn[NC];
#pragma unroll
      for (int q = 0; q < NC; ++q) kk[q] = ld_dev_f64(kv + q);
#pragma unroll
      for (int q = 0; q < NC; ++q) kn[q] = ld_dev_f64(kv + NC + q);
      tpos[tid] = pos;
      tphys[tid] = ph;
      tidx[tid] = ph >= 0 ? tid : -1;
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        tkey[tid][q] = kk[q];
        tnxt[tid][q] = kn[q];
      }
    }
    __syncthreads();
    if (tid < 64) {
      double bk[NC];
      int bp = 0x7fffffff, bi = -1;
#pragma unroll
      for (int q = 0; q < NC; ++q) bk[q] = 0.0;
      // leading magnitudes of this lane's entries first; the full order
      // only when they do not single out the winner
      double lead = -1.0;
      int nlead = 0, lb = 0;
      for (int gi = tid; gi < G; gi += 64) {
        if (tidx[gi] < 0) continue;
        const double m = fabs(tkey[gi][0]);
        if (m != m) lead = m;
        else if (m > lead) { lead = m; nlead = 1; lb = gi; }
        else if (m == lead) ++nlead;
      }
      int w = 0;
      const int how = lead_winner(lead, nlead, w);
      if (how == 1) {
        bi = __builtin_amdgcn_readlane(lb, w);
        bp = tpos[bi];
#pragma unroll
        for (int q = 0; q < NC; ++q) bk[q] = tkey[bi][q];
      } else if (how == 2) {
        for (int gi = tid; gi < G; gi += 64) {
          double kk[NC];
#pragma unroll
          for (int q = 0; q < NC; ++q) kk[q] = tkey[gi][q];
          if (cand_better<NC>(kk, tpos[gi], tidx[gi], bk, bp, bi)) {
#pragma unroll
            for (int q = 0; q < NC; ++q) bk[q] = kk[q];
            bp = tpos[gi];
            bi = tidx[gi];
          }
        }
        cand_allreduce<NC>(bk, bp, bi);
      }
      if (tid == 0) {
        // the winner, and (for a consistent table) the bookkeeping of the
        // interchange, before the single barrier below
        const int wi0 = bi, pp0 = bp, ph0 = bi >= 0 ? tphys[bi] : -1;
        bool z = true;
#pragma unroll
        for (int q = 0; q < NC; ++q) z = z && (bk[q] == 0.0);
        s_wi = wi0;
        s_ppos = pp0;
        s_pphys = ph0;
        s_zero = z ? 1 : 0;
        if (!(wi0 < 0 || pp0 < j || pp0 >= nr || ph0 < 0 || ph0 >= nr)) {
#pragma unroll
          for (int q = 0; q < NC; ++q) {
            piv[(size_t)j * NC + q] = tkey[wi0][q];
            if (j + 1 < kb) piv[(size_t)(j + 1) * NC + q] = tnxt[wi0][q];
          }
          const int q = sperm[j];
          sperm[j] = ph0;
          sperm[pp0] = q;
          sinv[ph0] = j;
          sinv[q] = pp0;
          if (ph0 >= r0 && ph0 < r0 + cnt) active &= ~(1u << (ph0 - r0));
          if (z && s_info == 0) s_info = (int)(k + j + 1);
          if (wg == 0) ipiv[k + j] = k + pp0;
        }
      }
    }
    __syncthreads();
    const int wi = s_wi, ppos = s_ppos, pphys = s_pphys, zero = s_zero;
    // an empty or inconsistent table can only follow a failed wait
    if (wi < 0 || ppos < j || ppos >= nr || pphys < 0 || pphys >= nr) {
      if (tid == 0) __hip_atomic_store(err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    const bool last = j + 1 >= kb;
    if (tid < 64) {
      // wavefront 0: l = a / pivot for the active rows (one per lane, R <=
      // 32), then column j+1, whose values stay in the lanes: the local
      // candidate for column j+1 is their butterfly maximum in the pivot
      // order (the order of pick(), which any reduction tree respects)
      double ck[NC];
      int cpos = 0x7fffffff, cidx = -1;
#pragma unroll
      for (int q = 0; q < NC; ++q) ck[q] = 0.0;
      const int r = tid;
      if (r < cnt && ((active >> r) & 1u)) {
        double x[NC];
        if (!last) ozx::load<NC>(RW(r, j + 1), x);
        if (!zero) {
          double a[NC], d[NC], l[NC];
          ozx::load<NC>(RW(r, j), a);
          ozx::load<NC>(piv + (size_t)j * NC, d);
          ozx::div<NC>(a, d, l);
          ozx::store<NC>(RW(r, j), l);
          if (!last) {
            double u[NC], o[NC];
            ozx::load<NC>(piv + (size_t)(j + 1) * NC, u);
            ozx::fms<NC>(x, l, u, o);
            ozx::store<NC>(RW(r, j + 1), o);
#pragma unroll
            for (int q = 0; q < NC; ++q) x[q] = o[q];
          }
        }
        if (!last) {
#pragma unroll
          for (int q = 0; q < NC; ++q) ck[q] = x[q];
          cpos = sinv[r0 + r];
          cidx = r;
        }
      }
      if (!last) {
        int w = 0;
        const int how = lead_winner(cidx >= 0 ? fabs(ck[0]) : -1.0, 1, w);
        if (how == 1) cidx = __builtin_amdgcn_readlane(cidx, w);
        else if (how == 2) cand_allreduce<NC>(ck, cpos, cidx);
        if (tid == 0) s_best = cidx;
      }
    } else {
      // the other wavefronts: columns j+2 .. kb-1 of the pivot row, PF
      // loads in flight per thread before their LDS stores (see above)
      constexpr int PF = 8;
      const double *cr = CROW(buf, wi) + (size_t)(j + 2) * NC;
      double *pd = piv + (size_t)(j + 2) * NC;
      const int total = (kb - j - 2) * NC;
      for (int b0 = tid - 64; b0 < total; b0 += (PANEL_NT - 64) * PF) {
        double v[PF];
#pragma unroll
        for (int u = 0; u < PF; ++u) {
          const int idx = b0 + u * (PANEL_NT - 64);
          v[u] = idx < total ? ld_dev_f64(cr + idx) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < PF; ++u) {
          const int idx = b0 + u * (PANEL_NT - 64);
          if (idx < total) pd[idx] = v[u];
        }
      }
    }
    __syncthreads();
    if (last) break;
    // candidate for column j+1 (s_best, from wavefront 0): finish its row
    // first, publish, arrive
    const int best = s_best;
    const int width = kb - j - 2;
    if (!zero && best >= 0) {
      for (int c = j + 2 + tid; c < kb; c += PANEL_NT) {
        double x[NC], l[NC], u[NC], o[NC];
        ozx::load<NC>(RW(best, c), x);
        ozx::load<NC>(RW(best, j), l);
        ozx::load<NC>(piv + (size_t)c * NC, u);
        ozx::fms<NC>(x, l, u, o);
        ozx::store<NC>(RW(best, c), o);
      }
      __syncthreads();
    }
    publish(j + 1, (j + 1) & 1);
    cand_arrive(LINE((j + 1) & 1, wg), (uint32_t)(j + 2));
    // the rest of the rank-1 update, overlapped with the other arrivals
    if (!zero && width > 0) {
      for (int idx = tid; idx < cnt * width; idx += PANEL_NT) {
        const int r = idx % cnt, c = j + 2 + idx / cnt;
        if (((active >> r) & 1u) && r != best) {
          double a[NC], l[NC], u[NC], o[NC];
          ozx::load<NC>(RW(r, c), a);
          ozx::load<NC>(RW(r, j), l);
          ozx::load<NC>(piv + (size_t)c * NC, u);
          ozx::fms<NC>(a, l, u, o);
          ozx::store<NC>(RW(r, c), o);
        }
      }
    }
    __syncthreads();
  }
  // write the rows back to their physical places
  for (int idx = tid; idx < cnt * kb; idx += PANEL_NT) {
    const int r = idx % cnt, c = idx / cnt;
    double *dst = A + ((k + r0 + r) + (k + c) * lda) * NC;
#pragma unroll
    for (int q = 0; q < NC; ++q) dst[q] = RW(r, c)[q];
  }
  if (wg == 0) {
    __shared__ int s_nm;
    if (tid == 0) s_nm = 0;
    __syncthreads();
    for (int p = tid; p < nr; p += PANEL_NT) {
      perm_out[p] = sperm[p];
      if (sperm[p] != p) {
        const int slot = atomicAdd(&s_nm, 1);
        moved[slot] = p;
      }
    }
    __syncthreads();
    if (tid == 0) {
      *nmoved = s_nm;
      if (s_info != 0 && *info == 0) *info = s_info;
    }
  }
}

// ---------------------------------------------------------------------------
// (P2) apply the panel's row permutation to columns [c0, c1):
// new row k+p = old row k+perm[p] for every moved position p.
// ---------------------------------------------------------------------------
template <int NC>
__global__ __launch_bounds__(256) void k_laswp(double *A, int64_t lda, int64_t k, int64_t c0,
                                               int64_t c1, const int *perm, const int *moved,
                                               const int *nmoved) {
  const int64_t c = c0 + blockIdx.x;
  if (c >= c1) return;
  const int nm = *nmoved;
  constexpr int PER = 4;  // up to 1024 moved positions per column
  double v[PER][NC];
  int pos[PER];
#pragma unroll
  for (int t = 0; t < PER; ++t) {
    const int e = threadIdx.x + 256 * t;
    pos[t] = -1;
    if (e < nm) {
      const int p = moved[e];
      pos[t] = p;
      ozx::load<NC>(A + ((k + perm[p]) + c * lda) * NC, v[t]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < PER; ++t)
    if (pos[t] >= 0) ozx::store<NC>(A + ((k + pos[t]) + c * lda) * NC, v[t]);
}

// ---------------------------------------------------------------------------
// (P3) X <- L^{-1} X for a unit lower-triangular kb x kb block L (at Lp, ld
// lda) and kb x ncols right-hand sides X (at Xp, ld ldx): element i is
// updated for h = 0 .. i-1 in ascending order.  One workgroup per CPB
// columns; thread t owns rows t, t+256, ...
// ---------------------------------------------------------------------------
template <int NC, int CPB, int RPT>
__global__ __launch_bounds__(256) void k_trsm_lower_unit(const double *Lp, int64_t lda, double *Xp,
                                                         int64_t ldx, int kb, int64_t ncols) {
  __shared__ double xs[2][CPB][NC];
  const int tid = threadIdx.x;
  const int64_t cbase = (int64_t)blockIdx.x * CPB;
  double x[RPT][CPB][NC];
#pragma unroll
  for (int rr = 0; rr < RPT; ++rr) {
    const int i = tid + 256 * rr;
#pragma unroll
    for (int cc = 0; cc < CPB; ++cc) {
      const int64_t c = cbase + cc;
      if (i < kb && c < ncols) ozx::load<NC>(Xp + (i + c * ldx) * NC, x[rr][cc]);
      else
#pragma unroll
        for (int q = 0; q < NC; ++q) x[rr][cc][q] = 0.0;
    }
  }
  for (int h = 0; h < kb; ++h) {
    const int b = h & 1;
    if (tid == (h & 255)) {
#pragma unroll
      for (int rr = 0; rr < RPT; ++rr)
        if (rr == h / 256)
#pragma unroll
          for (int cc = 0; cc < CPB; ++cc)
#pragma unroll
            for (int q = 0; q < NC; ++q) xs[b][cc][q] = x[rr][cc][q];
    }
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr) {
      const int i = tid + 256 * rr;
      if (i > h && i < kb) {
        double l[NC];
        ozx::load<NC>(Lp + (i + (int64_t)h * lda) * NC, l);
#pragma unroll
        for (int cc = 0; cc < CPB; ++cc) {
          double u[NC], o[NC];
#pragma unroll
          for (int q = 0; q < NC; ++q) u[q] = xs[b][cc][q];
          ozx::fms<NC>(x[rr][cc], l, u, o);
#pragma unroll
          for (int q = 0; q < NC; ++q) x[rr][cc][q] = o[q];
        }
      }
    }
  }
#pragma unroll
  for (int rr = 0; rr < RPT; ++rr) {
    const int i = tid + 256 * rr;
#pragma unroll
    for (int cc = 0; cc < CPB; ++cc) {
      const int64_t c = cbase + cc;
      if (i < kb && c < ncols) ozx::store<NC>(Xp + (i + c * ldx) * NC, x[rr][cc]);
    }
  }
}

// U12 solve for kb <= 64 WPC: each column is held by WPC wavefronts, row
// 64 p + l in lane l of the column's wavefront p (4 / WPC columns per
// 256-thread workgroup).  Wavefront p first applies the values of rows
// 0 .. 64 p - 1 as the wavefronts before it publish them (LDS, one counter
// per column), then solves its own 64 rows with no barrier: row h's final
// value is read from lane h - 64 p into scalar registers, published for
// the wavefronts after it, and applied to the later rows.  Every element
// receives its multiply-subtracts in ascending k, the order of
// k_trsm_lower_unit.
template <int NC, int WPC>
__global__ __launch_bounds__(256) void k_trsm_lower_unit_w(const double *Lp, int64_t lda,
                                                           double *Xp, int64_t ldx, int kb,
                                                           int64_t ncols) {
  constexpr int CPB = 4 / WPC;
  __shared__ double xs[CPB][WPC > 1 ? 64 * (WPC - 1) : 1][NC];
  __shared__ int done[CPB];
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int cc = wv / WPC, part = wv % WPC;
  const int64_t c = (int64_t)blockIdx.x * CPB + cc;
  if (tid < CPB) done[tid] = 0;
  __syncthreads();
  if (c >= ncols) return;  // whole wavefronts of a column past the end
  const int i = 64 * part + lane;
  const bool mine = i < kb;
  auto L = [&](int r, int k) { return Lp + (r + (int64_t)k * lda) * NC; };
  double x[NC], l[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    x[q] = 0.0;
    l[q] = 0.0;
  }
  if (mine) ozx::load<NC>(Xp + (i + c * ldx) * NC, x);
  const int h0 = 64 * part, h1 = kb < h0 + 64 ? kb : h0 + 64;
  if (h0 >= kb) return;
  // factor entry l_(i,h) of the next step is loaded while this one computes
  if (mine && i > 0) ozx::load<NC>(L(i, 0), l);
  for (int h = 0; h < h0; ++h) {
    double ln[NC] = {}, y[NC], o[NC];
    if (mine && h + 1 < i) ozx::load<NC>(L(i, h + 1), ln);
    // the value of row h, published by an earlier wavefront of this column
    // (it never waits itself before publishing, so this ends)
    while (__hip_atomic_load(&done[cc], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) <= h)
      __builtin_amdgcn_s_sleep(1);
#pragma unroll
    for (int q = 0; q < NC; ++q) y[q] = xs[cc][h][q];
    if (mine) {
      ozx::fms<NC>(x, l, y, o);
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        x[q] = o[q];
        l[q] = ln[q];
      }
    }
  }
  for (int h = h0; h < h1; ++h) {
    double ln[NC] = {}, y[NC], o[NC];
    if (mine && h + 1 < i) ozx::load<NC>(L(i, h + 1), ln);
    // row h is final
#pragma unroll
    for (int q = 0; q < NC; ++q) y[q] = readlane_f64(x[q], h - h0);
    if (part + 1 < WPC && lane == h - h0) {
#pragma unroll
      for (int q = 0; q < NC; ++q) xs[cc][h][q] = y[q];
      __hip_atomic_store(&done[cc], h + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    if (mine && i > h) {
      ozx::fms<NC>(x, l, y, o);
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        x[q] = o[q];
        l[q] = ln[q];
      }
    }
  }
  if (mine) ozx::store<NC>(Xp + (i + c * ldx) * NC, x);
}

// X <- U^{-1} X for an upper-triangular kb x kb block: for h = kb-1 .. 0,
// x_h <- x_h / u_hh (expansion division), then x_i -= u_ih x_h for i < h
// (descending order).
template <int NC, int CPB, int RPT>
__global__ __launch_bounds__(256) void k_trsm_upper(const double *Up, int64_t lda, double *Xp,
                                                    int64_t ldx, int kb, int64_t ncols) {
  __shared__ double xs[2][CPB][NC];
  const int tid = threadIdx.x;
  const int64_t cbase = (int64_t)blockIdx.x * CPB;
  double x[RPT][CPB][NC];
#pragma unroll
  for (int rr = 0; rr < RPT; ++rr) {
    const int i = tid + 256 * rr;
#pragma unroll
    for (int cc = 0; cc < CPB; ++cc) {
      const int64_t c = cbase + cc;
      if (i < kb && c < ncols) ozx::load<NC>(Xp + (i + c * ldx) * NC, x[rr][cc]);
      else
#pragma unroll
        for (int q = 0; q < NC; ++q) x[rr][cc][q] = 0.0;
    }
  }
  for (int h = kb - 1; h >= 0; --h) {
    const int b = h & 1;
    if (tid == (h & 255)) {
#pragma unroll
      for (int rr = 0; rr < RPT; ++rr)
        if (rr == h / 256) {
          double d[NC];
          ozx::load<NC>(Up + (h + (int64_t)h * lda) * NC, d);
#pragma unroll
          for (int cc = 0; cc < CPB; ++cc) {
            double o[NC];
            ozx::div<NC>(x[rr][cc], d, o);
#pragma unroll
            for (int q = 0; q < NC; ++q) {
              x[rr][cc][q] = o[q];
              xs[b][cc][q] = o[q];
            }
          }
        }
    }
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr) {
      const int i = tid + 256 * rr;
      if (i < h) {
        double u[NC];
        ozx::load<NC>(Up + (i + (int64_t)h * lda) * NC, u);
#pragma unroll
        for (int cc = 0; cc < CPB; ++cc) {
          double xh[NC], o[NC];
#pragma unroll
          for (int q = 0; q < NC; ++q) xh[q] = xs[b][cc][q];
          ozx::fms<NC>(x[rr][cc], u, xh, o);
#pragma unroll
          for (int q = 0; q < NC; ++q) x[rr][cc][q] = o[q];
        }
      }
    }
  }
#pragma unroll
  for (int rr = 0; rr < RPT; ++rr) {
    const int i = tid + 256 * rr;
#pragma unroll
    for (int cc = 0; cc < CPB; ++cc) {
      const int64_t c = cbase + cc;
      if (i < kb && c < ncols) ozx::store<NC>(Xp + (i + c * ldx) * NC, x[rr][cc]);
    }
  }
}

// ---------------------------------------------------------------------------
// Native expansion product: C <- C - A B with one rounded multiply-subtract
// per inner index, h ascending (desc = 0) or descending (desc = 1).
// A is M x K (lda), B is K x N (ldb).  Tile TM x TN outputs per workgroup.
// ---------------------------------------------------------------------------
template <int NC, int TM, int TN>
__global__ __launch_bounds__(256) void k_naive_gemm(const double *A, int64_t lda, const double *B,
                                                    int64_t ldb, double *C, int64_t ldc, int64_t M,
                                                    int64_t N, int64_t K, int desc) {
  static_assert(TM * TN == 256, "tile");
  constexpr int KC = TM >= 128 ? 4 : 16;
  __shared__ double As[KC][TM][NC];
  __shared__ double Bs[TN][KC][NC];
  const int tid = threadIdx.x;
  const int ti = tid % TM, tj = tid / TM;
  const int64_t i = (int64_t)blockIdx.x * TM + ti, j = (int64_t)blockIdx.y * TN + tj;
  double acc[NC];
  const bool in = i < M && j < N;
  if (in) ozx::load<NC>(C + (i + j * ldc) * NC, acc);
  else
#pragma unroll
    for (int q = 0; q < NC; ++q) acc[q] = 0.0;
  const int64_t nch = (K + KC - 1) / KC;
  for (int64_t cc = 0; cc < nch; ++cc) {
    const int64_t ch = desc ? nch - 1 - cc : cc;
    const int64_t h0 = ch * KC;
    for (int e = tid; e < KC * TM; e += 256) {
      const int r = e % TM, hh = e / TM;
      const int64_t gi = (int64_t)blockIdx.x * TM + r, gh = h0 + hh;
#pragma unroll
      for (int q = 0; q < NC; ++q)
        As[hh][r][q] = (gi < M && gh < K) ? A[(gi + gh * lda) * NC + q] : 0.0;
    }
    for (int e = tid; e < KC * TN; e += 256) {
      const int hh = e % KC, cj = e / KC;
      const int64_t gj = (int64_t)blockIdx.y * TN + cj, gh = h0 + hh;
#pragma unroll
      for (int q = 0; q < NC; ++q)
        Bs[cj][hh][q] = (gj < N && gh < K) ? B[(gh + gj * ldb) * NC + q] : 0.0;
    }
    __syncthreads();
    if (in) {
      const int hmax = (int)((K - h0) < KC ? (K - h0) : KC);
      for (int t = 0; t < hmax; ++t) {
        const int hh = desc ? hmax - 1 - t : t;
        double a[NC], b[NC], o[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) {
          a[q] = As[hh][ti][q];
          b[q] = Bs[tj][hh][q];
        }
        ozx::fms<NC>(acc, a, b, o);
#pragma unroll
        for (int q = 0; q < NC; ++q) acc[q] = o[q];
      }
    }
    __syncthreads();
  }
  if (in) ozx::store<NC>(C + (i + j * ldc) * NC, acc);
}

// getrs: apply the interchanges ipiv[0..n) in order to one column of B.
// Row interchanges of the solve, b <- P b with P the product of the
// transpositions (j, ipiv[j]), j ascending (LAPACK's i?laswp).  One
// workgroup per right-hand side.  use_lds: the pivots are staged in LDS,
// thread 0 composes the transpositions on row indices (src[j] = row that
// ends at position j), and the expansions are then gathered in parallel.
template <int NC>
__global__ __launch_bounds__(256) void k_apply_ipiv(double *B, int64_t ldb, int64_t n,
                                                    const int64_t *ipiv, int use_lds) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  double *col = B + (int64_t)blockIdx.x * ldb * NC;
  if (use_lds) {
    double *xs = (double *)smem_raw;               // n * NC
    int *pv = (int *)(xs + n * NC);                // n
    int *src = pv + n;                             // n
    for (int64_t e = threadIdx.x; e < n * NC; e += 256) xs[e] = col[e];
    for (int64_t j = threadIdx.x; j < n; j += 256) {
      pv[j] = (int)ipiv[j];
      src[j] = (int)j;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int j = 0; j < (int)n; ++j) {
        const int p = pv[j];
        const int t = src[j];
        src[j] = src[p];
        src[p] = t;
      }
    }
    __syncthreads();
    for (int64_t e = threadIdx.x; e < n * NC; e += 256) col[e] = xs[(int64_t)src[e / NC] * NC + e % NC];
  } else if (threadIdx.x == 0) {
    for (int64_t j = 0; j < n; ++j) {
      const int64_t p = ipiv[j];
      if (p != j) {
#pragma unroll
        for (int q = 0; q < NC; ++q) {
          double t = col[j * NC + q];
          col[j * NC + q] = col[p * NC + q];
          col[p * NC + q] = t;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Triangular solves of getrs for one right-hand side, pipelined over the
// whole grid (one ordinary launch per direction).  A workgroup takes its
// block of rows from an atomic ticket when it starts, so block t belongs to
// the t-th workgroup to run: every block it waits for is owned by a
// workgroup that is already running, whatever order the hardware dispatches
// workgroups in and however few fit on the device at once.  Block t holds
// the rows at processing positions [t R, t R + R): rows 0.. in the forward
// solve with the unit lower factor, rows n-1.. in the backward solve with
// the upper factor.  Each row's value lives in one lane of wavefront 0.
//
// While earlier blocks are being finished the workgroup applies their
// published solution values to its rows: the products l_ik x_k by all
// wavefronts, then the subtractions in the order the specification fixes
// (ascending k forward, descending backward), so every element sees exactly
// fms(x_i, l_ik, x_k) = x_i (+) (-(l_ik (x) x_k)) in that order.  Its
// diagonal block, staged in LDS when the workgroup starts, is then solved by
// wavefront 0 alone, with no barrier: row q's final value (backward: its
// value divided by u_qq) is read from lane q into scalar registers and
// applied to the later rows of the block.  Wavefront 1 publishes the final
// values in groups of TRSV_PUB rows (stores, agent release, then the count
// of finished positions), so the critical chain of the solve never waits
// for a store.  Waits are bounded like the panel's.
constexpr int TRSV_R = 32;    // rows per workgroup (lanes of wavefront 0)
constexpr int TRSV_B = 32;    // solution values applied per batch
constexpr int TRSV_PUB = 4;   // rows of the diagonal block published at a time

template <int NC, bool FWD>
__global__ __launch_bounds__(256) void k_trsv(const double *LU, int64_t lda, double *x,
                                              int64_t n, uint32_t *ready, uint32_t *ticket,
                                              int *err) {
  __shared__ double dg[TRSV_R][TRSV_R][NC];  // dg[q][r]: factor entry of row r, column q
  __shared__ double pr[TRSV_B][TRSV_R][NC];  // negated products of one batch
  __shared__ double ys[TRSV_B][NC];          // published values of one batch
  __shared__ double xs[TRSV_R][NC];          // final values of the block
  __shared__ int s_avail, s_fail, s_blk, s_done;
  const int tid = threadIdx.x;
  if (tid == 0) s_blk = (int)atomicAdd(ticket, 1u);
  __syncthreads();
  const int64_t p0 = (int64_t)s_blk * TRSV_R;
  const int cnt = (int)(n - p0 < TRSV_R ? n - p0 : TRSV_R);
  auto row = [&](int64_t p) { return FWD ? p : n - 1 - p; };
  auto L = [&](int64_t i, int64_t k) { return LU + (i + k * lda) * NC; };
  // the diagonal block (strict triangle, plus the diagonal backward); the
  // row index runs fastest, so each column is one contiguous read
  for (int e = tid; e < TRSV_R * TRSV_R * NC; e += 256) {
    const int q = e / (TRSV_R * NC), r = (e / NC) % TRSV_R, c = e % NC;
    if (q < cnt && r < cnt && (r > q || (!FWD && r == q)))
      dg[q][r][c] = L(row(p0 + r), row(p0 + q))[c];
  }
  double v[NC];  // the row value of lane tid (wavefront 0, tid < cnt)
#pragma unroll
  for (int c = 0; c < NC; ++c) v[c] = tid < cnt ? x[row(p0 + tid) * NC + c] : 0.0;
  if (tid == 0) {
    s_fail = 0;
    s_done = 0;
  }
  __syncthreads();
  int64_t applied = 0;
  while (applied < p0) {
    if (tid == 0) {
      const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
      uint32_t spins = 0, w;
      while ((int64_t)(w = ld_dev_u32(ready)) <= applied) {
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) { s_fail = 1; break; }
        if ((++spins & 63u) == 0 && __builtin_amdgcn_s_memrealtime() - t0 > 100000000ull) {
          __hip_atomic_store(err, 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          s_fail = 1;
          break;
        }
      }
      s_avail = (int)((int64_t)w < p0 ? (int64_t)w : p0);
    }
    __syncthreads();
    if (s_fail) return;
    const int64_t avail = s_avail;
    for (int64_t c0 = applied; c0 < avail; c0 += TRSV_B) {
      const int nb = (int)(avail - c0 < TRSV_B ? avail - c0 : TRSV_B);
      // published values: device-coherent loads, issued after the count was seen
      if (tid < nb * NC) (&ys[0][0])[tid] = ld_dev_f64(x + row(c0 + tid / NC) * NC + tid % NC);
      __syncthreads();
      for (int idx = tid; idx < cnt * nb; idx += 256) {
        const int q = idx % cnt, t = idx / cnt;
        double a[NC], y[NC], o[NC];
        ozx::load<NC>(L(row(p0 + q), row(c0 + t)), a);
#pragma unroll
        for (int c = 0; c < NC; ++c) y[c] = ys[t][c];
        ozx::mul<NC>(a, y, o);
#pragma unroll
        for (int c = 0; c < NC; ++c) pr[t][q][c] = -o[c];
      }
      __syncthreads();
      // the subtractions, in order; the next batch's barrier waits for them
      if (tid < cnt) {
        for (int t = 0; t < nb; ++t) {
          double pv[NC], o[NC];
#pragma unroll
          for (int c = 0; c < NC; ++c) pv[c] = pr[t][tid][c];
          ozx::add<NC>(v, pv, o);
#pragma unroll
          for (int c = 0; c < NC; ++c) v[c] = o[c];
        }
      }
    }
    applied = avail;
  }
  __syncthreads();
  if (tid < 64) {
    // wavefront 0: the diagonal block; the factor entries of the next step
    // are read from LDS while this one computes
    const int lane = tid;
    double a[NC], u[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      a[c] = lane > 0 && lane < cnt ? dg[0][lane][c] : 0.0;
      u[c] = FWD ? 0.0 : dg[0][0][c];
    }
    for (int q = 0; q < cnt; ++q) {
      double an[NC], un[NC];
      const int qn = q + 1 < cnt ? q + 1 : q;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        an[c] = lane > qn && lane < cnt ? dg[qn][lane][c] : 0.0;
        un[c] = FWD ? 0.0 : dg[qn][qn][c];
      }
      if (!FWD && lane == q) {
        double o[NC];
        ozx::div<NC>(v, u, o);
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c] = o[c];
      }
      // row q is final
      double y[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) y[c] = readlane_f64(v[c], q);
      if (lane == q) {
#pragma unroll
        for (int c = 0; c < NC; ++c) xs[q][c] = v[c];
      }
      if (lane > q && lane < cnt) {
        double o[NC];
        ozx::fms<NC>(v, a, y, o);
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c] = o[c];
      }
      if ((q + 1) % TRSV_PUB == 0 || q + 1 == cnt) {
        // the group's values are in LDS before the count is raised
        if (lane == 0)
          __hip_atomic_store(&s_done, q + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        a[c] = an[c];
        u[c] = un[c];
      }
    }
  } else if (tid < 128) {
    // wavefront 1: publication of the finished rows
    const int lane = tid - 64;
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    int done = 0;
    while (done < cnt) {
      const int d = __hip_atomic_load(&s_done, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (d <= done) {
        if (__builtin_amdgcn_s_memrealtime() - t0 > 100000000ull) {
          if (lane == 0) __hip_atomic_store(err, 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          return;
        }
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      for (int e = lane; e < (d - done) * NC; e += 64) {
        const int q = done + e / NC, c = e % NC;
        x[row(p0 + q) * NC + c] = xs[q][c];
      }
      // this wavefront's stores complete before the count is raised
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      if (lane == 0)
        __hip_atomic_store(ready, (uint32_t)(p0 + d), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      done = d;
    }
  }
}

__global__ void k_fill_int(int *p, int v, int64_t cnt) {
  int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < cnt) p[e] = v;
}

}  // namespace

namespace ozl {

size_t panel_lds_bytes(int nc, int kb, int R, int64_t nr) {
  return (size_t)R * kb * nc * 8 + (size_t)kb * nc * 8 + (size_t)nr * 8;
}

const void *panel_kernel_ptr(int nc) {
  if (nc == 2) return (const void *)k_panel<2>;
  if (nc == 3) return (const void *)k_panel<3>;
  return (const void *)k_panel<4>;
}

hipError_t launch_panel(int nc, double *A, int64_t lda, int64_t n, int64_t k, int kb, int R, int G,
                        int64_t *ipiv, int32_t *info, uint32_t *lines, int *err, double *crow,
                        int *perm, int *moved, int *nmoved, hipStream_t s) {
  const size_t lds = panel_lds_bytes(nc, kb, R, n - k);
  const void *fn = panel_kernel_ptr(nc);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  void *args[] = {&A, &lda, &n, &k, &kb, &R, &ipiv, &info, &lines, &err,
                  &crow, &perm, &moved, &nmoved};
  return hipLaunchCooperativeKernel(fn, dim3(G), dim3(PANEL_NT), args, (unsigned)lds, s);
}

hipError_t panel_max_blocks(int nc, int kb, int R, int64_t nr, int *maxblocks) {
  const size_t lds = panel_lds_bytes(nc, kb, R, nr);
  const void *fn = panel_kernel_ptr(nc);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int per = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, PANEL_NT, lds);
  if (e != hipSuccess) return e;
  int dev = 0, ncu = 0;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  *maxblocks = per * ncu;
  return hipSuccess;
}

hipError_t launch_laswp(int nc, double *A, int64_t lda, int64_t k, int64_t c0, int64_t c1,
                        const int *perm, const int *moved, const int *nmoved, hipStream_t s) {
  if (c1 <= c0) return hipSuccess;
  dim3 g((unsigned)(c1 - c0));
  if (nc == 2) hipLaunchKernelGGL(k_laswp<2>, g, dim3(256), 0, s, A, lda, k, c0, c1, perm, moved, nmoved);
  else if (nc == 3) hipLaunchKernelGGL(k_laswp<3>, g, dim3(256), 0, s, A, lda, k, c0, c1, perm, moved, nmoved);
  else hipLaunchKernelGGL(k_laswp<4>, g, dim3(256), 0, s, A, lda, k, c0, c1, perm, moved, nmoved);
  return hipGetLastError();
}

template <int NC>
static void trsm_l(int kb, dim3 g, hipStream_t s, const double *L, int64_t lda, double *X,
                   int64_t ldx, int64_t ncols) {
  if (kb <= 64)
    hipLaunchKernelGGL((k_trsm_lower_unit_w<NC, 1>), dim3((unsigned)((ncols + 3) / 4)), dim3(256),
                       0, s, L, lda, X, ldx, kb, ncols);
  else if (kb <= 128)
    hipLaunchKernelGGL((k_trsm_lower_unit_w<NC, 2>), dim3((unsigned)((ncols + 1) / 2)),
                       dim3(256), 0, s, L, lda, X, ldx, kb, ncols);
  else if (kb <= 256)
    hipLaunchKernelGGL((k_trsm_lower_unit_w<NC, 4>), dim3((unsigned)ncols), dim3(256), 0, s, L,
                       lda, X, ldx, kb, ncols);
  else
    hipLaunchKernelGGL((k_trsm_lower_unit<NC, 1, 2>), g, dim3(256), 0, s, L, lda, X, ldx, kb, ncols);
}

hipError_t launch_trsm_lower_unit(int nc, const double *L, int64_t lda, double *X, int64_t ldx,
                                  int kb, int64_t ncols, hipStream_t s) {
  if (ncols <= 0 || kb <= 0) return hipSuccess;
  if (kb > 512) return hipErrorInvalidValue;
  const int cpb = kb <= 256 ? 2 : 1;
  dim3 g((unsigned)((ncols + cpb - 1) / cpb));
  if (nc == 2) trsm_l<2>(kb, g, s, L, lda, X, ldx, ncols);
  else if (nc == 3) trsm_l<3>(kb, g, s, L, lda, X, ldx, ncols);
  else trsm_l<4>(kb, g, s, L, lda, X, ldx, ncols);
  return hipGetLastError();
}

template <int NC>
static void trsm_u(int kb, dim3 g, hipStream_t s, const double *U, int64_t lda, double *X,
                   int64_t ldx, int64_t ncols) {
  if (kb <= 256) hipLaunchKernelGGL((k_trsm_upper<NC, 1, 1>), g, dim3(256), 0, s, U, lda, X, ldx, kb, ncols);
  else hipLaunchKernelGGL((k_trsm_upper<NC, 1, 2>), g, dim3(256), 0, s, U, lda, X, ldx, kb, ncols);
}

hipError_t launch_trsm_upper(int nc, const double *U, int64_t lda, double *X, int64_t ldx, int kb,
                             int64_t ncols, hipStream_t s) {
  if (ncols <= 0 || kb <= 0) return hipSuccess;
  if (kb > 512) return hipErrorInvalidValue;
  dim3 g((unsigned)ncols);
  if (nc == 2) trsm_u<2>(kb, g, s, U, lda, X, ldx, ncols);
  else if (nc == 3) trsm_u<3>(kb, g, s, U, lda, X, ldx, ncols);
  else trsm_u<4>(kb, g, s, U, lda, X, ldx, ncols);
  return hipGetLastError();
}

template <int NC>
static void naive_nc(int64_t M, int64_t N, hipStream_t s, const double *A, int64_t lda,
                     const double *B, int64_t ldb, double *C, int64_t ldc, int64_t K, int desc) {
  if (N >= 16) {
    dim3 g((unsigned)((M + 15) / 16), (unsigned)((N + 15) / 16));
    hipLaunchKernelGGL((k_naive_gemm<NC, 16, 16>), g, dim3(256), 0, s, A, lda, B, ldb, C, ldc, M, N, K, desc);
  } else {
    dim3 g((unsigned)((M + 255) / 256), (unsigned)N);
    hipLaunchKernelGGL((k_naive_gemm<NC, 256, 1>), g, dim3(256), 0, s, A, lda, B, ldb, C, ldc, M, N, K, desc);
  }
}

hipError_t launch_naive_gemm(int nc, const double *A, int64_t lda, const double *B, int64_t ldb,
                             double *C, int64_t ldc, int64_t M, int64_t N, int64_t K, int desc,
                             hipStream_t s) {
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  if (nc == 2) naive_nc<2>(M, N, s, A, lda, B, ldb, C, ldc, K, desc);
  else if (nc == 3) naive_nc<3>(M, N, s, A, lda, B, ldb, C, ldc, K, desc);
  else naive_nc<4>(M, N, s, A, lda, B, ldb, C, ldc, K, desc);
  return hipGetLastError();
}

hipError_t launch_apply_ipiv(int nc, double *B, int64_t ldb, int64_t n, int64_t nrhs,
                             const int64_t *ipiv, hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  const size_t lds = (size_t)n * nc * 8 + (size_t)n * 8;  // expansions + pivots + sources
  const int use_lds = lds <= 160 * 1024 ? 1 : 0;
  const void *fn = nc == 2 ? (const void *)k_apply_ipiv<2>
                           : (nc == 3 ? (const void *)k_apply_ipiv<3> : (const void *)k_apply_ipiv<4>);
  if (use_lds) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  dim3 g((unsigned)nrhs);
  const unsigned shm = use_lds ? (unsigned)lds : 0u;
  if (nc == 2) hipLaunchKernelGGL(k_apply_ipiv<2>, g, dim3(256), shm, s, B, ldb, n, ipiv, use_lds);
  else if (nc == 3) hipLaunchKernelGGL(k_apply_ipiv<3>, g, dim3(256), shm, s, B, ldb, n, ipiv, use_lds);
  else hipLaunchKernelGGL(k_apply_ipiv<4>, g, dim3(256), shm, s, B, ldb, n, ipiv, use_lds);
  return hipGetLastError();
}

hipError_t launch_trsv(int nc, int fwd, const double *LU, int64_t lda, double *x, int64_t n,
                       uint32_t *sync, int *err, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int G = (int)((n + TRSV_R - 1) / TRSV_R);
  // sync[0]: finished positions, sync[1]: ticket of the next row block
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(256), 0, s, (int *)sync, 0, (int64_t)2);
#define OZ_TRSV(NC_, F_)                                                                      \
  hipLaunchKernelGGL((k_trsv<NC_, F_>), dim3((unsigned)G), dim3(256), 0, s, LU, lda, x, n, sync, \
                     sync + 1, err)
  if (fwd) {
    if (nc == 2) OZ_TRSV(2, true); else if (nc == 3) OZ_TRSV(3, true); else OZ_TRSV(4, true);
  } else {
    if (nc == 2) OZ_TRSV(2, false); else if (nc == 3) OZ_TRSV(3, false); else OZ_TRSV(4, false);
  }
#undef OZ_TRSV
  return hipGetLastError();
}

hipError_t launch_fill_int(int *p, int v, int64_t cnt, hipStream_t s) {
  if (cnt <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_int, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, p, v, cnt);
  return hipGetLastError();
}

}  // namespace ozl
