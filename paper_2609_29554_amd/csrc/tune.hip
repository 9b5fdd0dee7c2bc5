// Autotuner of the LU configuration for one precision and order n: panel
// width b, Schur-update back-end (or the native update), the schedule (with
// or without look-ahead), then for the winner the slice count S and the
// (S4) workgroup tile.
//
// The paper sizes the slices with a cost model (Eq. Lhint) and ranks the
// engines by bits per modulus times throughput, but finds that only timing at
// the actual size is trustworthy (Sec. 4.1).  Here the model only orders the
// candidates; every feasible candidate is then timed with HIP events around
// a full ozII_getrf of a synthetic diagonally dominant matrix of the
// requested order, and the fastest wins.  Stage 2 times the winner with S
// one above the plan rule's minimum (Eq. Lhint trades slices against
// conversion cost) and with each GEMM tile.  Results are cached in a JSON
// file, one object per line, keyed by device, component count and n.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/ozii.h"

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ull;
  x ^= x >> 33;
  return x;
}

// Synthetic matrix for timing: a_ij = u_ij + n [i == j], u in [-1, 1), lower
// components below half an ulp of the one above.
template <int NC>
__global__ __launch_bounds__(256) void k_tune_fill(double *A, int64_t n, uint64_t seed) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * n) return;
  const int64_t i = e % n, j = e / n;
  double x0 = (double)(int64_t)(mix64(seed ^ (uint64_t)e) >> 11) * 0x1p-52 - 1.0;
  if (i == j) x0 += (double)n;
  int ex = 0;
  __builtin_frexp(x0, &ex);
  double *dst = A + e * NC;
  dst[0] = x0;
#pragma unroll
  for (int c = 1; c < NC; ++c) {
    const double u = (double)(mix64(seed + 0x9e3779b97f4a7c15ull * (uint64_t)c ^ (uint64_t)e) >> 11) * 0x1p-53;
    dst[c] = __builtin_ldexp(u - 0.5, ex - 53 * c - 1);
  }
}

// Synthetic limb matrix for timing: random normalised mantissas, random
// signs, exponents in [-2, 2] (no diagonal dominance: the pivot search and
// interchanges run as on a general matrix).
__global__ __launch_bounds__(256) void k_tune_fill_limbs(uint64_t *limb, int32_t *ex, uint8_t *sg,
                                                         int64_t n, int nl, uint64_t seed) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * n) return;
  for (int q = 0; q < nl; ++q) {
    uint64_t v = mix64(seed ^ ((uint64_t)e * 64 + (uint64_t)q));
    if (q == nl - 1) v |= 1ull << 63;
    limb[(int64_t)q * n * n + e] = v;
  }
  const uint64_t h = mix64(~seed ^ (uint64_t)e);
  ex[e] = (int32_t)(h % 5) - 2;
  sg[e] = (uint8_t)((h >> 32) & 1u);
}

struct Cand {
  ozII_opts o;
  double model_ms;
  double ms;
};

double peak_ops(int backend) {
  // dense MFMA peaks of MI355X [op/s] for the modular products
  if (backend == OZII_BE_F64MOD) return 78.6e12;
  if (backend == OZII_BE_FP8_B17) return 5.0e15;
  if (backend == OZII_BE_FP16) return 2.5e15;
  return 5.0e15;
}

// Cost model (ordering only): per Schur update, MFMA time at a quarter of the
// engine's peak (issued operations: x4 for FP8) plus residue-plane, t-plane
// and A22 traffic at half the HBM bandwidth; native updates at the measured
// order of magnitude of an expansion multiply-subtract per element; the panel
// at ~20 us per column.
double model_ms(int nc, int64_t n, const ozII_opts &o) {
  const int b = o.block;
  const double panel = 20e-6 * (double)n;
  double t = 0.0;
  for (int64_t k = 0; k + b < n; k += b) {
    const double m = (double)(n - k - b);
    if (o.method == OZII_METHOD_NAIVE) {
      t += m * m * b * 500.0 / (256.0 * 64.0 * 2.4e9);  // ~500 VALU ops per QD fms
      continue;
    }
    int32_t S = 0, w = 0, Q = 0, N = 0;
    if (ozII_plan_query(53 * nc, b, &o, &S, &w, &Q, &N, nullptr) != OZII_OK) return 1e30;
    const int ng = S;  // kept groups S-1..2S-2
    const double pairs = (double)S * (S + 1) / 2.0;
    const double br = o.backend == OZII_BE_F64MOD ? 8.0 : (o.backend == OZII_BE_FP8_B17 ? 2.0 : 1.0);
    const double bt = o.backend == OZII_BE_F64MOD ? 4.0 : 1.0;
    const double ops = 2.0 * m * m * b * pairs * N * (o.backend == OZII_BE_FP8_B17 ? 4.0 : 1.0);
    const double bytes = 2.0 * m * b * (8.0 * nc + S * N * br) + 2.0 * ng * N * m * m * bt + 16.0 * nc * m * m;
    t += ops / (0.25 * peak_ops(o.backend)) + bytes / 4e12;
  }
  // look-ahead: the update runs beside the next panel on half the device
  if (!(o.flags & OZII_F_NO_LOOKAHEAD)) t = std::max(0.0, 2.0 * t - panel) + 0.1 * t;
  return (panel + t) * 1e3;
}

std::string device_key(int nc, int64_t n, const char *fmt = "nc") {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  hipDeviceProp_t prop;
  std::string name = "unknown";
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) name = std::string(prop.gcnArchName);
  std::ostringstream k;
  k << name << "|" << fmt << "=" << nc << "|n=" << n;
  return k.str();
}

bool cache_lookup(const char *path, const std::string &key, ozII_opts *o, double *ms) {
  std::ifstream f(path);
  if (!f) return false;
  std::string line, want = "\"key\": \"" + key + "\"";
  while (std::getline(f, line)) {
    if (line.find(want) == std::string::npos) continue;
    int be = 0, me = 0, b = 0, s = 0, t = 0, fl = 0, lf = 0;
    double v = 0;
    const size_t p = line.find("\"backend\"");
    if (p == std::string::npos) return false;
    if (std::sscanf(line.c_str() + p,
                    "\"backend\": %d, \"method\": %d, \"block\": %d, \"nslice\": %d, "
                    "\"gemm_tile\": %d, \"flags\": %d, \"ms\": %lf",
                    &be, &me, &b, &s, &t, &fl, &v) != 7)
      return false;
    const size_t pl = line.find("\"panel_leaf\"");
    if (pl != std::string::npos && std::sscanf(line.c_str() + pl, "\"panel_leaf\": %d", &lf) != 1)
      return false;
    std::memset(o, 0, sizeof(*o));
    o->panel_leaf = lf;
    o->backend = be;
    o->method = me;
    o->block = b;
    o->nslice = s;
    o->gemm_tile = t;
    o->flags = fl;
    *ms = v;
    return true;
  }
  return false;
}

void cache_store(const char *path, const std::string &key, const ozII_opts &o, double ms) {
  std::vector<std::string> keep;
  {
    std::ifstream f(path);
    std::string line, want = "\"key\": \"" + key + "\"";
    while (f && std::getline(f, line))
      if (line.find("\"key\"") != std::string::npos && line.find(want) == std::string::npos) {
        while (!line.empty() && (line.back() == ',' || line.back() == ' ')) line.pop_back();
        keep.push_back(line);
      }
  }
  char buf[512];
  std::snprintf(buf, sizeof(buf),
                "{\"key\": \"%s\", \"backend\": %d, \"method\": %d, \"block\": %d, \"nslice\": %d, "
                "\"gemm_tile\": %d, \"flags\": %d, \"ms\": %.4f, \"panel_leaf\": %d}",
                key.c_str(), o.backend, o.method, o.block, o.nslice, o.gemm_tile, o.flags, ms,
                o.panel_leaf);
  keep.push_back(buf);
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp, std::ios::trunc);
    f << "[\n";
    for (size_t i = 0; i < keep.size(); ++i) f << keep[i] << (i + 1 < keep.size() ? ",\n" : "\n");
    f << "]\n";
  }
  std::rename(tmp.c_str(), path);
}

}  // namespace

extern "C" ozII_status ozII_stream_of(ozII_handle h, void **stream);

extern "C" ozII_status ozII_tune(ozII_handle h, int32_t nc, int64_t n, const char *cache_path,
                                 int32_t flags, ozII_opts *best, ozII_tune_report *rep) {
  if (!h || !best || nc < 2 || nc > 4 || n < 2 || n > (1 << 16)) return OZII_EINVAL;
  if (flags & ~OZII_TUNE_RETUNE) return OZII_EINVAL;
  const std::string key = device_key(nc, n);
  if (rep) std::memset(rep, 0, sizeof(*rep));
  if (cache_path && !(flags & OZII_TUNE_RETUNE)) {
    double ms = 0;
    if (cache_lookup(cache_path, key, best, &ms)) {
      if (rep) {
        rep->from_cache = 1;
        rep->ncand = 1;
        rep->cand[0] = *best;
        rep->ms[0] = ms;
      }
      return OZII_OK;
    }
  }
  // stage 1 candidates: panel width x (three back-ends + the native update)
  // x schedule (look-ahead or not)
  std::vector<Cand> cands;
  for (int b : {64, 128, 256, 512}) {
    if (b >= n) continue;
    for (int be : {(int)OZII_BE_INT8, (int)OZII_BE_FP8_B17, (int)OZII_BE_F64MOD, (int)OZII_BE_FP16,
                   0}) {
      for (int fl : {0, (int)OZII_F_NO_LOOKAHEAD}) {
        Cand c;
        std::memset(&c.o, 0, sizeof(c.o));
        c.o.block = b;
        c.o.backend = be ? be : OZII_BE_INT8;
        c.o.method = be ? OZII_METHOD_OZAKI : OZII_METHOD_NAIVE;
        c.o.flags = fl;
        if (be) {
          int32_t S, w, Q, N;
          if (ozII_plan_query(53 * nc, b, &c.o, &S, &w, &Q, &N, nullptr) != OZII_OK) continue;
        }
        c.model_ms = model_ms(nc, n, c.o);
        c.ms = 0;
        cands.push_back(c);
      }
    }
  }
  if (cands.empty()) {
    // n too small for any blocked candidate: unblocked
    std::memset(best, 0, sizeof(*best));
    best->block = (int32_t)std::max<int64_t>(1, n - 1);
    best->method = OZII_METHOD_NAIVE;
    return OZII_OK;
  }
  std::sort(cands.begin(), cands.end(), [](const Cand &a, const Cand &b) { return a.model_ms < b.model_ms; });
  // room for stage 2 (up to 8 refinements of the winner)
  if ((int)cands.size() > OZII_TUNE_MAXCAND - 8) cands.resize(OZII_TUNE_MAXCAND - 8);

  void *sv = nullptr;
  ozII_status st = ozII_stream_of(h, &sv);
  if (st != OZII_OK) return st;
  hipStream_t s = (hipStream_t)sv;
  double *A = nullptr;
  int64_t *ipiv = nullptr;
  int32_t *info = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc((void **)&A, sizeof(double) * nc * n * n);
  if (e == hipSuccess) e = hipMalloc((void **)&ipiv, sizeof(int64_t) * n);
  if (e == hipSuccess) e = hipMalloc((void **)&info, sizeof(int32_t));
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  auto cleanup = [&]() {  // best effort: the status of the tuning itself is what is returned
    if (A) (void)hipFree(A);
    if (ipiv) (void)hipFree(ipiv);
    if (info) (void)hipFree(info);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if (e != hipSuccess) {
    cleanup();
    return e == hipErrorOutOfMemory ? OZII_ENOMEM : OZII_EHIP;
  }
  const unsigned grid = (unsigned)((n * n + 255) / 256);
  auto fill = [&]() {
    if (nc == 2) hipLaunchKernelGGL(k_tune_fill<2>, dim3(grid), dim3(256), 0, s, A, n, 20260929ull);
    else if (nc == 3) hipLaunchKernelGGL(k_tune_fill<3>, dim3(grid), dim3(256), 0, s, A, n, 20260929ull);
    else hipLaunchKernelGGL(k_tune_fill<4>, dim3(grid), dim3(256), 0, s, A, n, 20260929ull);
    return hipGetLastError();
  };
  // Candidates the library cannot run at this size (a panel that does not
  // fit in LDS, a plan beyond the compiled word sizes) report
  // OZII_EUNSUPPORTED before anything is enqueued and are skipped; any other
  // failure ends the tuning.
  std::vector<Cand> timed;
  auto time_all = [&](const std::vector<Cand> &list) {
    for (size_t ci = 0; ci < list.size() && (int)timed.size() < OZII_TUNE_MAXCAND; ++ci) {
      Cand c = list[ci];
      st = ozII_reserve(h, nc, 0, 0, 0, n, &c.o);
      float ms = 0;
      for (int rep_i = 0; rep_i < 2 && st == OZII_OK; ++rep_i) {  // warm-up, then timed
        if ((e = fill()) != hipSuccess) break;
        if ((e = hipEventRecord(e0, s)) != hipSuccess) break;
        st = ozII_getrf(h, nc, n, A, n, ipiv, info, &c.o);
        if (st != OZII_OK) break;
        if ((e = hipEventRecord(e1, s)) != hipSuccess) break;
        if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
        if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
      }
      if (st == OZII_EUNSUPPORTED && e == hipSuccess) {
        st = OZII_OK;
        continue;
      }
      if (st == OZII_OK && e == hipSuccess) st = ozII_sync_check(h);
      if (st != OZII_OK || e != hipSuccess) return;
      c.ms = ms;
      timed.push_back(c);
    }
  };
  time_all(cands);
  // stage 2: the winner with one slice more and with every GEMM tile
  if (st == OZII_OK && e == hipSuccess && !timed.empty()) {
    int w0 = 0;
    for (size_t ci = 1; ci < timed.size(); ++ci)
      if (timed[ci].ms < timed[w0].ms) w0 = (int)ci;
    const Cand win = timed[w0];
    if (win.o.method == OZII_METHOD_OZAKI) {
      std::vector<Cand> ref;
      int32_t S = 0, w = 0, Q = 0, N = 0;
      if (ozII_plan_query(53 * nc, win.o.block, &win.o, &S, &w, &Q, &N, nullptr) == OZII_OK) {
        for (int ns : {0, S + 1})
          for (int tile : {(int)OZII_TILE_AUTO, (int)OZII_TILE_128x128, (int)OZII_TILE_256x128,
                           (int)OZII_TILE_256x256}) {
            if (ns == 0 && tile == OZII_TILE_AUTO) continue;  // the winner itself
            if (win.o.backend != OZII_BE_INT8 && tile != OZII_TILE_AUTO) continue;
            Cand c = win;
            c.o.nslice = ns;
            c.o.gemm_tile = tile;
            int32_t S2, w2, Q2, N2;
            if (ozII_plan_query(53 * nc, c.o.block, &c.o, &S2, &w2, &Q2, &N2, nullptr) != OZII_OK)
              continue;
            c.model_ms = model_ms(nc, n, c.o);
            c.ms = 0;
            ref.push_back(c);
          }
      }
      if (win.o.backend == OZII_BE_INT8) {
        // and with the fused (S4)-(S6) kernel
        Cand c = win;
        c.o.flags |= OZII_F_FUSED;
        ref.push_back(c);
      }
      time_all(ref);
    }
  }
  cleanup();
  if (st != OZII_OK) return st;
  if (e != hipSuccess) return OZII_EHIP;
  if (timed.empty()) return OZII_EUNSUPPORTED;
  // the fused (S4)-(S6) kernel only when it is clearly faster: stand-alone it
  // is the slower product, inside the LU its time hides behind the panel and
  // a tie is timing noise
  int bi = -1, bf = -1;
  for (size_t ci = 0; ci < timed.size(); ++ci) {
    int &b = (timed[ci].o.flags & OZII_F_FUSED) ? bf : bi;
    if (b < 0 || timed[ci].ms < timed[b].ms) b = (int)ci;
  }
  if (bi < 0 || (bf >= 0 && timed[bf].ms < 0.97 * timed[bi].ms)) bi = bf;
  *best = timed[bi].o;
  if (rep) {
    rep->ncand = (int32_t)timed.size();
    rep->best = bi;
    for (size_t ci = 0; ci < timed.size(); ++ci) {
      rep->cand[ci] = timed[ci].o;
      rep->ms[ci] = timed[ci].ms;
      rep->model_ms[ci] = timed[ci].model_ms;
    }
  }
  if (cache_path) cache_store(cache_path, key, *best, timed[bi].ms);
  return OZII_OK;
}

extern "C" ozII_status ozII_getrf_limbs(ozII_handle h, int32_t nlimb, int64_t n, ozII_limbs *A,
                                        int64_t *ipiv, int32_t *info, const ozII_opts *o);

// The limb-format LU: stage 1 times the panel width b (64 .. 512 below n) x
// the panel leaf (0 = unblocked panel, 16, 32, 64 below b) with the Ozaki-II
// update, and the native update (unblocked panel) at each b while n <= 512
// (beyond, its O(n^3) p-bit multiply-subtracts take minutes); stage 2 times
// the winner with each GEMM tile and with S one above the plan rule's.
extern "C" ozII_status ozII_tune_limbs(ozII_handle h, int32_t nlimb, int64_t n,
                                       const char *cache_path, int32_t flags, ozII_opts *best,
                                       ozII_tune_report *rep) {
  if (!h || !best || nlimb < 1 || nlimb > 64 || n < 2 || n > (1 << 15)) return OZII_EINVAL;
  if (flags & ~OZII_TUNE_RETUNE) return OZII_EINVAL;
  const std::string key = device_key(nlimb, n, "nlimb");
  if (rep) std::memset(rep, 0, sizeof(*rep));
  if (cache_path && !(flags & OZII_TUNE_RETUNE)) {
    double ms = 0;
    if (cache_lookup(cache_path, key, best, &ms)) {
      if (rep) {
        rep->from_cache = 1;
        rep->ncand = 1;
        rep->cand[0] = *best;
        rep->ms[0] = ms;
      }
      return OZII_OK;
    }
  }
  const int p = 64 * nlimb;
  std::vector<Cand> cands;
  for (int b : {64, 128, 256, 512}) {
    if (b >= n) continue;
    for (int lf : {0, 16, 32, 64}) {
      if (lf >= b) continue;
      Cand c;
      std::memset(&c.o, 0, sizeof(c.o));
      c.o.block = b;
      c.o.backend = OZII_BE_INT8;
      c.o.method = OZII_METHOD_OZAKI;
      c.o.panel_leaf = lf;
      int32_t S, w, Q, N;
      if (ozII_plan_query(p, b, &c.o, &S, &w, &Q, &N, nullptr) != OZII_OK) continue;
      // model: only orders the candidates (wider leaves, then b)
      c.model_ms = (double)(lf ? lf : b) + 1e-3 * b;
      c.ms = 0;
      cands.push_back(c);
    }
    if (n <= 512) {
      Cand c;
      std::memset(&c.o, 0, sizeof(c.o));
      c.o.block = b;
      c.o.method = OZII_METHOD_NAIVE;
      c.model_ms = 1e6 + b;
      c.ms = 0;
      cands.push_back(c);
    }
  }
  if (cands.empty()) {
    std::memset(best, 0, sizeof(*best));
    best->block = (int32_t)n;
    best->method = OZII_METHOD_NAIVE;
    return OZII_OK;
  }
  std::sort(cands.begin(), cands.end(), [](const Cand &a, const Cand &b) { return a.model_ms < b.model_ms; });
  if ((int)cands.size() > OZII_TUNE_MAXCAND - 7) cands.resize(OZII_TUNE_MAXCAND - 7);

  void *sv = nullptr;
  ozII_status st = ozII_stream_of(h, &sv);
  if (st != OZII_OK) return st;
  hipStream_t s = (hipStream_t)sv;
  uint64_t *limb = nullptr;
  int32_t *ex = nullptr, *info = nullptr;
  uint8_t *sg = nullptr;
  int64_t *ipiv = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc((void **)&limb, sizeof(uint64_t) * nlimb * n * n);
  if (e == hipSuccess) e = hipMalloc((void **)&ex, sizeof(int32_t) * n * n);
  if (e == hipSuccess) e = hipMalloc((void **)&sg, (size_t)(n * n));
  if (e == hipSuccess) e = hipMalloc((void **)&ipiv, sizeof(int64_t) * n);
  if (e == hipSuccess) e = hipMalloc((void **)&info, sizeof(int32_t));
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  auto cleanup = [&]() {
    if (limb) (void)hipFree(limb);
    if (ex) (void)hipFree(ex);
    if (sg) (void)hipFree(sg);
    if (ipiv) (void)hipFree(ipiv);
    if (info) (void)hipFree(info);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if (e != hipSuccess) {
    cleanup();
    return e == hipErrorOutOfMemory ? OZII_ENOMEM : OZII_EHIP;
  }
  ozII_limbs A;
  A.limb = limb;
  A.exp = ex;
  A.sign = sg;
  A.ld = n;
  A.plane = n * n;
  const unsigned grid = (unsigned)((n * n + 255) / 256);
  std::vector<Cand> timed;
  auto time_all = [&](const std::vector<Cand> &list) {
    for (size_t ci = 0; ci < list.size() && (int)timed.size() < OZII_TUNE_MAXCAND; ++ci) {
      Cand c = list[ci];
      float ms = 0;
      for (int rep_i = 0; rep_i < 2 && st == OZII_OK; ++rep_i) {  // warm-up, then timed
        hipLaunchKernelGGL(k_tune_fill_limbs, dim3(grid), dim3(256), 0, s, limb, ex, sg, n, nlimb,
                           20261203ull);
        if ((e = hipGetLastError()) != hipSuccess) break;
        if ((e = hipEventRecord(e0, s)) != hipSuccess) break;
        st = ozII_getrf_limbs(h, nlimb, n, &A, ipiv, info, &c.o);
        if (st != OZII_OK) break;
        if ((e = hipEventRecord(e1, s)) != hipSuccess) break;
        if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
        if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
      }
      if (st == OZII_EUNSUPPORTED && e == hipSuccess) {
        st = OZII_OK;
        continue;
      }
      if (st == OZII_OK && e == hipSuccess) st = ozII_sync_check(h);
      if (st != OZII_OK || e != hipSuccess) return;
      c.ms = ms;
      timed.push_back(c);
    }
  };
  time_all(cands);
  if (st == OZII_OK && e == hipSuccess && !timed.empty()) {
    int w0 = 0;
    for (size_t ci = 1; ci < timed.size(); ++ci)
      if (timed[ci].ms < timed[w0].ms) w0 = (int)ci;
    const Cand win = timed[w0];
    if (win.o.method == OZII_METHOD_OZAKI) {
      std::vector<Cand> ref;
      int32_t S = 0, w = 0, Q = 0, N = 0;
      if (ozII_plan_query(p, win.o.block, &win.o, &S, &w, &Q, &N, nullptr) == OZII_OK) {
        for (int ns : {0, S + 1})
          for (int tile : {(int)OZII_TILE_AUTO, (int)OZII_TILE_128x128, (int)OZII_TILE_256x128,
                           (int)OZII_TILE_256x256}) {
            if (ns == 0 && tile == OZII_TILE_AUTO) continue;
            Cand c = win;
            c.o.nslice = ns;
            c.o.gemm_tile = tile;
            int32_t S2, w2, Q2, N2;
            if (ozII_plan_query(p, c.o.block, &c.o, &S2, &w2, &Q2, &N2, nullptr) != OZII_OK)
              continue;
            c.ms = 0;
            ref.push_back(c);
          }
      }
      time_all(ref);
    }
  }
  cleanup();
  if (st != OZII_OK) return st;
  if (e != hipSuccess) return OZII_EHIP;
  if (timed.empty()) return OZII_EUNSUPPORTED;
  int bi = 0;
  for (size_t ci = 1; ci < timed.size(); ++ci)
    if (timed[ci].ms < timed[bi].ms) bi = (int)ci;
  *best = timed[bi].o;
  if (rep) {
    rep->ncand = (int32_t)timed.size();
    rep->best = bi;
    for (size_t ci = 0; ci < timed.size(); ++ci) {
      rep->cand[ci] = timed[ci].o;
      rep->ms[ci] = timed[ci].ms;
      rep->model_ms[ci] = timed[ci].model_ms;
    }
  }
  if (cache_path) cache_store(cache_path, key, *best, timed[bi].ms);
  return OZII_OK;
}
