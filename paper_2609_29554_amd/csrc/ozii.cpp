// Host side of libozii: the plan rule, the device plan tables, workspace
// management and the orchestration of the product, the LU and the solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/ozii.h"
#include "ozii_elem.hpp"
#include "ozii_kernels.hpp"

namespace {

using ozk::DevPlan;

enum {
  OZ_STAGE_EXP = 0,
  OZ_STAGE_PRODUCER = 1,
  OZ_STAGE_GEMM = 2,
  OZ_STAGE_CONSUMER = 3,
  OZ_STAGE_PANEL = 4,
  OZ_STAGE_LASWP = 5,
  OZ_STAGE_TRSM = 6,
  OZ_STAGE_NAIVE = 7,
  OZ_STAGE_GETRS = 8,
  OZ_STAGE_ROUND = 9,  // limb format: rounding of the group sums and the update
  OZ_STAGE_FUSED = 10, // (S4)-(S6) in one kernel (OZII_F_FUSED)
  OZ_NSTAGES = 11
};

// ---------------------------------------------------------------------------
// Plan rule (Sec. 3.2, paragraph "Determining w and N"):
//   slack = ceil(log2 2K) + 16 + g_ex; for S = 1, 2, ...:
//   w = ceil((p + slack)/S), need = 2w + log2 K + log2 S + 5,
//   N = fewest leading moduli whose cumulative log2 exceeds need;
//   accept the first S whose need fits and whose accumulator bound holds.
// Moduli: the 54 largest prime powers <= 256, descending (54 moduli and
// 362.8 bits in Sec. 3.2).
// ---------------------------------------------------------------------------
std::vector<int> int8_moduli() {
  std::vector<int> out;
  for (int p = 2; p <= 256; ++p) {
    bool prime = true;
    for (int d = 2; d * d <= p; ++d)
      if (p % d == 0) {
        prime = false;
        break;
      }
    if (!prime) continue;
    int q = p;
    while (q * p <= 256) q *= p;
    out.push_back(q);
  }
  std::sort(out.begin(), out.end(), std::greater<int>());
  return out;
}

// binary64-moduli back-end (Sec. "binary64 back-end", Eq. fp64mod): the
// F64_MAXMOD largest primes m with K S m^2 < 2^53, descending, so that every
// digit-group product (inner dimension K npairs <= K S) accumulates exactly
// in FP64.  At most 20 of them: read this way the plan reproduces the
// DD/TD/QD GEMM counts 13/18/36 printed for K = 512.
constexpr int F64_MAXMOD = 20;

bool is_prime(int64_t n) {
  if (n < 2) return false;
  for (int64_t d = 2; d * d <= n; ++d)
    if (n % d == 0) return false;
  return true;
}

std::vector<int> f64_moduli(int64_t K, int S) {
  std::vector<int> out;
  const double ks = (double)K * S;
  int64_t m = (int64_t)std::floor(std::sqrt(9007199254740992.0 / ks)) + 2;
  for (; m > 2 && (int)out.size() < F64_MAXMOD; --m) {
    if (ks * (double)m * (double)m >= 9007199254740992.0) continue;  // exact: all terms < 2^53
    if (is_prime(m)) out.push_back((int)m);
  }
  return out;
}

struct HostPlan {
  int p = 0;
  int64_t K = 0;
  int backend = OZII_BE_INT8;
  int S = 0, w = 0, Q = 0, nmod = 0, g0 = 0, ng = 0;
  int nwx = 0, nh = 0, nwc = 0, nd = 0;
  double need = 0;
  std::vector<int> mods;
  // storage of one back-end: bytes per plane element, planes per (slice,
  // modulus), bytes per t-value, inner-dimension padding
  int el_bytes() const { return backend == OZII_BE_F64MOD ? 8 : 1; }
  int planes_per() const { return backend == OZII_BE_FP8_B17 ? 2 : 1; }
  int t_bytes() const { return backend == OZII_BE_F64MOD ? 4 : 1; }
  int k_align() const { return backend == OZII_BE_FP8_B17 ? 128 : 64; }
  int planes_kind() const {
    return backend == OZII_BE_F64MOD ? ozl::PLANES_F64
                                     : backend == OZII_BE_FP8_B17 ? ozl::PLANES_F8 : ozl::PLANES_I8;
  }
};

// Accumulator bounds: INT8 K S 128^2 < 2^31 (residues in [-128, 127]); FP8
// the same (it also keeps 2 K S 64 < 2^24, so the three FP32 sub-product
// accumulators are exact); binary64 holds by the choice of the moduli.
bool accum_ok(int backend, int64_t K, int S) {
  const double ks = (double)K * S;
  // FP16: FP32 partial sums of at most 1024 products (exact), folded into
  // int32: the INT8 bound
  if (backend == OZII_BE_INT8 || backend == OZII_BE_FP16) return ks * 128.0 * 128.0 < 2147483648.0;
  if (backend == OZII_BE_FP8_B17) return ks * 128.0 * 128.0 < 2147483648.0 && 2.0 * ks * 64.0 < 16777216.0;
  return true;
}

ozII_status make_plan(int p, int64_t K, const ozII_opts *o, HostPlan &pl, std::string *why,
                      bool check_sizes = true) {
  const int backend = (o && o->backend) ? o->backend : OZII_BE_INT8;
  const int nslice = o ? o->nslice : 0;
  const int extra = o ? o->extra_groups : 0;
  const int gex = o ? o->guard_ex : 0;
  const int qbits = o ? o->qbits : 0;
  if (p <= 0 || K <= 0 || nslice < 0 || extra < 0 || gex < 0 || qbits < 0) return OZII_EINVAL;
  if (qbits > 0 && (nslice > 1 || extra > 0)) {
    if (why) *why = "qbits: one slice and no extra groups";
    return OZII_EINVAL;
  }
  if (o && (o->gemm_tile < OZII_TILE_AUTO || o->gemm_tile > OZII_TILE_256x256)) {
    if (why) *why = "gemm_tile must be 0..3";
    return OZII_EINVAL;
  }
  if (backend < OZII_BE_INT8 || backend > OZII_BE_FP16) {
    if (why) *why = "unknown back-end";
    return OZII_EINVAL;
  }
  const std::vector<int> mods8 = int8_moduli();
  const int slack = (int)std::ceil(std::log2(2.0 * (double)K)) + 16 + gex;
  // qbits: the unsliced product of Sec. 3.1 at a stated scaling, |X| <
  // 2^qbits: S = 1, Q = w = qbits + 1, and N covers the CRT range 2 K
  // 2^(2 qbits) of the exact products (need = 1 + log2 K + 2 qbits)
  const int s_lo = qbits > 0 ? 1 : (nslice > 0 ? nslice : 1);
  const int s_hi = qbits > 0 ? 1 : (nslice > 0 ? nslice : 4096);
  bool any_acc = false;
  for (int S = s_lo; S <= s_hi; ++S) {
    if (!accum_ok(backend, K, S)) continue;
    const std::vector<int> mods = backend == OZII_BE_F64MOD ? f64_moduli(K, S) : mods8;
    if (mods.empty()) continue;
    any_acc = true;
    const int w = qbits > 0 ? qbits + 1 : (p + slack + S - 1) / S;
    const double need = qbits > 0 ? 1.0 + std::log2((double)K) + 2.0 * qbits
                                  : 2.0 * w + std::log2((double)K) + std::log2((double)S) + 5.0;
    double cum = 0.0;
    int N = 0;
    for (size_t i = 0; i < mods.size(); ++i) {
      cum += std::log2((double)mods[i]);
      if (cum > need) {
        N = (int)i + 1;
        break;
      }
    }
    if (N == 0) continue;
    pl.p = p;
    pl.K = K;
    pl.backend = backend;
    pl.S = S;
    pl.w = w;
    pl.Q = w * S;
    pl.nmod = N;
    pl.g0 = std::max(0, S - 1 - extra);
    pl.ng = 2 * S - 1 - pl.g0;
    pl.need = need;
    pl.mods.assign(mods.begin(), mods.begin() + N);
    pl.nwx = (pl.Q + 2 + 31) / 32;
    pl.nh = (w + 2 + 15) / 16;
    const int sbits = 2 * w + (int)std::ceil(std::log2((double)K * S)) + 2;
    pl.nwc = (sbits + w * (pl.ng - 1) + 1 + 31) / 32;
    {
      // 16-bit digits of sum_l t_l M_l < nmod P (one sign bit to spare)
      double lp = 0.0;
      for (int i = 0; i < N; ++i) lp += std::log2((double)mods[i]);
      const int bits = (int)std::ceil(lp + std::log2((double)N)) + 2;
      pl.nd = ((bits + 15) / 16 + 1) & ~1;
    }
    if (check_sizes && (pl.nwx > 12 || pl.nh > ozk::NHMAX || pl.nwc > 16 || w > 300 ||
                        pl.nd > (backend == OZII_BE_F64MOD ? 32 : 24))) {
      if (why) *why = "plan exceeds the compiled word sizes";
      return OZII_EUNSUPPORTED;
    }
    return OZII_OK;
  }
  if (why) *why = any_acc ? "need exceeds the CRT capacity of the modulus set" : "accumulator bound";
  return any_acc ? OZII_ECAPACITY : OZII_EOVERFLOW;
}

// ---------------------------------------------------------------------------
// Small unsigned big integers (little-endian 32-bit limbs) for the CRT
// constants P and M_l.
// ---------------------------------------------------------------------------
typedef std::vector<uint32_t> Big;
void big_mul_small(Big &a, uint32_t m) {
  uint64_t carry = 0;
  for (auto &x : a) {
    uint64_t t = (uint64_t)x * m + carry;
    x = (uint32_t)t;
    carry = t >> 32;
  }
  if (carry) a.push_back((uint32_t)carry);
}
uint32_t big_mod_small(const Big &a, uint32_t m) {
  uint64_t r = 0;
  for (size_t i = a.size(); i-- > 0;) r = ((r << 32) | a[i]) % m;
  return (uint32_t)r;
}
uint16_t big_digit16(const Big &a, int k) {
  size_t wi = (size_t)k / 2;
  if (wi >= a.size()) return 0;
  return (uint16_t)(a[wi] >> (16 * (k & 1)));
}

void build_devplan(const HostPlan &hp, DevPlan &dp) {
  std::memset(&dp, 0, sizeof(dp));
  dp.S = hp.S;
  dp.w = hp.w;
  dp.Q = hp.Q;
  dp.nmod = hp.nmod;
  dp.g0 = hp.g0;
  dp.ng = hp.ng;
  dp.nwx = hp.nwx;
  dp.nh = hp.nh;
  Big P{1};
  for (int m : hp.mods) big_mul_small(P, (uint32_t)m);
  for (int l = 0; l < hp.nmod; ++l) {
    const uint32_t m = (uint32_t)hp.mods[l];
    dp.m[l] = (int32_t)m;
    dp.inv_m[l] = 1.0 / (double)m;
    Big Ml{1};
    for (int k = 0; k < hp.nmod; ++k)
      if (k != l) big_mul_small(Ml, (uint32_t)hp.mods[k]);
    // y_l = M_l^{-1} mod m_l by the extended Euclidean algorithm
    int64_t r0 = (int64_t)m, r1 = (int64_t)big_mod_small(Ml, m), s0 = 0, s1 = 1;
    while (r1 != 0) {
      const int64_t qq = r0 / r1, r2 = r0 - qq * r1, s2 = s0 - qq * s1;
      r0 = r1;
      r1 = r2;
      s0 = s1;
      s1 = s2;
    }
    dp.y[l] = (int32_t)(((s0 % (int64_t)m) + (int64_t)m) % (int64_t)m);
    for (int k = 0; k < ozk::NDCRT; ++k) dp.Mdig[l][k] = big_digit16(Ml, k);
    uint64_t pw = 1 % m;
    for (int k = 0; k < ozk::NHMAX; ++k) {
      dp.pw16[l][k] = (uint32_t)pw;
      pw = (pw << 16) % m;
    }
    uint64_t p2 = 1 % m;
    for (int b = 0; b < hp.w; ++b) p2 = (p2 * 2) % m;
    dp.p2w[l] = (uint32_t)p2;
  }
  for (int k = 0; k < ozk::NDCRT; ++k) dp.Pdig[k] = big_digit16(P, k);
  dp.nd = ozk::NDCRT;
  // records of the byte back-ends (see DevPlan::rec)
  dp.nwt = (hp.w + 2 + 31) / 32;
  if (hp.backend != OZII_BE_F64MOD) {
    for (int l = 0; l < hp.nmod; ++l) {
      const uint64_t m = (uint64_t)hp.mods[l];
      uint32_t *r = dp.rec[l];
      uint64_t pw = 1 % m;
      for (int j = 0; j < ozk::REC_PWMAX; ++j) {
        uint32_t word = 0;
        for (int i = 0; i < 4; ++i) {
          if (j < dp.nwt) word |= (uint32_t)pw << (8 * i);
          pw = (pw << 8) % m;
        }
        r[j] = word;
      }
      uint64_t p2w = 1 % m, p2t = 1 % m;
      for (int b = 0; b < hp.w; ++b) p2w = (p2w * 2) % m;
      for (int b = 0; b < 32 * dp.nwt; ++b) p2t = (p2t * 2) % m;
      const uint32_t h = (uint32_t)(m / 2);
      r[ozk::REC_H] = h;
      r[ozk::REC_HW] = h + (uint32_t)((m - p2w) % m);
      r[ozk::REC_HT] = h + (uint32_t)((m - p2t) % m);
      int k = 1;
      while (((1ull << (32 - k)) + m - 1) / m >= (1ull << 24)) ++k;
      r[ozk::REC_MAGIC] = (uint32_t)(((1ull << (32 - k)) + m - 1) / m);
      r[ozk::REC_M] = (uint32_t)m;
      r[ozk::REC_K] = (uint32_t)k;
    }
    for (int l = 0; l < hp.nmod; ++l) {
      const uint32_t m = (uint32_t)hp.mods[l];
      Big Ml{1};
      for (int k = 0; k < hp.nmod; ++k)
        if (k != l) big_mul_small(Ml, (uint32_t)hp.mods[k]);
      uint32_t *c4 = dp.crt4[l / 4];
      const int sh = 8 * (l % 4);
      for (int b = 0; b < ozk::CRT4_NB; ++b)
        c4[b] |= ((big_digit16(Ml, b / 2) >> (8 * (b % 2))) & 0xffu) << sh;
      const uint32_t f = (65536u + m / 2) / m;
      c4[ozk::CRT4_NB] |= (f & 0xffu) << sh;
      c4[ozk::CRT4_NB + 1] |= (f >> 8) << sh;
    }
    for (int b = 0; b < ozk::CRT4_NB; ++b)
      dp.pbyte[b] = (int32_t)((big_digit16(P, b / 2) >> (8 * (b % 2))) & 0xffu);
    // the matrix-core form of the same table (DevPlan::crtm, crtc): f_l and
    // M_l in balanced bytes; M_l < P < 2^363 (at most 54 moduli <= 256)
    // leaves bytes 46 and 47 zero
    for (int l = 0; l < hp.nmod; ++l) {
      const uint32_t m = (uint32_t)hp.mods[l];
      Big Ml{1};
      for (int k = 0; k < hp.nmod; ++k)
        if (k != l) big_mul_small(Ml, (uint32_t)hp.mods[k]);
      int32_t col[64] = {0};
      const int32_t f = (int32_t)((65536u + m / 2) / m), fh = (f + 128) >> 8;
      col[0] = f - 256 * fh;
      col[1] = fh;
      int32_t carry = 0;
      for (int b = 0; b < ozk::CRT4_NB; ++b) {
        int32_t v = (int32_t)((big_digit16(Ml, b / 2) >> (8 * (b % 2))) & 0xffu) + carry;
        carry = v >= 128 ? 1 : 0;
        col[2 + b] = v - 256 * carry;
      }
      // columns 48, 49 (bytes 46, 47) are 0 for every M_l < 2^363
      for (int j = 0; j < 48; ++j) {
        dp.crtm[j / 16][16 * (l / 16) + j % 16][l % 16] = (int8_t)col[j];
        dp.crtc[j] += 128 * col[j];
      }
    }
  }
}

int64_t roundup(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

}  // namespace

// ---------------------------------------------------------------------------
// handle
// ---------------------------------------------------------------------------
struct ozII_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string last_error;
  // Ozaki workspace
  char *ws = nullptr;
  size_t ws_bytes = 0;
  // panel scratch
  uint32_t *bar = nullptr;
  uint32_t *flags = nullptr;  // panel candidate lines, two 128-byte lines per workgroup
  int *err = nullptr;
  double *crow = nullptr;
  int *perm = nullptr, *moved = nullptr, *nmoved = nullptr;
  int64_t panel_n = 0;
  int panel_kb = 0;
  // limb LU: pivot candidates of one panel column and the zero-pivot word
  int64_t *lcand = nullptr;
  int32_t *lflag = nullptr;
  // getrf look-ahead: a side stream (default priority) for the rest of each
  // Schur update while the next panel runs, and the fork / join events
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // batched LU: the uploaded item table (processing order) and its queue
  ozII_batch_item *batch = nullptr;
  int batch_cap = 0, batch_count = 0, batch_grid = 1;
  int *batch_queue = nullptr;
  // batched LU with the Ozaki-II update: panel width (0: native unblocked
  // path), plans per nc = 2, 3, 4 and the per-workgroup scratch
  int batch_b = 0;
  const DevPlan *batch_pl[3] = {nullptr, nullptr, nullptr};
  uint8_t *batch_ws = nullptr;
  size_t batch_ws_bytes = 0;
  int64_t batch_slot = 0;
  std::map<std::tuple<int, int64_t, int, int, int, int>, std::pair<HostPlan, DevPlan *>> plans;
  // per-stage profiling (HIP events on the handle's stream)
  struct ProfRec {
    int stage;
    hipEvent_t a, b;
    double bytes, ops;
  };
  bool profiling = false;
  int prof_block = 0;  // > 0 inside ozII_gemm_noalloc: no events are created
  std::vector<ProfRec> prof;
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;
};

namespace {

ozII_status fail(ozII_ctx *h, ozII_status s, const std::string &msg) {
  if (h) h->last_error = msg;
  return s;
}

ozII_status hip_fail(ozII_ctx *h, hipError_t e, const char *where) {
  return fail(h, OZII_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

hipEvent_t prof_event(ozII_ctx *h) {
  if (h->pool_used == h->pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->pool.push_back(e);
  }
  return h->pool[h->pool_used++];
}

// Bracket one launch with events when profiling is on.
// Bracket one launch with events when profiling is on, on the stream the
// launch goes to (the handle's stream unless given).
struct ProfScope {
  ozII_ctx *h;
  hipStream_t s;
  int idx = -1;
  ProfScope(ozII_ctx *hh, int stage, double bytes, double ops) : ProfScope(hh, stage, bytes, ops, hh->stream) {}
  ProfScope(ozII_ctx *hh, int stage, double bytes, double ops, hipStream_t st) : h(hh), s(st) {
    if (!h->profiling || h->prof_block) return;
    hipEvent_t a = prof_event(h), b = prof_event(h);
    if (!a || !b) return;
    hipEventRecord(a, s);
    h->prof.push_back({stage, a, b, bytes, ops});
    idx = (int)h->prof.size() - 1;
  }
  ~ProfScope() {
    if (idx >= 0) hipEventRecord(h->prof[idx].b, s);
  }
};

// limbs: plans for the limb format, whose fixed point and group sums live in
// memory rather than registers; only the slice window (w <= 300) and the
// byte CRT (at most 24 16-bit digits) bound them.
ozII_status get_plan(ozII_ctx *h, int p, int64_t K, const ozII_opts *o, const HostPlan **hp,
                     const DevPlan **dp, bool limbs = false) {
  const int backend = (o && o->backend) ? o->backend : OZII_BE_INT8;
  auto key = std::make_tuple(p, K, backend, o ? o->nslice : 0, o ? o->extra_groups : 0,
                             ((o ? o->guard_ex : 0) * 2 + (limbs ? 1 : 0)) * 4096 + (o ? o->qbits : 0));
  auto it = h->plans.find(key);
  if (it == h->plans.end()) {
    HostPlan pl;
    std::string why;
    ozII_status st = make_plan(p, K, o, pl, &why, !limbs);
    if (st != OZII_OK) return fail(h, st, "plan: " + why);
    if (limbs && (pl.w > 300 || pl.nd > (pl.backend == OZII_BE_F64MOD ? ozk::NDCRT : 24)))
      return fail(h, OZII_EUNSUPPORTED, "plan: limb plan exceeds the compiled sizes");
    DevPlan host_dp;
    build_devplan(pl, host_dp);
    DevPlan *d = nullptr;
    hipError_t e = hipMalloc((void **)&d, sizeof(DevPlan));
    if (e != hipSuccess) return hip_fail(h, e, "hipMalloc(plan)");
    e = hipMemcpy(d, &host_dp, sizeof(DevPlan), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(h, e, "hipMemcpy(plan)");
    it = h->plans.emplace(key, std::make_pair(pl, d)).first;
  }
  *hp = &it->second.first;
  *dp = it->second.second;
  return OZII_OK;
}

// ---------------------------------------------------------------------------
// Static scratch of ozII_gemm_noalloc, for callers that cannot allocate
// device memory.  Each GPU the library runs on holds its own copy of the
// array until the process ends.  Host code never passes the array's name to
// a kernel or a copy: ozII_create maps it once per device with
// hipGetSymbolAddress (device current) and every use goes through that
// per-device address.  Layout: NOALLOC_SLOTS plan tables of
// NOALLOC_SLOT_BYTES each, then the workspace of one product.
// ---------------------------------------------------------------------------
constexpr size_t NOALLOC_BYTES = (size_t)64 << 20;
constexpr int NOALLOC_SLOTS = 8;
constexpr size_t NOALLOC_SLOT_BYTES = 32 << 10;
constexpr size_t NOALLOC_WS_OFF = NOALLOC_SLOTS * NOALLOC_SLOT_BYTES;
static_assert(sizeof(DevPlan) <= NOALLOC_SLOT_BYTES, "plan slot too small");

static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

struct NoallocDev {
  char *base = nullptr;         // device address of `scratch` on this device
  hipError_t map_err = hipSuccess;
  bool used[NOALLOC_SLOTS] = {};
  std::tuple<int, int64_t, int, int, int, int> key[NOALLOC_SLOTS];
  HostPlan host_plan[NOALLOC_SLOTS];
  DevPlan host_dev[NOALLOC_SLOTS];  // the uploaded tables (source of the copies)
  int next = 0;
};
std::mutex g_noalloc_mu;
std::map<int, NoallocDev> g_noalloc;

// Map the static scratch on the current device (once per device).
void noalloc_map(int device) {
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  NoallocDev &nd = g_noalloc[device];
  if (nd.base || nd.map_err != hipSuccess) return;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    nd.map_err = e != hipSuccess ? e : hipErrorInvalidSymbol;
    return;
  }
  nd.base = (char *)ptr;
}

// The plan of (p, K, o) in one of the device's scratch slots: the tables are
// built on the host and copied into a slot on the handle's stream the first
// time a plan is used (or after it was evicted by NOALLOC_SLOTS others).
ozII_status noalloc_plan(ozII_ctx *h, int p, int64_t K, const ozII_opts *o, const HostPlan **hp,
                         const DevPlan **dp, char **ws) {
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  auto it = g_noalloc.find(h->device);
  if (it == g_noalloc.end() || !it->second.base)
    return fail(h, OZII_EHIP, std::string("static scratch not mapped: ") +
                                  hipGetErrorString(it == g_noalloc.end() ? hipErrorInvalidSymbol
                                                                          : it->second.map_err));
  NoallocDev &nd = it->second;
  const int backend = (o && o->backend) ? o->backend : OZII_BE_INT8;
  const auto key = std::make_tuple(p, K, backend, o ? o->nslice : 0, o ? o->extra_groups : 0,
                                   (o ? o->guard_ex : 0) * 2 * 4096 + (o ? o->qbits : 0));
  *ws = nd.base + NOALLOC_WS_OFF;
  for (int sl = 0; sl < NOALLOC_SLOTS; ++sl)
    if (nd.used[sl] && nd.key[sl] == key) {
      *hp = &nd.host_plan[sl];
      *dp = (const DevPlan *)(nd.base + sl * NOALLOC_SLOT_BYTES);
      return OZII_OK;
    }
  HostPlan pl;
  std::string why;
  const ozII_status st = make_plan(p, K, o, pl, &why, true);
  if (st != OZII_OK) return fail(h, st, "plan: " + why);
  const int sl = nd.next;
  nd.next = (nd.next + 1) % NOALLOC_SLOTS;
  nd.used[sl] = false;
  nd.host_plan[sl] = pl;
  build_devplan(pl, nd.host_dev[sl]);
  char *dst = nd.base + sl * NOALLOC_SLOT_BYTES;
  const hipError_t e = hipMemcpyAsync(dst, &nd.host_dev[sl], sizeof(DevPlan),
                                      hipMemcpyHostToDevice, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "plan upload");
  nd.used[sl] = true;
  nd.key[sl] = key;
  *hp = &nd.host_plan[sl];
  *dp = (const DevPlan *)dst;
  return OZII_OK;
}

struct GemmLayout {
  int64_t Mp, Np, Kp, planeA, planeB, tplBytes;
  size_t off_ea, off_eb, off_pa, off_pb, off_tpl, total;
};

GemmLayout gemm_layout(const HostPlan &hp, int64_t M, int64_t N, int64_t K, int tile) {
  GemmLayout L;
  // rows and columns padded to the 256-wide tiles of the large GEMM kernels
  // once they exceed one 128-wide tile (or when such a tile is forced)
  L.Mp = roundup(std::max<int64_t>(M, 1), (M > 128 || tile >= ozl::GEMM_TILE_256x128) ? 256 : 128);
  L.Np = roundup(std::max<int64_t>(N, 1), (N > 128 || tile == ozl::GEMM_TILE_256x256) ? 256 : 128);
  L.Kp = roundup(std::max<int64_t>(K, 1), hp.k_align());
  L.planeA = L.Mp * L.Kp;  // elements per plane
  L.planeB = L.Np * L.Kp;
  L.tplBytes = (int64_t)hp.ng * hp.nmod * L.Mp * L.Np * hp.t_bytes();
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o += (bytes + 255) / 256 * 256;
    return r;
  };
  L.off_ea = take(sizeof(int32_t) * L.Mp);
  L.off_eb = take(sizeof(int32_t) * L.Np);
  L.off_pa = take((size_t)hp.S * hp.nmod * hp.planes_per() * L.planeA * hp.el_bytes());
  L.off_pb = take((size_t)hp.S * hp.nmod * hp.planes_per() * L.planeB * hp.el_bytes());
  L.off_tpl = take((size_t)L.tplBytes);
  L.total = o;
  return L;
}

ozII_status ensure_ws(ozII_ctx *h, size_t bytes) {
  if (bytes <= h->ws_bytes) return OZII_OK;
  if (h->ws) {
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamSynchronize");
    hipFree(h->ws);
    h->ws = nullptr;
    h->ws_bytes = 0;
  }
  hipError_t e = hipMalloc((void **)&h->ws, bytes);
  if (e != hipSuccess) {
    h->ws = nullptr;
    return fail(h, OZII_ENOMEM, "workspace allocation failed");
  }
  h->ws_bytes = bytes;
  return OZII_OK;
}

ozII_status ensure_panel(ozII_ctx *h, int64_t n, int kb) {
  if (n <= h->panel_n && kb <= h->panel_kb) return OZII_OK;
  if (h->bar) {
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamSynchronize");
    hipFree(h->crow);
    hipFree(h->perm);
    hipFree(h->moved);
  }
  const int64_t nn = std::max<int64_t>(n, h->panel_n);
  const int kk = std::max(kb, h->panel_kb);
  const int G = 256;
  hipError_t e = hipSuccess;
  if (!h->bar) {
    e = hipMalloc((void **)&h->bar, 64);
    if (e == hipSuccess) e = hipMemset(h->bar, 0, 64);
    if (e == hipSuccess) {
      h->err = (int *)(h->bar + 4);
      h->nmoved = (int *)(h->bar + 8);
    }
  }
  if (e == hipSuccess && !h->flags) e = hipMalloc((void **)&h->flags, 2 * 128 * G);
  if (e == hipSuccess) e = hipMalloc((void **)&h->crow, sizeof(double) * 2 * G * kk * 4);
  if (e == hipSuccess) e = hipMalloc((void **)&h->perm, sizeof(int) * nn);
  if (e == hipSuccess) e = hipMalloc((void **)&h->moved, sizeof(int) * nn);
  if (e != hipSuccess) return fail(h, OZII_ENOMEM, "panel scratch allocation failed");
  h->panel_n = nn;
  h->panel_kb = kk;
  return OZII_OK;
}

bool valid_nc(int nc) { return nc >= 2 && nc <= 4; }

ozII_status gemm_impl(ozII_ctx *h, int mode, int nc, int64_t M, int64_t N, int64_t K,
                      const double *A, int64_t lda, const double *B, int64_t ldb, double *C,
                      int64_t ldc, const ozII_opts *o, int32_t *ea_out, int32_t *eb_out,
                      void *pa_out, void *pb_out, void *tpl_out, uint64_t *sbar_out,
                      int nlimb, bool noalloc = false, hipStream_t stream = nullptr,
                      char *ws_given = nullptr, size_t ws_cap = 0) {
  if (!h) return OZII_EINVAL;
  hipStream_t s = ws_given ? stream : h->stream;
  if (!valid_nc(nc)) return fail(h, OZII_EUNSUPPORTED, "nc must be 2, 3 or 4");
  if (mode != 0 && mode != 1) return fail(h, OZII_EINVAL, "mode must be 0 or 1");
  if (M < 0 || N < 0 || K < 0) return fail(h, OZII_EINVAL, "negative size");
  if (M == 0 || N == 0) return OZII_OK;
  if (lda < std::max<int64_t>(M, 1) || ldb < std::max<int64_t>(K, 1) || ldc < M)
    return fail(h, OZII_EINVAL, "leading dimension too small");
  if (!C || (K > 0 && (!A || !B))) return fail(h, OZII_EINVAL, "null matrix pointer");
  if (K == 0) {
    if (mode == 1) return OZII_OK;
    // C = 0 (a fill kernel: stays correct inside a captured graph)
    hipError_t e = ozl::launch_zero_expansions(nc, C, ldc, M, N, s);
    return e == hipSuccess ? OZII_OK : hip_fail(h, e, "zero C");
  }
  const HostPlan *hp;
  const DevPlan *dp;
  char *ws = nullptr;
  ozII_status st;
  if (noalloc) {
    st = noalloc_plan(h, 53 * nc, K, o, &hp, &dp, &ws);
    if (st != OZII_OK) return st;
  } else {
    st = get_plan(h, 53 * nc, K, o, &hp, &dp);
    if (st != OZII_OK) return st;
  }
  GemmLayout L = gemm_layout(*hp, M, N, K, o ? o->gemm_tile : 0);
  if (noalloc) {
    if (L.total > NOALLOC_BYTES - NOALLOC_WS_OFF)
      return fail(h, OZII_EINVAL,
                  "ozII_gemm_noalloc: the product needs " + std::to_string(L.total) +
                      " bytes of workspace, the static scratch holds " +
                      std::to_string(NOALLOC_BYTES - NOALLOC_WS_OFF));
  } else if (ws_given) {
    if (L.total > ws_cap) return fail(h, OZII_EINVAL, "internal: workspace region too small");
    ws = ws_given;
  } else {
    st = ensure_ws(h, L.total);
    if (st != OZII_OK) return st;
    ws = h->ws;
  }
  int32_t *ea = (int32_t *)(ws + L.off_ea);
  int32_t *eb = (int32_t *)(ws + L.off_eb);
  void *pa = ws + L.off_pa;
  void *pb = ws + L.off_pb;
  void *tpl = ws + L.off_tpl;
  hipError_t e;
  const double pairs = (double)hp->nmod * [&] {
    int np = 0;
    for (int g = hp->g0; g <= 2 * hp->S - 2; ++g)
      for (int ta = 0; ta < hp->S; ++ta)
        if (g - ta >= 0 && g - ta < hp->S) ++np;
    return np;
  }();
  // algorithmic bytes of the residue planes and t-planes of this back-end
  const double res_bytes = (double)hp->S * hp->nmod * hp->planes_per() * hp->el_bytes();
  const double t_bytes = (double)hp->ng * hp->nmod * hp->t_bytes();
  {
    ProfScope ps(h, OZ_STAGE_EXP, 8.0 * nc * (double)(M * K + K * N), 0, s);
    if ((e = ozl::launch_exponents(nc, A, lda, M, K, 1, ea, s)) != hipSuccess) return hip_fail(h, e, "exponents(A)");
    if ((e = ozl::launch_exponents(nc, B, ldb, K, N, 0, eb, s)) != hipSuccess) return hip_fail(h, e, "exponents(B)");
  }
  {
    ProfScope ps(h, OZ_STAGE_PRODUCER, (double)M * K * (8.0 * nc + res_bytes), 0, s);
    if ((e = ozl::launch_producer(nc, hp->nwx, hp->nh, (hp->w + 2 + 31) / 32, A, lda, 1, M, L.Mp, K, L.Kp, ea, dp,
                                  hp->nmod, hp->planes_kind(), pa, L.planeA, s)) != hipSuccess)
      return hip_fail(h, e, "producer(A)");
  }
  {
    ProfScope ps(h, OZ_STAGE_PRODUCER, (double)N * K * (8.0 * nc + res_bytes), 0, s);
    if ((e = ozl::launch_producer(nc, hp->nwx, hp->nh, (hp->w + 2 + 31) / 32, B, ldb, 0, N, L.Np, K, L.Kp, eb, dp,
                                  hp->nmod, hp->planes_kind(), pb, L.planeB, s)) != hipSuccess)
      return hip_fail(h, e, "producer(B)");
  }
  // (S4)-(S6) fused: the t-values of a tile stay in LDS (INT8, no stage copies)
  if (o && (o->flags & OZII_F_FUSED) && hp->backend == OZII_BE_INT8 && !ea_out && !eb_out &&
      !pa_out && !pb_out && !tpl_out && !sbar_out && hp->ng * hp->nmod <= ozl::fused_max_products() &&
      hp->nd <= 24) {
    ProfScope ps(h, OZ_STAGE_FUSED, res_bytes * (double)(M + N) * K + 8.0 * nc * (mode ? 2 : 1) * M * N,
                 2.0 * (double)M * N * K * pairs, s);
    if ((e = ozl::launch_fused_b(nc, hp->nwc, hp->nd, (const int8_t *)pa, (const int8_t *)pb, dp,
                                 hp->ng, hp->nmod, L.Kp, L.planeA, L.planeB, C, ldc, M, N, ea, eb,
                                 mode, s)) != hipSuccess)
      return hip_fail(h, e, "fused product");
    return OZII_OK;
  }
  {
    // issued operations: the FP8 back-end runs four sub-products per pair
    const double ops = 2.0 * (double)M * N * K * pairs * (hp->backend == OZII_BE_FP8_B17 ? 4.0 : 1.0);
    ProfScope ps(h, OZ_STAGE_GEMM, res_bytes * (double)(M + N) * K + t_bytes * M * N, ops, s);
    if (hp->backend == OZII_BE_FP8_B17)
      e = ozl::launch_gemm_f8((const uint8_t *)pa, (const uint8_t *)pb, (uint8_t *)tpl, dp, hp->ng,
                              hp->nmod, L.Mp, L.Np, L.Kp, L.planeA, L.planeB, s);
    else if (hp->backend == OZII_BE_F64MOD)
      e = ozl::launch_gemm_f64((const double *)pa, (const double *)pb, (uint32_t *)tpl, dp, hp->ng,
                               hp->nmod, L.Mp, L.Np, L.Kp, L.planeA, L.planeB, s);
    else if (hp->backend == OZII_BE_FP16)
      e = ozl::launch_gemm_f16((const int8_t *)pa, (const int8_t *)pb, (uint8_t *)tpl, dp, hp->ng,
                               hp->nmod, L.Mp, L.Np, L.Kp, L.planeA, L.planeB, s);
    else
      e = ozl::launch_gemm_i8((const int8_t *)pa, (const int8_t *)pb, (uint8_t *)tpl, dp, hp->ng,
                              hp->nmod, L.Mp, L.Np, L.Kp, L.planeA, L.planeB,
                              o ? o->gemm_tile : 0, s);
    if (e != hipSuccess) return hip_fail(h, e, "modular gemm");
  }
  const size_t pl_bytes_a = (size_t)hp->S * hp->nmod * hp->planes_per() * L.planeA * hp->el_bytes();
  const size_t pl_bytes_b = (size_t)hp->S * hp->nmod * hp->planes_per() * L.planeB * hp->el_bytes();
  if (ea_out && (e = hipMemcpyAsync(ea_out, ea, 4 * M, hipMemcpyDeviceToDevice, s)) != hipSuccess) return hip_fail(h, e, "copy ea");
  if (eb_out && (e = hipMemcpyAsync(eb_out, eb, 4 * N, hipMemcpyDeviceToDevice, s)) != hipSuccess) return hip_fail(h, e, "copy eb");
  if (pa_out && (e = hipMemcpyAsync(pa_out, pa, pl_bytes_a, hipMemcpyDeviceToDevice, s)) != hipSuccess)
    return hip_fail(h, e, "copy planesA");
  if (pb_out && (e = hipMemcpyAsync(pb_out, pb, pl_bytes_b, hipMemcpyDeviceToDevice, s)) != hipSuccess)
    return hip_fail(h, e, "copy planesB");
  if (tpl_out && (e = hipMemcpyAsync(tpl_out, tpl, (size_t)L.tplBytes, hipMemcpyDeviceToDevice, s)) != hipSuccess)
    return hip_fail(h, e, "copy tpl");
  if (sbar_out && (e = ozl::launch_crt_export(tpl, hp->t_bytes(), hp->nd, L.Mp, L.Np, M, N, dp, sbar_out, nlimb, 1, s)) != hipSuccess)
    return hip_fail(h, e, "crt_export");
  {
    ProfScope ps(h, OZ_STAGE_CONSUMER, (double)M * N * (t_bytes + 8.0 * nc * (mode ? 2 : 1)), 0, s);
    if ((e = ozl::launch_consumer(nc, hp->nwc, hp->nd, tpl, hp->t_bytes(), L.Mp, L.Np, C, ldc, M, N,
                                  ea, eb, dp, mode, s)) != hipSuccess)
      return hip_fail(h, e, "consumer");
  }
  return OZII_OK;
}

// Words of the exact group-sum column kept per element by the limb consumer
// (the same walk as the kernel's), and the words per shifted group sum.
void limb_words(const HostPlan &hp, int *nvw, int *nwords) {
  const int sbits = 2 * hp.w + (int)std::ceil(std::log2((double)hp.K * hp.S)) + 2;
  *nvw = (sbits + 31) / 32 + 1;
  int hw = 0;
  for (int gi = 0; gi < hp.ng; ++gi) {
    const int q0 = (hp.w * gi) >> 5;
    if (q0 > hw) hw = q0;
    hw = std::max(q0 + *nvw, hw + 1);
  }
  *nwords = hw + 1;
}

bool limbs_ok(const ozII_limbs *X, int64_t rows, int64_t cols) {
  if (!X || !X->limb || !X->exp || !X->sign) return false;
  if (X->ld < std::max<int64_t>(rows, 1)) return false;
  return X->plane >= X->ld * cols;
}

ozII_status gemm_limbs_impl(ozII_ctx *h, int mode, int nlimb, int64_t M, int64_t N, int64_t K,
                            const ozII_limbs *A, const ozII_limbs *B, ozII_limbs *C,
                            const ozII_opts *o, uint64_t *sbar_out = nullptr,
                            int nlimb_out = 0) {
  if (!h) return OZII_EINVAL;
  if (mode != 0 && mode != 1) return fail(h, OZII_EINVAL, "mode must be 0 or 1");
  if (nlimb < 1 || nlimb > OZII_GEMM_LIMBS_MAX)
    return fail(h, OZII_EINVAL, "nlimb must be 1..OZII_GEMM_LIMBS_MAX");
  if (M < 0 || N < 0 || K < 0) return fail(h, OZII_EINVAL, "negative size");
  if (o && o->backend && o->backend != OZII_BE_INT8 && o->backend != OZII_BE_F64MOD)
    return fail(h, OZII_EUNSUPPORTED, "the limb product runs on the INT8 or binary64 back-end");
  if (M == 0 || N == 0) return OZII_OK;
  if (!limbs_ok(C, M, N) || (K > 0 && (!limbs_ok(A, M, K) || !limbs_ok(B, K, N))))
    return fail(h, OZII_EINVAL, "bad limb matrix descriptor");
  hipStream_t s = h->stream;
  hipError_t e;
  if (K == 0) {
    if (mode == 1) return OZII_OK;
    e = ozl::launch_limb_zero(C->limb, C->exp, C->sign, C->ld, C->plane, nlimb, M, N, s);
    return e == hipSuccess ? OZII_OK : hip_fail(h, e, "limb zero");
  }
  const int p = 64 * nlimb;
  const HostPlan *hp;
  const DevPlan *dp;
  ozII_status st = get_plan(h, p, K, o, &hp, &dp, true);
  if (st != OZII_OK) return st;
  int nvw = 0, nwords = 0;
  limb_words(*hp, &nvw, &nwords);
  if (nvw > hp->nd / 2 + 1) return fail(h, OZII_EUNSUPPORTED, "group sum wider than its digits");
  GemmLayout L = gemm_layout(*hp, M, N, K, o ? o->gemm_tile : 0);
  // after the planes and t-planes: the group-sum columns (reused as the
  // update's scratch), then the rounded product of mode 1
  const int64_t MN = M * N;
  const size_t cw_words = (size_t)std::max(nwords, 2 * nlimb + 2);
  const size_t off_cw = (L.total + 255) / 256 * 256;
  const size_t off_tl = off_cw + (cw_words * MN * 4 + 255) / 256 * 256;
  const size_t off_te = off_tl + ((size_t)nlimb * MN * 8 + 255) / 256 * 256;
  const size_t off_ts = off_te + ((size_t)MN * 4 + 255) / 256 * 256;
  const size_t total = off_ts + ((size_t)MN + 255) / 256 * 256;
  st = ensure_ws(h, mode ? total : off_tl);
  if (st != OZII_OK) return st;
  int32_t *ea = (int32_t *)(h->ws + L.off_ea);
  int32_t *eb = (int32_t *)(h->ws + L.off_eb);
  uint8_t *pa = (uint8_t *)(h->ws + L.off_pa);
  uint8_t *pb = (uint8_t *)(h->ws + L.off_pb);
  uint8_t *tpl = (uint8_t *)(h->ws + L.off_tpl);
  uint32_t *cw = (uint32_t *)(h->ws + off_cw);
  const int nwt = (hp->w + 2 + 31) / 32;
  const bool f64 = hp->backend == OZII_BE_F64MOD;
  const double pairs = (double)hp->nmod * [&] {
    int np = 0;
    for (int g = hp->g0; g <= 2 * hp->S - 2; ++g)
      for (int ta = 0; ta < hp->S; ++ta)
        if (g - ta >= 0 && g - ta < hp->S) ++np;
    return np;
  }();
  const double in_bytes = 8.0 * nlimb + 5.0;  // limbs, exponent and sign per element
  const double res_bytes = (double)hp->S * hp->nmod * hp->el_bytes(),
               t_bytes = (double)hp->ng * hp->nmod * hp->t_bytes();
  {
    ProfScope ps(h, OZ_STAGE_EXP, 12.0 * (double)(M * K + K * N), 0);
    if ((e = ozl::launch_limb_exponents(A->limb, A->exp, A->ld, A->plane, nlimb, M, K, 1, ea, s)) != hipSuccess)
      return hip_fail(h, e, "limb exponents(A)");
    if ((e = ozl::launch_limb_exponents(B->limb, B->exp, B->ld, B->plane, nlimb, K, N, 0, eb, s)) != hipSuccess)
      return hip_fail(h, e, "limb exponents(B)");
  }
  {
    ProfScope ps(h, OZ_STAGE_PRODUCER, (double)M * K * (in_bytes + res_bytes), 0);
    if ((e = ozl::launch_producer_limbs(A->limb, A->exp, A->sign, A->ld, A->plane, nlimb, 1, M,
                                        L.Mp, K, L.Kp, ea, dp, hp->nmod, nwt, hp->planes_kind(), pa,
                                        L.planeA, s)) != hipSuccess)
      return hip_fail(h, e, "limb producer(A)");
  }
  {
    ProfScope ps(h, OZ_STAGE_PRODUCER, (double)N * K * (in_bytes + res_bytes), 0);
    if ((e = ozl::launch_producer_limbs(B->limb, B->exp, B->sign, B->ld, B->plane, nlimb, 0, N,
                                        L.Np, K, L.Kp, eb, dp, hp->nmod, nwt, hp->planes_kind(), pb,
                                        L.planeB, s)) != hipSuccess)
      return hip_fail(h, e, "limb producer(B)");
  }
  {
    ProfScope ps(h, OZ_STAGE_GEMM, res_bytes * (double)(M + N) * K + t_bytes * M * N,
                 2.0 * (double)M * N * K * pairs);
    if (f64)
      e = ozl::launch_gemm_f64((const double *)pa, (const double *)pb, (uint32_t *)tpl, dp, hp->ng,
                               hp->nmod, L.Mp, L.Np, L.Kp, L.planeA, L.planeB, s);
    else
      e = ozl::launch_gemm_i8((const int8_t *)pa, (const int8_t *)pb, tpl, dp, hp->ng, hp->nmod,
                              L.Mp, L.Np, L.Kp, L.planeA, L.planeB, o ? o->gemm_tile : 0, s);
    if (e != hipSuccess) return hip_fail(h, e, "modular gemm");
  }
  if (sbar_out && (e = ozl::launch_crt_export(tpl, hp->t_bytes(), hp->nd, L.Mp, L.Np, M, N, dp,
                                              sbar_out, nlimb_out, 0, s)) != hipSuccess)
    return hip_fail(h, e, "crt_export");
  {
    // t-planes read once, each group's window of the sum read and written
    ProfScope ps(h, OZ_STAGE_CONSUMER,
                 (double)M * N * (t_bytes + 8.0 * nvw * hp->ng), 0);
    if ((e = ozl::launch_consumer_limbs(tpl, hp->t_bytes(), L.Mp, L.Np, M, N, dp, hp->nd, nvw, cw,
                                        s)) != hipSuccess)
      return hip_fail(h, e, "limb consumer");
  }
  // rounding: the group-sum column read, the p-bit product written (to C, or
  // to the temporary product of mode 1); update: C and the product read, the
  // difference written and read back, C written
  if (mode == 0) {
    ProfScope ps(h, OZ_STAGE_ROUND, (double)M * N * (4.0 * nwords + in_bytes), 0);
    if ((e = ozl::launch_limb_round(cw, nwords, M, N, ea, eb, hp->w, hp->g0, hp->Q, nlimb, C->limb,
                                    C->exp, C->sign, C->ld, C->plane, s)) != hipSuccess)
      return hip_fail(h, e, "limb round");
  } else {
    uint64_t *tl = (uint64_t *)(h->ws + off_tl);
    int32_t *te = (int32_t *)(h->ws + off_te);
    uint8_t *ts = (uint8_t *)(h->ws + off_ts);
    {
      ProfScope ps(h, OZ_STAGE_ROUND, (double)M * N * (4.0 * nwords + in_bytes), 0);
      if ((e = ozl::launch_limb_round(cw, nwords, M, N, ea, eb, hp->w, hp->g0, hp->Q, nlimb, tl,
                                      te, ts, M, MN, s)) != hipSuccess)
        return hip_fail(h, e, "limb round");
    }
    {
      ProfScope ps(h, OZ_STAGE_ROUND, (double)M * N * (3.0 * in_bytes + 8.0 * (2 * nlimb + 2)), 0);
      if ((e = ozl::launch_limb_sub(C->limb, C->exp, C->sign, C->ld, C->plane, tl, te, ts, nlimb, M,
                                    N, cw, s)) != hipSuccess)
        return hip_fail(h, e, "limb update");
    }
  }
  return OZII_OK;
}

// Pivot-candidate and zero-pivot scratch of the limb LU (allocated once).
ozII_status limb_scratch(ozII_ctx *h) {
  if (h->lcand) return OZII_OK;
  hipError_t e = hipMalloc((void **)&h->lcand, sizeof(int64_t) * ozl::LPIV_MAXGRID + 256);
  if (e != hipSuccess) return hip_fail(h, e, "hipMalloc(limb pivot scratch)");
  h->lflag = (int32_t *)(h->lcand + ozl::LPIV_MAXGRID);
  return OZII_OK;
}

// the sub-matrix starting at element (i, j)
ozII_limbs limbs_at(const ozII_limbs *A, int64_t i, int64_t j) {
  const int64_t off = i + j * A->ld;
  ozII_limbs r;
  r.limb = A->limb + off;
  r.exp = A->exp + off;
  r.sign = A->sign + off;
  r.ld = A->ld;
  r.plane = A->plane;
  return r;
}

ozl::LimbMat limb_mat(const ozII_limbs *A) {
  ozl::LimbMat m;
  m.limb = A->limb;
  m.exp = A->exp;
  m.sign = A->sign;
  m.ld = A->ld;
  m.plane = A->plane;
  return m;
}

// Left part of a recursive split of w > leaf columns (or rows): half of the
// leaf-wide blocks, rounded up.
int64_t limb_split(int64_t w, int64_t leaf) {
  const int64_t blocks = (w + leaf - 1) / leaf;
  return (blocks + 1) / 2 * leaf;
}

// The steps of the LU on limb matrices (Sec. 3.4) on one n x n matrix:
// panel, U12 solve and updates; with leaf > 0 the panel and the solve
// recurse on halves down to leaf columns (rows) and their inner updates are
// made like the Schur update -- the Ozaki-II product of the panel that
// Sec. 5.2 proposes.
struct LimbLU {
  ozII_ctx *h;
  const ozII_limbs *A;
  ozl::LimbMat M;
  int nl;
  int64_t n;
  int method;
  int64_t leaf;
  const ozII_opts *o;
  int64_t *ipiv;
  int32_t *info;

  double el() const { return 8.0 * nl + 5.0; }

  // the inner dimensions of the updates a panel (or, solve = true, a U12
  // solve) of width w makes
  void inner_dims(int64_t w, std::vector<int64_t> &ks, bool solve) const {
    if (solve) ks.push_back(w);  // the Schur update after this panel
    if (!leaf || w <= leaf) return;
    const int64_t w1 = limb_split(w, leaf);
    ks.push_back(w1);
    inner_dims(w1, ks, false);
    inner_dims(w - w1, ks, false);
  }

  // A[i0:i1, c0:c1] -= A[i0:i1, k0:k0+K] A[k0:k0+K, c0:c1]
  ozII_status update(int64_t i0, int64_t i1, int64_t c0, int64_t c1, int64_t k0, int64_t K) {
    if (i1 <= i0 || c1 <= c0 || K <= 0) return OZII_OK;
    if (method == OZII_METHOD_NAIVE) {
      ProfScope ps(h, OZ_STAGE_NAIVE, el() * (double)(i1 - i0) * (c1 - c0), 0);
      const hipError_t e = ozl::launch_lschur_naive(M, nl, i0, i1, c0, c1, k0, K, h->stream);
      return e == hipSuccess ? OZII_OK : hip_fail(h, e, "limb native update");
    }
    const ozII_limbs La = limbs_at(A, i0, k0), Lb = limbs_at(A, k0, c0);
    ozII_limbs Lc = limbs_at(A, i0, c0);
    return gemm_limbs_impl(h, 1, nl, i1 - i0, c1 - c0, K, &La, &Lb, &Lc, o);
  }

  // A[r0:r0+hh, b0:b1] <- L^-1 A[r0:r0+hh, b0:b1], L unit lower at (r0, r0)
  ozII_status trsm(int64_t r0, int64_t hh, int64_t b0, int64_t b1) {
    if (b1 <= b0 || hh <= 1) return OZII_OK;
    if (!leaf || hh <= leaf) {
      ProfScope ps(h, OZ_STAGE_TRSM, el() * (double)hh * (b1 - b0), 0);
      const hipError_t e = ozl::launch_ltrsm(M, nl, r0, hh, b0, b1, h->stream);
      return e == hipSuccess ? OZII_OK : hip_fail(h, e, "limb U12 solve");
    }
    const int64_t h1 = limb_split(hh, leaf);
    ozII_status st;
    if ((st = trsm(r0, h1, b0, b1)) != OZII_OK) return st;
    if ((st = update(r0 + h1, r0 + hh, b0, b1, r0, h1)) != OZII_OK) return st;
    return trsm(r0 + h1, hh - h1, b0, b1);
  }

  // columns [c0, c0+w) over rows [c0, n), interchanges across [P0, P1)
  ozII_status panel(int64_t c0, int64_t w, int64_t P0, int64_t P1) {
    if (!leaf || w <= leaf) {
      // interchanges inside the leaf per column, then on the rest of the
      // panel once per leaf (the same rows end up in the same places)
      ProfScope ps(h, OZ_STAGE_PANEL, el() * (double)(n - c0) * w, 0);
      for (int64_t j = c0; j < c0 + w; ++j) {
        const hipError_t e = ozl::launch_lpanel_column(M, nl, j, n, c0, c0 + w, c0 + w, h->lcand,
                                                       ipiv, info, h->lflag, h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "limb panel");
      }
      const hipError_t e = ozl::launch_llaswp(M, nl, ipiv, c0, w, P0, c0, c0 + w, P1, h->stream);
      return e == hipSuccess ? OZII_OK : hip_fail(h, e, "limb panel interchanges");
    }
    const int64_t w1 = limb_split(w, leaf);
    ozII_status st;
    if ((st = panel(c0, w1, P0, P1)) != OZII_OK) return st;
    if ((st = trsm(c0, w1, c0 + w1, c0 + w)) != OZII_OK) return st;
    if ((st = update(c0 + w1, n, c0 + w1, c0 + w, c0, w1)) != OZII_OK) return st;
    return panel(c0 + w1, w - w1, P0, P1);
  }
};

// The side stream and the fork / join events of the look-ahead (created on
// first use, on the handle's device, at the default priority).
ozII_status ensure_side(ozII_ctx *h) {
  if (h->side) return OZII_OK;
  hipError_t e = hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming);
  if (e != hipSuccess) return hip_fail(h, e, "look-ahead stream");
  return OZII_OK;
}

// Workspace of getrf's Ozaki-II updates: one region for the look-ahead
// columns (the next panel's, on the handle's stream) and one for the rest of
// the update (on the side stream), which run concurrently.
struct LuWs {
  size_t la_off = 0, la_cap = 0, rest_off = 0, rest_cap = 0, total = 0;
};

LuWs lu_workspace(const HostPlan &hp, int64_t n, int b, int tile, bool lookahead) {
  LuWs w;
  if (n <= b) return w;
  if (!lookahead) {  // one product per step over the whole trailing matrix
    w.la_cap = w.total = gemm_layout(hp, n - b, n - b, b, tile).total;
    return w;
  }
  w.la_cap = gemm_layout(hp, n - b, b, b, tile).total;
  w.rest_off = (w.la_cap + 255) / 256 * 256;
  w.rest_cap = n > 2 * b ? gemm_layout(hp, n - b, n - 2 * b, b, tile).total : 0;
  w.total = w.rest_off + w.rest_cap;
  return w;
}

}  // namespace

extern "C" {

ozII_status ozII_gemm_limbs(ozII_handle h, int32_t mode, int32_t nlimb, int64_t M, int64_t N,
                            int64_t K, const ozII_limbs *A, const ozII_limbs *B, ozII_limbs *C,
                            const ozII_opts *o) {
  return gemm_limbs_impl(h, mode, nlimb, M, N, K, A, B, C, o);
}

ozII_status ozII_gemm_limbs_stages(ozII_handle h, int32_t mode, int32_t nlimb, int64_t M,
                                   int64_t N, int64_t K, const ozII_limbs *A,
                                   const ozII_limbs *B, ozII_limbs *C, const ozII_opts *o,
                                   uint64_t *sbar, int32_t nlimb_out) {
  if (!h) return OZII_EINVAL;
  if (sbar && (nlimb_out < 1 || nlimb_out > 6)) return fail(h, OZII_EINVAL, "nlimb_out must be 1..6");
  return gemm_limbs_impl(h, mode, nlimb, M, N, K, A, B, C, o, sbar, nlimb_out);
}

ozII_status ozII_create(ozII_handle *out, int device, void *stream) {
  if (!out) return OZII_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return OZII_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return OZII_EHIP;
  // the static scratch of ozII_gemm_noalloc, mapped with this device
  // current (a failure is reported by ozII_gemm_noalloc, not here)
  noalloc_map(device);
  ozII_ctx *h = new ozII_ctx();
  h->device = device;
  h->stream = (hipStream_t)stream;
  *out = h;
  return OZII_OK;
}

ozII_status ozII_destroy(ozII_handle h) {
  if (!h) return OZII_EINVAL;
  hipStreamSynchronize(h->stream);
  if (h->ws) hipFree(h->ws);
  for (auto &kv : h->plans) hipFree(kv.second.second);
  for (auto ev : h->pool) hipEventDestroy(ev);
  if (h->side) {
    hipStreamSynchronize(h->side);
    hipStreamDestroy(h->side);
  }
  if (h->ev_fork) hipEventDestroy(h->ev_fork);
  if (h->ev_join) hipEventDestroy(h->ev_join);
  if (h->batch) hipFree(h->batch);
  if (h->batch_queue) hipFree(h->batch_queue);
  if (h->batch_ws) hipFree(h->batch_ws);
  if (h->lcand) hipFree(h->lcand);
  if (h->bar) {
    hipFree(h->bar);
    hipFree(h->flags);
    hipFree(h->crow);
    hipFree(h->perm);
    hipFree(h->moved);
  }
  delete h;
  return OZII_OK;
}

ozII_status ozII_set_stream(ozII_handle h, void *stream) {
  if (!h) return OZII_EINVAL;
  h->stream = (hipStream_t)stream;
  return OZII_OK;
}

ozII_status ozII_plan_query(int32_t p, int64_t K, const ozII_opts *o, int32_t *S, int32_t *w,
                            int32_t *Q, int32_t *nmod, int32_t *moduli) {
  HostPlan pl;
  ozII_status st = make_plan(p, K, o, pl, nullptr, false);
  if (st != OZII_OK) return st;
  if (S) *S = pl.S;
  if (w) *w = pl.w;
  if (Q) *Q = pl.Q;
  if (nmod) *nmod = pl.nmod;
  if (moduli)
    for (int i = 0; i < pl.nmod && i < 64; ++i) moduli[i] = pl.mods[i];
  return OZII_OK;
}

ozII_status ozII_reserve(ozII_handle h, int32_t nc, int64_t M, int64_t N, int64_t K, int64_t n,
                         const ozII_opts *o) {
  if (!h || !valid_nc(nc) || M < 0 || N < 0 || K < 0 || n < 0) return OZII_EINVAL;
  if (K > 0 && M > 0 && N > 0) {
    const HostPlan *hp;
    const DevPlan *dp;
    ozII_status st = get_plan(h, 53 * nc, K, o, &hp, &dp);
    if (st != OZII_OK) return st;
    st = ensure_ws(h, gemm_layout(*hp, M, N, K, o ? o->gemm_tile : 0).total);
    if (st != OZII_OK) return st;
  }
  if (n > 0) {
    const int b = (o && o->block > 0) ? o->block : 256;
    ozII_status st = ensure_panel(h, n, b);
    if (st != OZII_OK) return st;
    if (!(o && o->method == OZII_METHOD_NAIVE) && n > b) {
      const HostPlan *hp;
      const DevPlan *dp;
      st = get_plan(h, 53 * nc, b, o, &hp, &dp);
      if (st != OZII_OK) return st;
      const bool la = !(o && (o->flags & OZII_F_NO_LOOKAHEAD));
      st = ensure_ws(h, lu_workspace(*hp, n, b, o ? o->gemm_tile : 0, la).total);
      if (st != OZII_OK) return st;
      if (la) {
        st = ensure_side(h);
        if (st != OZII_OK) return st;
      }
    }
  }
  return OZII_OK;
}

ozII_status ozII_gemm(ozII_handle h, int32_t mode, int32_t nc, int64_t M, int64_t N, int64_t K,
                      const double *A, int64_t lda, const double *B, int64_t ldb, double *C,
                      int64_t ldc, const ozII_opts *o) {
  return gemm_impl(h, mode, nc, M, N, K, A, lda, B, ldb, C, ldc, o, nullptr, nullptr, nullptr,
                   nullptr, nullptr, nullptr, 0);
}

ozII_status ozII_gemm_noalloc(ozII_handle h, int32_t mode, int32_t nc, int64_t M, int64_t N,
                              int64_t K, const double *A, int64_t lda, const double *B,
                              int64_t ldb, double *C, int64_t ldc, const ozII_opts *o) {
  if (!h) return OZII_EINVAL;
  ++h->prof_block;
  const ozII_status st = gemm_impl(h, mode, nc, M, N, K, A, lda, B, ldb, C, ldc, o, nullptr,
                                   nullptr, nullptr, nullptr, nullptr, nullptr, 0, true);
  --h->prof_block;
  return st;
}

ozII_status ozII_gemm_noalloc_capacity(int64_t *bytes) {
  if (!bytes) return OZII_EINVAL;
  *bytes = (int64_t)(NOALLOC_BYTES - NOALLOC_WS_OFF);
  return OZII_OK;
}

ozII_status ozII_gemm_stages(ozII_handle h, int32_t mode, int32_t nc, int64_t M, int64_t N,
                             int64_t K, const double *A, int64_t lda, const double *B,
                             int64_t ldb, double *C, int64_t ldc, const ozII_opts *o,
                             int32_t *ea, int32_t *eb, void *planesA, void *planesB,
                             void *tpl, uint64_t *sbar, int32_t nlimb) {
  if (sbar && (nlimb < 1 || nlimb > 6)) return fail(h, OZII_EINVAL, "nlimb must be 1..6");
  return gemm_impl(h, mode, nc, M, N, K, A, lda, B, ldb, C, ldc, o, ea, eb, planesA, planesB, tpl,
                   sbar, nlimb);
}

ozII_status ozII_gemm_stage_dims(int32_t nc, int64_t M, int64_t N, int64_t K, const ozII_opts *o,
                                 int64_t *Mp, int64_t *Np, int64_t *Kp, int32_t *S,
                                 int32_t *nmod, int32_t *ng) {
  if (!valid_nc(nc) || M <= 0 || N <= 0 || K <= 0) return OZII_EINVAL;
  HostPlan pl;
  ozII_status st = make_plan(53 * nc, K, o, pl, nullptr);
  if (st != OZII_OK) return st;
  GemmLayout L = gemm_layout(pl, M, N, K, o ? o->gemm_tile : 0);
  if (Mp) *Mp = L.Mp;
  if (Np) *Np = L.Np;
  if (Kp) *Kp = L.Kp;
  if (S) *S = pl.S;
  if (nmod) *nmod = pl.nmod;
  if (ng) *ng = pl.ng;
  return OZII_OK;
}

ozII_status ozII_getrf(ozII_handle h, int32_t nc, int64_t n, double *A, int64_t lda,
                       int64_t *ipiv, int32_t *info, const ozII_opts *o) {
  if (!h) return OZII_EINVAL;
  if (!valid_nc(nc)) return fail(h, OZII_EUNSUPPORTED, "nc must be 2, 3 or 4");
  if (n < 0 || lda < std::max<int64_t>(n, 1)) return fail(h, OZII_EINVAL, "bad n or lda");
  if (n == 0) return OZII_OK;
  if (!A || !ipiv || !info) return fail(h, OZII_EINVAL, "null pointer");
  const int b = (o && o->block > 0) ? o->block : 256;
  const int method = o ? o->method : OZII_METHOD_OZAKI;
  const int flags = o ? o->flags : 0;
  if (b > 512) return fail(h, OZII_EUNSUPPORTED, "panel width above 512");
  if (method != OZII_METHOD_OZAKI && method != OZII_METHOD_NAIVE) return fail(h, OZII_EINVAL, "bad method");
  if (flags & ~(OZII_F_NO_LOOKAHEAD | OZII_F_FUSED)) return fail(h, OZII_EINVAL, "unknown flags");
  if (n > (int64_t)1 << 20) return fail(h, OZII_EUNSUPPORTED, "n too large");
  const bool lookahead = !(flags & OZII_F_NO_LOOKAHEAD);
  ozII_status st = ensure_panel(h, n, b);
  if (st != OZII_OK) return st;
  LuWs W;
  if (method == OZII_METHOD_OZAKI && n > b) {
    const HostPlan *hp;
    const DevPlan *dp;
    st = get_plan(h, 53 * nc, b, o, &hp, &dp);
    if (st != OZII_OK) return st;
    W = lu_workspace(*hp, n, b, o ? o->gemm_tile : 0, lookahead);
    st = ensure_ws(h, W.total);
    if (st != OZII_OK) return st;
  }
  if (lookahead && n > b) {
    st = ensure_side(h);
    if (st != OZII_OK) return st;
  }
  hipStream_t s = h->stream;
  hipError_t e;
  // C -= L21 U12 on columns [c0, c0 + nb) of the trailing matrix at step k,
  // on stream st with workspace region (off, cap)
  auto update = [&](int64_t k, int kb, int64_t c0, int64_t nb, hipStream_t st_, size_t off,
                    size_t cap) -> ozII_status {
    const int64_t m2 = n - k - kb;
    const double *L21 = A + ((k + kb) + k * lda) * nc;
    const double *U12 = A + (k + (k + kb + c0) * lda) * nc;
    double *A22 = A + ((k + kb) + (k + kb + c0) * lda) * nc;
    if (method == OZII_METHOD_OZAKI)
      return gemm_impl(h, 1, nc, m2, nb, kb, L21, lda, U12, lda, A22, lda, o, nullptr, nullptr,
                       nullptr, nullptr, nullptr, nullptr, 0, false, st_, h->ws + off, cap);
    ProfScope ps(h, OZ_STAGE_NAIVE, 16.0 * nc * (double)m2 * nb + 16.0 * nc * (double)(m2 + nb) * kb,
                 (double)m2 * nb * kb, st_);
    const hipError_t ee = ozl::launch_naive_gemm(nc, L21, lda, U12, lda, A22, lda, m2, nb, kb, 0, st_);
    return ee == hipSuccess ? OZII_OK : hip_fail(h, ee, "naive update");
  };
  auto trsm = [&](int64_t k, int kb, int64_t c0, int64_t nb, hipStream_t st_) -> ozII_status {
    const double *L11 = A + (k + k * lda) * nc;
    double *A12 = A + (k + (k + kb + c0) * lda) * nc;
    ProfScope ps(h, OZ_STAGE_TRSM, 16.0 * nc * (double)kb * nb + 8.0 * nc * kb * kb / 2.0,
                 (double)nb * kb * kb / 2.0, st_);
    const hipError_t ee = ozl::launch_trsm_lower_unit(nc, L11, lda, A12, lda, kb, nb, st_);
    return ee == hipSuccess ? OZII_OK : hip_fail(h, ee, "trsm");
  };
  if ((e = ozl::launch_fill_int(info, 0, 1, s)) != hipSuccess) return hip_fail(h, e, "fill info");
  bool side_busy = false;
  for (int64_t k = 0; k < n; k += b) {
    const int kb = (int)std::min<int64_t>(b, n - k);
    const int64_t nr = n - k;
    // panel geometry: G co-resident workgroups of R rows each.  Fewer,
    // taller workgroups make the per-column exchange cheaper (every
    // workgroup reads every candidate line), so 128 are tried first and 256
    // when 128 would not hold the rows in LDS (static LDS of the kernel:
    // about 20 KiB).
    int G = 0, R = 0;
    for (int G0 : {128, 256}) {
      int g = G0, r = 0, maxb = 0;
      bool ok = false;
      for (;;) {
        r = (int)((nr + g - 1) / g);
        if (r > 32 || ozl::panel_lds_bytes(nc, kb, r, nr) + 20480 > 160 * 1024) break;
        e = ozl::panel_max_blocks(nc, kb, r, nr, &maxb);
        if (e != hipSuccess) return hip_fail(h, e, "panel occupancy");
        if (maxb >= g) {
          ok = true;
          break;
        }
        g = maxb;
        if (g <= 0) break;
      }
      if (ok) {
        G = g;
        R = r;
        break;
      }
    }
    if (G <= 0) return fail(h, OZII_EUNSUPPORTED, "panel does not fit in LDS for a resident kernel");
    G = (int)std::min<int64_t>(G, (nr + R - 1) / R);
    if ((e = ozl::launch_fill_int((int *)h->flags, 0, 2 * 32 * 256, s)) != hipSuccess) return hip_fail(h, e, "fill lines");
    // a panel that stops early leaves no moved rows behind for laswp
    if ((e = ozl::launch_fill_int(h->nmoved, 0, 1, s)) != hipSuccess) return hip_fail(h, e, "fill nmoved");
    {
      // (P1) panel k; with look-ahead it runs while the side stream finishes
      // the previous step's update on the columns right of it
      ProfScope ps(h, OZ_STAGE_PANEL, 16.0 * nc * (double)nr * kb, (double)nr * kb * kb / 2.0);
      if ((e = ozl::launch_panel(nc, A, lda, n, k, kb, R, G, ipiv, info, h->flags, h->err, h->crow,
                                 h->perm, h->moved, h->nmoved, s)) != hipSuccess)
        return hip_fail(h, e, "panel");
    }
    if (side_busy) {
      // join: the interchanges below touch the columns the side stream updates
      if ((e = hipEventRecord(h->ev_join, h->side)) != hipSuccess) return hip_fail(h, e, "join record");
      if ((e = hipStreamWaitEvent(s, h->ev_join, 0)) != hipSuccess) return hip_fail(h, e, "join wait");
      side_busy = false;
    }
    {
      ProfScope ps(h, OZ_STAGE_LASWP, 32.0 * nc * (double)kb * n, 0);
      if ((e = ozl::launch_laswp(nc, A, lda, k, 0, n, h->perm, h->moved, h->nmoved, s)) != hipSuccess)
        return hip_fail(h, e, "laswp");
    }
    if (k + kb >= n) break;
    const int64_t m2 = n - k - kb;
    // (P3) + (P4): the next panel's columns first (look-ahead), then the rest
    const int64_t la = lookahead ? std::min<int64_t>(b, m2) : m2;
    if ((st = trsm(k, kb, 0, la, s)) != OZII_OK) return st;
    if ((st = update(k, kb, 0, la, s, 0, W.la_cap)) != OZII_OK) return st;
    if (la < m2) {
      if ((e = hipEventRecord(h->ev_fork, s)) != hipSuccess) return hip_fail(h, e, "fork record");
      if ((e = hipStreamWaitEvent(h->side, h->ev_fork, 0)) != hipSuccess) return hip_fail(h, e, "fork wait");
      if ((st = trsm(k, kb, la, m2 - la, h->side)) != OZII_OK) return st;
      if ((st = update(k, kb, la, m2 - la, h->side, W.rest_off, W.rest_cap)) != OZII_OK) return st;
      side_busy = true;
    }
  }
  if (side_busy) {
    if ((e = hipEventRecord(h->ev_join, h->side)) != hipSuccess) return hip_fail(h, e, "join record");
    if ((e = hipStreamWaitEvent(s, h->ev_join, 0)) != hipSuccess) return hip_fail(h, e, "join wait");
  }
  return OZII_OK;
}

ozII_status ozII_getrs(ozII_handle h, int32_t nc, int64_t n, int64_t nrhs, const double *LU,
                       int64_t lda, const int64_t *ipiv, double *B, int64_t ldb) {
  if (!h) return OZII_EINVAL;
  if (!valid_nc(nc)) return fail(h, OZII_EUNSUPPORTED, "nc must be 2, 3 or 4");
  if (n < 0 || nrhs < 0 || lda < std::max<int64_t>(n, 1) || ldb < std::max<int64_t>(n, 1))
    return fail(h, OZII_EINVAL, "bad size or leading dimension");
  if (n == 0 || nrhs == 0) return OZII_OK;
  if (!LU || !ipiv || !B) return fail(h, OZII_EINVAL, "null pointer");
  hipStream_t s = h->stream;
  hipError_t e;
  ProfScope ps(h, OZ_STAGE_GETRS, 8.0 * nc * (double)n * n + 16.0 * nc * (double)n * nrhs,
               (double)n * n * nrhs);
  if ((e = ozl::launch_apply_ipiv(nc, B, ldb, n, nrhs, ipiv, s)) != hipSuccess) return hip_fail(h, e, "apply ipiv");
  if (nrhs == 1) {
    // one right-hand side: the pipelined solves (same operations per element)
    if (!h->bar) {
      const ozII_status st = ensure_panel(h, 1, 1);
      if (st != OZII_OK) return st;
    }
    uint32_t *sync = h->bar + 12;  // finished-position counter and row-block ticket
    if ((e = ozl::launch_trsv(nc, 1, LU, lda, B, n, sync, h->err, s)) != hipSuccess)
      return hip_fail(h, e, "forward solve");
    if ((e = ozl::launch_trsv(nc, 0, LU, lda, B, n, sync, h->err, s)) != hipSuccess)
      return hip_fail(h, e, "backward solve");
    return OZII_OK;
  }
  const int bs = 256;
  for (int64_t i0 = 0; i0 < n; i0 += bs) {
    const int ib = (int)std::min<int64_t>(bs, n - i0);
    if ((e = ozl::launch_trsm_lower_unit(nc, LU + (i0 + i0 * lda) * nc, lda, B + i0 * nc, ldb, ib, nrhs, s)) != hipSuccess)
      return hip_fail(h, e, "forward block");
    if (i0 + ib < n) {
      if ((e = ozl::launch_naive_gemm(nc, LU + ((i0 + ib) + i0 * lda) * nc, lda, B + i0 * nc, ldb,
                                      B + (i0 + ib) * nc, ldb, n - i0 - ib, nrhs, ib, 0, s)) != hipSuccess)
        return hip_fail(h, e, "forward update");
    }
  }
  const int64_t nblk = (n + bs - 1) / bs;
  for (int64_t bi = nblk - 1; bi >= 0; --bi) {
    const int64_t j0 = bi * bs;
    const int ib = (int)std::min<int64_t>(bs, n - j0);
    if ((e = ozl::launch_trsm_upper(nc, LU + (j0 + j0 * lda) * nc, lda, B + j0 * nc, ldb, ib, nrhs,
                                    s)) != hipSuccess)
      return hip_fail(h, e, "backward block");
    if (j0 > 0) {
      if ((e = ozl::launch_naive_gemm(nc, LU + (j0 * lda) * nc, lda, B + j0 * nc, ldb, B, ldb, j0,
                                      nrhs, ib, 1, s)) != hipSuccess)
        return hip_fail(h, e, "backward update");
    }
  }
  return OZII_OK;
}

ozII_status ozII_getrf_limbs(ozII_handle h, int32_t nlimb, int64_t n, ozII_limbs *A,
                             int64_t *ipiv, int32_t *info, const ozII_opts *o) {
  if (!h) return OZII_EINVAL;
  if (nlimb < 1 || nlimb > 64) return fail(h, OZII_EINVAL, "nlimb must be 1..64");
  if (n < 0) return fail(h, OZII_EINVAL, "negative size");
  if (!ipiv || !info) return fail(h, OZII_EINVAL, "null pointer");
  if (n > 0 && !limbs_ok(A, n, n)) return fail(h, OZII_EINVAL, "bad limb matrix descriptor");
  if (o && o->backend && o->backend != OZII_BE_INT8)
    return fail(h, OZII_EUNSUPPORTED, "the limb format runs on the INT8 back-end only");
  const int method = o ? o->method : OZII_METHOD_OZAKI;
  if (method != OZII_METHOD_OZAKI && method != OZII_METHOD_NAIVE)
    return fail(h, OZII_EINVAL, "unknown method");
  if (o && o->panel_leaf < 0) return fail(h, OZII_EINVAL, "negative panel leaf");
  LimbLU L;
  L.h = h;
  L.A = A;
  L.M = limb_mat(A);
  L.nl = nlimb;
  L.n = n;
  L.method = method;
  L.leaf = o ? o->panel_leaf : 0;
  L.o = o;
  L.ipiv = ipiv;
  L.info = info;
  const int64_t b = (o && o->block > 0) ? o->block : 256;
  ozII_status st = limb_scratch(h);
  if (st != OZII_OK) return st;
  if (method == OZII_METHOD_OZAKI) {
    // the plans of every inner dimension the updates use, before anything runs
    std::vector<int64_t> ks;
    for (int64_t k0 = 0; k0 < n; k0 += b) {
      const int64_t kb = std::min(b, n - k0);
      if (n - k0 - kb > 0) L.inner_dims(kb, ks, true);
      L.inner_dims(kb, ks, false);
    }
    std::sort(ks.begin(), ks.end());
    ks.erase(std::unique(ks.begin(), ks.end()), ks.end());
    for (int64_t K : ks) {
      const HostPlan *hp;
      const DevPlan *dp;
      if ((st = get_plan(h, 64 * nlimb, K, o, &hp, &dp, true)) != OZII_OK) return st;
    }
  }
  hipError_t e;
  if ((e = ozl::launch_lfill_i32(info, 0, 1, h->stream)) != hipSuccess) return hip_fail(h, e, "info");
  const double el = 8.0 * nlimb + 5.0;
  for (int64_t k0 = 0; k0 < n; k0 += b) {
    const int64_t kb = std::min(b, n - k0);
    if ((st = L.panel(k0, kb, k0, k0 + kb)) != OZII_OK) return st;
    {
      ProfScope ps(h, OZ_STAGE_LASWP, 2.0 * el * kb * (double)(n - kb), 0);
      if ((e = ozl::launch_llaswp(L.M, nlimb, ipiv, k0, kb, 0, k0, k0 + kb, n, h->stream)) != hipSuccess)
        return hip_fail(h, e, "limb laswp");
    }
    if (n - k0 - kb == 0) continue;
    if ((st = L.trsm(k0, kb, k0 + kb, n)) != OZII_OK) return st;
    if ((st = L.update(k0 + kb, n, k0 + kb, n, k0, kb)) != OZII_OK) return st;
  }
  return OZII_OK;
}

ozII_status ozII_getrs_limbs(ozII_handle h, int32_t nlimb, int64_t n, int64_t nrhs,
                             const ozII_limbs *LU, const int64_t *ipiv, ozII_limbs *B) {
  if (!h) return OZII_EINVAL;
  if (nlimb < 1 || nlimb > 64) return fail(h, OZII_EINVAL, "nlimb must be 1..64");
  if (n < 0 || nrhs < 0) return fail(h, OZII_EINVAL, "negative size");
  if (n == 0 || nrhs == 0) return OZII_OK;
  if (!ipiv || !limbs_ok(LU, n, n) || !limbs_ok(B, n, nrhs))
    return fail(h, OZII_EINVAL, "bad limb matrix descriptor or null pointer");
  ProfScope ps(h, OZ_STAGE_GETRS, (8.0 * nlimb + 5.0) * ((double)n * n + 2.0 * n * nrhs), 0);
  const hipError_t e = ozl::launch_lgetrs(limb_mat(LU), nlimb, n, ipiv, limb_mat(B), nrhs, h->stream);
  return e == hipSuccess ? OZII_OK : hip_fail(h, e, "limb solve");
}

ozII_status ozII_limbs_arith(ozII_handle h, int32_t op, int32_t nlimb, int64_t count,
                             const ozII_limbs *A, const ozII_limbs *B, ozII_limbs *C) {
  if (!h) return OZII_EINVAL;
  if (op < 0 || op > 3) return fail(h, OZII_EINVAL, "op must be 0..3");
  if (nlimb < 1 || nlimb > 64) return fail(h, OZII_EINVAL, "nlimb must be 1..64");
  if (count < 0) return fail(h, OZII_EINVAL, "negative size");
  if (count == 0) return OZII_OK;
  if (!limbs_ok(A, count, 1) || !limbs_ok(B, count, 1) || !limbs_ok(C, count, 1))
    return fail(h, OZII_EINVAL, "bad limb vector descriptor");
  const hipError_t e = ozl::launch_larith(op, nlimb, count, limb_mat(A), limb_mat(B), limb_mat(C),
                                          h->stream);
  return e == hipSuccess ? OZII_OK : hip_fail(h, e, "limb arithmetic");
}

ozII_status ozII_batch_prepare(ozII_handle h, int32_t count, const ozII_batch_item *items) {
  return ozII_batch_prepare_ex(h, count, items, nullptr);
}

ozII_status ozII_batch_prepare_ex(ozII_handle h, int32_t count, const ozII_batch_item *items,
                                  const ozII_opts *o) {
  if (!h || count < 0 || (count > 0 && !items)) return OZII_EINVAL;
  const int method = o ? o->method : OZII_METHOD_NAIVE;
  if (method != OZII_METHOD_OZAKI && method != OZII_METHOD_NAIVE) return fail(h, OZII_EINVAL, "bad method");
  const bool oz = method == OZII_METHOD_OZAKI;
  const int b = oz ? ((o && o->block > 0) ? o->block : 32) : 0;
  if (oz && b > 256) return fail(h, OZII_EUNSUPPORTED, "batched Ozaki-II LU: panel width above 256");
  if (oz && o->backend != OZII_BE_AUTO && o->backend != OZII_BE_INT8)
    return fail(h, OZII_EUNSUPPORTED, "batched Ozaki-II LU: INT8 back-end only");
  std::vector<ozII_batch_item> v(items, items + count);
  int64_t nmax[3] = {0, 0, 0};
  for (int i = 0; i < count; ++i) {
    const ozII_batch_item &it = v[i];
    if (it.nc < 2 || it.nc > 4 || it.n < 1 || it.n > 4096 || !it.A || !it.ipiv || !it.info)
      return fail(h, OZII_EINVAL, "batch item " + std::to_string(i) + " is invalid");
    if (oz && it.n > 1024)
      return fail(h, OZII_EUNSUPPORTED, "batched Ozaki-II LU: order above 1024");
    v[i].reserved = i;
    nmax[it.nc - 2] = std::max(nmax[it.nc - 2], it.n);
  }
  // plans at K = b (those of ozII_getrf with the same block) and the scratch
  // of one workgroup: exponents, residue planes of L21 and U12, t-planes
  const DevPlan *pls[3] = {nullptr, nullptr, nullptr};
  int64_t slot = 0;
  if (oz) {
    ozII_opts po = *o;
    po.backend = OZII_BE_INT8;
    for (int c = 0; c < 3; ++c) {
      if (nmax[c] == 0) continue;
      const int nc = c + 2;
      const HostPlan *hp;
      const DevPlan *dp;
      ozII_status st = get_plan(h, 53 * nc, b, &po, &hp, &dp);
      if (st != OZII_OK) return st;
      const int nwt = (hp->w + 2 + 31) / 32;
      if (hp->nwx > 8 || nwt > (nc == 2 ? 6 : 4) || hp->nwc > 12 || hp->nd > 18 || hp->nmod > 40)
        return fail(h, OZII_EUNSUPPORTED, "batched Ozaki-II LU: plan exceeds the compiled word sizes");
      pls[c] = dp;
      const int64_t Mp = roundup(std::max<int64_t>(nmax[c] - b, 1), 64), Kp = roundup(b, 64);
      const int64_t bytes = 8 * Mp + 2 * (int64_t)hp->S * hp->nmod * Mp * Kp +
                            (int64_t)hp->ng * hp->nmod * Mp * Mp;
      slot = std::max(slot, roundup(bytes, 256));
    }
  }
  // longest processing time first: cost ~ nc n^3, ties in caller order
  std::stable_sort(v.begin(), v.end(), [](const ozII_batch_item &a, const ozII_batch_item &b) {
    return (double)a.nc * a.n * a.n * a.n > (double)b.nc * b.n * b.n * b.n;
  });
  hipError_t e;
  if (count > h->batch_cap) {
    if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return hip_fail(h, e, "hipStreamSynchronize");
    if (h->batch) hipFree(h->batch);
    h->batch = nullptr;
    h->batch_cap = 0;
    if ((e = hipMalloc((void **)&h->batch, sizeof(ozII_batch_item) * count)) != hipSuccess)
      return fail(h, OZII_ENOMEM, "batch table allocation failed");
    h->batch_cap = count;
  }
  if (!h->batch_queue && (e = hipMalloc((void **)&h->batch_queue, 256)) != hipSuccess)
    return fail(h, OZII_ENOMEM, "batch queue allocation failed");
  if (count > 0 &&
      (e = hipMemcpyAsync(h->batch, v.data(), sizeof(ozII_batch_item) * count, hipMemcpyHostToDevice,
                          h->stream)) != hipSuccess)
    return hip_fail(h, e, "batch upload");
  if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return hip_fail(h, e, "hipStreamSynchronize");
  // persistent grid: one workgroup per CU, at most one per item
  int dev = 0, ncu = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess ||
      (e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return hip_fail(h, e, "device query");
  const int grid = std::max(1, std::min(count, ncu));
  if (oz && (size_t)(slot * grid) > h->batch_ws_bytes) {
    if (h->batch_ws) hipFree(h->batch_ws);
    h->batch_ws = nullptr;
    h->batch_ws_bytes = 0;
    if ((e = hipMalloc((void **)&h->batch_ws, (size_t)(slot * grid))) != hipSuccess)
      return fail(h, OZII_ENOMEM, "batch scratch allocation failed");
    h->batch_ws_bytes = (size_t)(slot * grid);
  }
  h->batch_count = count;
  h->batch_grid = grid;
  h->batch_b = b;
  h->batch_slot = slot;
  for (int c = 0; c < 3; ++c) h->batch_pl[c] = pls[c];
  return OZII_OK;
}

ozII_status ozII_batch_run(ozII_handle h, uint64_t *times) {
  if (!h) return OZII_EINVAL;
  if (h->batch_count == 0) return OZII_OK;
  hipError_t e =
      h->batch_b > 0
          ? ozl::launch_batch_oz(h->batch, h->batch_count, h->batch_queue, times, h->batch_grid,
                                 h->batch_pl[0], h->batch_pl[1], h->batch_pl[2], h->batch_ws,
                                 h->batch_slot, h->batch_b, h->stream)
          : ozl::launch_batch(h->batch, h->batch_count, h->batch_queue, times, h->batch_grid,
                              h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "batched LU");
  return OZII_OK;
}

ozII_status ozII_stream_of(ozII_handle h, void **stream) {
  if (!h || !stream) return OZII_EINVAL;
  *stream = (void *)h->stream;
  return OZII_OK;
}

ozII_status ozII_sync_check(ozII_handle h) {
  if (!h) return OZII_EINVAL;
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "hipStreamSynchronize");
  if (h->err) {
    int v = 0;
    e = hipMemcpy(&v, h->err, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(h, e, "read error flag");
    if (v) return fail(h, OZII_EDEVICE, "a grid-wide wait timed out (panel exchange or pipelined solve)");
  }
  return OZII_OK;
}

ozII_status ozII_set_profiling(ozII_handle h, int32_t on) {
  if (!h) return OZII_EINVAL;
  h->profiling = on != 0;
  return OZII_OK;
}

ozII_status ozII_profile_read(ozII_handle h, int32_t nstages, double *ms, int64_t *launches,
                              double *bytes, double *ops) {
  if (!h || nstages < 0) return OZII_EINVAL;
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "hipStreamSynchronize");
  for (int i = 0; i < nstages; ++i) {
    if (ms) ms[i] = 0;
    if (launches) launches[i] = 0;
    if (bytes) bytes[i] = 0;
    if (ops) ops[i] = 0;
  }
  for (auto &r : h->prof) {
    if (r.stage < 0 || r.stage >= nstages) continue;
    float t = 0.f;
    e = hipEventElapsedTime(&t, r.a, r.b);
    if (e != hipSuccess) return hip_fail(h, e, "hipEventElapsedTime");
    if (ms) ms[r.stage] += t;
    if (launches) launches[r.stage] += 1;
    if (bytes) bytes[r.stage] += r.bytes;
    if (ops) ops[r.stage] += r.ops;
  }
  h->prof.clear();
  h->pool_used = 0;
  return OZII_OK;
}

const char *ozII_status_string(ozII_status s) {
  switch (s) {
    case OZII_OK: return "ok";
    case OZII_EINVAL: return "invalid argument";
    case OZII_ECAPACITY: return "plan exceeds the CRT capacity";
    case OZII_EOVERFLOW: return "accumulator bound violated";
    case OZII_ENOMEM: return "out of device memory";
    case OZII_EHIP: return "HIP runtime error";
    case OZII_EUNSUPPORTED: return "unsupported format or option";
    case OZII_EDEVICE: return "device-side error";
  }
  return "unknown status";
}

const char *ozII_last_error(ozII_handle h) { return h ? h->last_error.c_str() : ""; }

}  // extern "C"
