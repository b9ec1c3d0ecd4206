// Host orchestrator and C ABI of libknnd.so (declared in include/knnd.h).
//
// A context owns the device copy of the points, the log table, a double-
// buffered snapshot (lists and keys of round r-1 are read, round r written to
// the other half), the reverse-neighbor CSR, receiver bins and the per-round
// counters.  Each round enqueues every kernel on the caller's stream and
// synchronises once, to read the counters the stop test needs (Section 3.3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <mutex>
#include <new>
#include <unordered_map>
#include <utility>
#include <vector>

#include "knnd.h"
#include "knnd_internal.h"

struct knnd_ctx {
  knnd::Ctx c;
};

// ---------------------------------------------------------------------------
// Device memory cache.  A descent uses a few gigabytes of scratch at n = 1e6,
// and hipMalloc / hipFree of it cost several milliseconds per call; blocks a
// finished call gives back are kept (per device, by rounded size) and handed
// to later calls.  At most half of the first device's memory stays cached
// (the oldest go first: a cap below what alternating workloads use together
// frees and reallocates blocks on every call); knnd_release_cache() returns
// all of them.  Thread-safe.
// ---------------------------------------------------------------------------
namespace knnd {
namespace {
struct PoolBlock {
  void* p;
  size_t bytes;
  int dev;
};
std::mutex g_pool_mu;
std::vector<PoolBlock> g_cached;
std::unordered_map<void*, PoolBlock> g_live;
size_t g_cached_bytes = 0;
size_t g_live_bytes = 0;
size_t g_peak_live = 0;  // the most the library has had in use at once
size_t g_cap = 0;  // set on the first allocation (under g_pool_mu)

// Sizes are rounded up (to 256 bytes, above 1 MiB to an eighth of their
// power of two) so that calls of slightly different sizes share blocks.
size_t pool_round(size_t b) {
  if (b <= ((size_t)1 << 20)) return (b + 255) & ~(size_t)255;
  size_t p = (size_t)1 << 20;
  while (p < b) p <<= 1;
  const size_t q = p / 8;
  return (b + q - 1) / q * q;
}

void free_block(const PoolBlock& b) {
  int cur = 0;
  const bool other = hipGetDevice(&cur) == hipSuccess && cur != b.dev;
  if (other) (void)hipSetDevice(b.dev);
  (void)hipFree(b.p);
  if (other) (void)hipSetDevice(cur);
}
}  // namespace

std::atomic<int64_t> g_fail_at{0};  // test support: allocations to go before an injected failure

hipError_t pool_malloc(void** out, size_t bytes) {
  *out = nullptr;
  if (g_fail_at.load() > 0 && g_fail_at.fetch_sub(1) == 1) return hipErrorOutOfMemory;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const size_t rb = pool_round(bytes);
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if (g_cap == 0) {
      size_t total = 0;
      g_cap = (hipDeviceTotalMem(&total, dev) == hipSuccess && total > 0) ? total / 2 : ((size_t)64 << 30);
    }
    for (size_t i = 0; i < g_cached.size(); ++i) {
      if (g_cached[i].dev == dev && g_cached[i].bytes == rb) {
        const PoolBlock b = g_cached[i];
        g_cached.erase(g_cached.begin() + (std::ptrdiff_t)i);
        g_cached_bytes -= rb;
        g_live.emplace(b.p, b);
        g_live_bytes += rb;
        g_peak_live = std::max(g_peak_live, g_live_bytes);
        *out = b.p;
        return hipSuccess;
      }
    }
  }
  void* p = nullptr;
  e = hipMalloc(&p, rb);
  if (e == hipErrorOutOfMemory) {  // give the cached blocks back and try once more
    (void)hipGetLastError();
    pool_release();
    e = hipMalloc(&p, rb);
  }
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_pool_mu);
  g_live.emplace(p, PoolBlock{p, rb, dev});
  g_live_bytes += rb;
  g_peak_live = std::max(g_peak_live, g_live_bytes);
  *out = p;
  return hipSuccess;
}

void pool_free(void* p) {
  if (!p) return;
  std::vector<PoolBlock> drop;
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    auto it = g_live.find(p);
    if (it == g_live.end()) return;  // (every library block comes from pool_malloc)
    g_cached.push_back(it->second);
    g_cached_bytes += it->second.bytes;
    g_live_bytes -= it->second.bytes;
    g_live.erase(it);
    // the cache keeps up to half the device's memory, or as much as the
    // library has had in use at once if that is more (so that a call larger
    // than half the memory, repeated, reuses its blocks)
    const size_t cap = std::max(g_cap, g_peak_live);
    while (g_cached_bytes > cap && !g_cached.empty()) {
      drop.push_back(g_cached.front());
      g_cached_bytes -= g_cached.front().bytes;
      g_cached.erase(g_cached.begin());
    }
  }
  for (const PoolBlock& b : drop) free_block(b);
}

void pool_stats(int64_t* live, int64_t* cached) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if (live) *live = (int64_t)g_live_bytes;
  if (cached) *cached = (int64_t)g_cached_bytes;
}

void pool_release() {
  std::vector<PoolBlock> drop;
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    drop.swap(g_cached);
    g_cached_bytes = 0;
    g_peak_live = g_live_bytes;  // (the cap starts over)
  }
  for (const PoolBlock& b : drop) free_block(b);
}
}  // namespace knnd

namespace {

using knnd::Ctx;

int map_err(hipError_t e) { return e == hipErrorOutOfMemory ? KNND_ERR_NOMEM : KNND_ERR_DEVICE; }

#define KNND_HIP(x)                                   \
  do {                                                \
    hipError_t e_ = (x);                              \
    if (e_ != hipSuccess) return map_err(e_);         \
  } while (0)

// Device buffers of a context: from the memory cache, or (fixed-scratch
// mode) carved from the context's arena at 256-byte alignment.
hipError_t ctx_alloc(Ctx& c, void** p, size_t bytes) {
  if (!c.arena) return knnd::pool_malloc(p, bytes);
  *p = nullptr;
  const size_t off = (c.arena_used + 255) & ~(size_t)255;
  if (off > c.arena_size || bytes > c.arena_size - off) return hipErrorOutOfMemory;
  *p = c.arena + off;
  c.arena_used = off + bytes;
  return hipSuccess;
}

template <class T>
hipError_t dalloc(Ctx& c, T** p, size_t count) {
  return ctx_alloc(c, reinterpret_cast<void**>(p), count * sizeof(T) + 16);
}

template <class T>
hipError_t balloc(Ctx& c, T** p, size_t bytes) {
  return ctx_alloc(c, reinterpret_cast<void**>(p), bytes);
}

// Give back optional buffers whose allocation did not complete (arena: roll
// the bump pointer back to `mark`); the pointers are cleared.
template <class... T>
void drop_optional(Ctx& c, size_t mark, T**... ps) {
  (void)hipGetLastError();
  if (c.arena)
    c.arena_used = mark;
  else
    (knnd::pool_free(*ps), ...);
  ((*ps = nullptr), ...);
}

// HIP events of the per-round timings (none in fixed-scratch mode)
hipError_t rec(hipEvent_t ev, hipStream_t s) { return ev ? hipEventRecord(ev, s) : hipSuccess; }

void free_ctx(Ctx& c) {
  void* bufs[] = {c.P,      c.L,      c.F[0],   c.F[1],      c.keys[0],     c.keys[1],  c.deg,
                  c.fill,   c.rowptr, c.col,    c.colslot,   c.seg,
                  c.tilesum, c.class_count, c.class_list, c.gtab, c.gcand, c.gckey, c.bcand, c.bckey,
                  c.dstats, c.dflag, c.Ph, c.Lh, c.S, c.seg32,
                  c.inst_of, c.ioff, c.iseed, c.iM, c.iD, c.iactive, c.istats, c.vcnt,
                  c.sl_n, c.sl_id, c.sl_key, c.csr_T, c.csr_bcount, c.csr_bfill, c.csr_bbase, c.Pw,
                  c.vchg, c.vev, c.Hrow};
  // the blocks go back to the cache: the context's work must have finished
  (void)hipStreamSynchronize(c.stream);
  if (!c.arena)
    for (void* b : bufs) knnd::pool_free(b);
  if (c.hstats && c.hstats != c.hstats_local) (void)hipHostFree(c.hstats);
  if (c.histats) (void)hipHostFree(c.histats);
  if (c.ev0) (void)hipEventDestroy(c.ev0);
  if (c.ev1) (void)hipEventDestroy(c.ev1);
  if (c.evj0) (void)hipEventDestroy(c.evj0);
  if (c.evj1) (void)hipEventDestroy(c.evj1);
  if (c.evh) (void)hipEventDestroy(c.evh);
  c = Ctx();
}

int64_t next_pow2(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

int resolve_params(const knnd_params* p, int64_t n, knnd_params* out) {
  knnd_default_params(out);
  if (p) *out = *p;
  if (out->fcr_samples <= 0) out->fcr_samples = n < 10000 ? n : 10000;
  if (out->max_rounds <= 0) out->max_rounds = 100;
  if (out->dtype != KNND_F32 && out->dtype != KNND_F64) return KNND_ERR_ARG;
  if (out->precision < KNND_PREC_FP64 || out->precision > KNND_PREC_AUTO) return KNND_ERR_ARG;
  if (out->stop_rule < KNND_STOP_FCR || out->stop_rule > KNND_STOP_DELTA) return KNND_ERR_ARG;
  if (out->comparator < KNND_CMP_KL || out->comparator > KNND_CMP_L2) return KNND_ERR_ARG;
  if (!(out->delta >= 0.0) || !std::isfinite(out->delta)) return KNND_ERR_ARG;
  return KNND_OK;
}

int check_shape(int64_t n, int32_t d, int32_t K) {
  if (n < 2 || d < 1 || K < 2 || K > n - 1 || K > 64) return KNND_ERR_ARG;
  if (n >= (int64_t)knnd::IDMASK_HOST) return KNND_ERR_ARG;
  if (d > 1 << 20) return KNND_ERR_ARG;
  return KNND_OK;
}

int prepare_mixed(Ctx& c, size_t nK);

// Device check, fields and every device buffer of a context of n points
// (a single instance, or a batched group with its per-instance arrays
// allocated by the caller).
int setup(Ctx& c, int64_t n, int32_t d, int32_t K, uint64_t seed, const knnd_params& prm, void* stream) {
  KNND_HIP(hipGetDevice(&c.device));
  hipDeviceProp_t prop;
  KNND_HIP(hipGetDeviceProperties(&prop, c.device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return KNND_ERR_DEVICE;
  c.num_cu = prop.multiProcessorCount;
  c.stream = reinterpret_cast<hipStream_t>(stream);
  c.n = n;
  c.own0 = 0;
  c.own1 = n;
  c.d = d;
  c.D = d + 1;
  c.Dp = (c.D + 1) & ~1;
  c.Ds = c.D | 1;  // odd LDS row stride (in doubles) for conflict-free column reads
  c.K = K;
  c.Ks = 8;
  while (c.Ks < K) c.Ks <<= 1;
  c.seed = seed;
  c.dtype = prm.dtype;
  // (the automatic mode splits operands like the BF16 mode when it runs mixed)
  c.auto_prec = prm.precision == KNND_PREC_AUTO;
  c.precision = c.auto_prec ? KNND_PREC_MIXED_BF16 : prm.precision;
  c.flags = prm.flags;
  // (the tuner times with HIP events: none in fixed-scratch mode)
  c.tune = c.auto_prec && !c.arena && !(prm.flags & KNND_FLAG_NO_TUNE);
  c.cmp = prm.comparator;
  c.ck = knnd::cmp_fold_kind(c.cmp);
  c.tk = knnd::cmp_table_kind(c.cmp);
  c.M = prm.fcr_samples;
  c.max_rounds = prm.max_rounds;

  const size_t esz = c.dtype == KNND_F32 ? 4 : 8;
  const size_t nK = (size_t)n * K;
  const int64_t ntiles = (n + 2047) / 2048;
  c.gstride = next_pow2(2 * n) < 1024 ? 1024 : next_pow2(2 * n);
  // blocks of the global-memory receiver class, each with its own table,
  // candidate list and keys (10 bytes per table slot): as many as 4 GiB
  // holds, between 32 and 128 (more than 32 cut its tail of few, very large
  // receivers; more than 128 gained nothing at 10^6 points)
  c.gblocks = (int)std::min<int64_t>(128, std::max<int64_t>(32, ((int64_t)4 << 30) / (10 * c.gstride)));
  // (fixed scratch: fewer blocks for the two global-memory classes, whose
  // per-block regions would otherwise dominate a small arena)
  if (c.arena) c.gblocks = 16;
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = balloc(c, &c.P, ((size_t)n * c.D + knnd::HUB_MAXD) * esz);
  if (e == hipSuccess) e = dalloc(c, &c.L, (size_t)n * c.Dp + knnd::HUB_MAXD);
  for (int b = 0; b < 2; ++b) {
    if (e == hipSuccess) e = dalloc(c, &c.F[b], (size_t)n * c.Ks);
    if (e == hipSuccess) e = dalloc(c, &c.keys[b], nK);
  }
  if (e == hipSuccess) e = dalloc(c, &c.deg, (size_t)n);
  if (e == hipSuccess) e = dalloc(c, &c.fill, (size_t)n);
  if (e == hipSuccess) e = dalloc(c, &c.rowptr, (size_t)n + 1);
  if (e == hipSuccess) e = dalloc(c, &c.col, nK);
  if (e == hipSuccess) e = dalloc(c, &c.colslot, nK);
  if (e == hipSuccess) e = dalloc(c, &c.tilesum, (size_t)ntiles + 1);
  // bucketed CSR: targets per bucket the smallest power of two >= 256 giving
  // at most CSR_MAXB buckets
  c.csr_shift = 8;
  while (c.csr_shift < 13 && ((n + ((int64_t)1 << c.csr_shift) - 1) >> c.csr_shift) > knnd::CSR_MAXB) ++c.csr_shift;
  if (((n + ((int64_t)1 << c.csr_shift) - 1) >> c.csr_shift) <= knnd::CSR_MAXB && nK < ((size_t)1 << 31) &&
      !(prm.flags & KNND_FLAG_ATOMIC_CSR)) {
    if (e == hipSuccess) e = dalloc(c, &c.csr_T, nK);
    if (e == hipSuccess) e = dalloc(c, &c.csr_bcount, (size_t)knnd::CSR_MAXB);
    if (e == hipSuccess) e = dalloc(c, &c.csr_bfill, (size_t)knnd::CSR_MAXB);
    if (e == hipSuccess) e = dalloc(c, &c.csr_bbase, (size_t)knnd::CSR_MAXB + 1);
  }
  if (e == hipSuccess) e = dalloc(c, &c.class_count, (size_t)knnd::NCLASS);
  if (e == hipSuccess) e = dalloc(c, &c.class_list, (size_t)knnd::NCLASS * n);
  if (e == hipSuccess) e = dalloc(c, &c.gtab, (size_t)c.gblocks * c.gstride);
  if (e == hipSuccess) e = dalloc(c, &c.gcand, (size_t)c.gblocks * (c.gstride / 2));
  if (e == hipSuccess) e = dalloc(c, &c.gckey, (size_t)c.gblocks * (c.gstride / 2));
  // (fixed scratch: one candidate region per CU for the big LDS classes)
  c.bblocks = c.arena ? std::min(c.num_cu, 64) : 4 * c.num_cu;
  if (e == hipSuccess) e = dalloc(c, &c.bcand, (size_t)c.bblocks * knnd::BIG_CAND);
  if (e == hipSuccess) e = dalloc(c, &c.bckey, (size_t)c.bblocks * knnd::BIG_CAND);
  if (e == hipSuccess) e = dalloc(c, &c.dstats, (size_t)knnd::STAT_N);
  if (e == hipSuccess) e = dalloc(c, &c.dflag, (size_t)4);
  if (c.arena) {
    c.hstats = c.hstats_local;
  } else {
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&c.hstats), knnd::STAT_N * sizeof(int64_t));
    if (e == hipSuccess) e = hipEventCreate(&c.ev0);
    if (e == hipSuccess) e = hipEventCreate(&c.ev1);
    if (e == hipSuccess) e = hipEventCreate(&c.evj0);
    if (e == hipSuccess) e = hipEventCreate(&c.evj1);
    if (e == hipSuccess) e = hipEventCreate(&c.evh);
  }
  if (e != hipSuccess) return map_err(e);
  // Hub form: candidate rows of a hub must fit in LDS, and the key slots
  // (K(2Ks+1) per point) must fit in memory; otherwise the pull form.  The
  // mixed-precision form needs the hub form, D <= 64 (MFMA K dimension) and
  // the KL comparator (its error bound is derived for that key).  Buffers of
  // the hub and mixed forms are optional: when they do not fit, the next
  // form runs (same results).
  c.use_hub = !(c.flags & KNND_FLAG_PULL) && (size_t)(K + 1) * c.Ds * sizeof(double) <= 64 * 1024;
  c.mixed = c.use_hub && c.precision != KNND_PREC_FP64 && c.D <= 64 && c.cmp == KNND_CMP_KL;
  if (c.use_hub) {
    const size_t mark = c.arena_used;
    const size_t sl = (size_t)n * knnd::SHORT_LIST;
    bool ok = dalloc(c, &c.sl_n, (size_t)n) == hipSuccess && dalloc(c, &c.sl_id, sl) == hipSuccess;
    if (ok && c.use_hub && c.ck == knnd::CK_REV && c.dtype == KNND_F32)
      ok = dalloc(c, &c.Pw, (size_t)n * c.D + knnd::HUB_MAXD) == hipSuccess;
    if (ok && c.mixed) {
      const size_t mmark = c.arena_used;
      c.dk = c.D <= 32 ? 32 : 64;
      // rows of 2 dk 16-bit values: dk high parts, then dk low parts
      const bool mok = balloc(c, &c.Ph, (size_t)n * c.dk * 4 + 64) == hipSuccess &&
                       balloc(c, &c.Lh, (size_t)n * c.dk * 4 + 64) == hipSuccess &&
                       dalloc(c, &c.S, (size_t)n) == hipSuccess &&
                       dalloc(c, &c.seg32, nK * (size_t)(2 * c.Ks + 1)) == hipSuccess;
      if (!mok) {
        drop_optional(c, mmark, &c.Ph, &c.Lh, &c.S, &c.seg32);
        c.mixed = false;
      }
    }
    // (the automatic mode keeps the exact form's slots too, so that either
    // form can run)
    if (ok && (!c.mixed || c.auto_prec)) {
      const size_t pmark = c.arena_used;
      const bool pok = dalloc(c, &c.seg, nK * (size_t)(2 * c.Ks + 1)) == hipSuccess &&
                       dalloc(c, &c.sl_key, sl) == hipSuccess;
      if (!pok) {
        drop_optional(c, pmark, &c.seg, &c.sl_key);
        ok = c.mixed;  // mixed only
      }
      // (the register hub kernel's rows, for rows of at most 24 coordinates,
      // the kernel's three-wave form; not in fixed-scratch mode)
      if (pok && !c.arena && c.D <= 24) {
        const size_t esz = c.dtype == KNND_F32 ? 4 : 8;
        c.hstride = (int64_t)(((size_t)c.D * (8 + esz) + 127) / 128 * 128);
        const size_t hmark = c.arena_used;
        if (balloc(c, &c.Hrow, (size_t)n * c.hstride + knnd::HUB_MAXD * 16) != hipSuccess) {
          drop_optional(c, hmark, &c.Hrow);
          c.hstride = 0;
        }
      }
    }
    if (!ok) {
      drop_optional(c, mark, &c.sl_n, &c.sl_id, &c.Pw, &c.Ph, &c.Lh, &c.S, &c.seg32, &c.seg, &c.sl_key, &c.Hrow);
      c.hstride = 0;
      c.use_hub = false;
      c.mixed = false;
    }
  }
  c.plain_ok = c.use_hub && c.seg && c.sl_key;
  return KNND_OK;
}

// After the points are in c.P: tail padding, log table with the domain
// check, and the mixed-precision operands.
int finish_create(Ctx& c) {
  const size_t esz = c.dtype == KNND_F32 ? 4 : 8;
  const size_t nK = (size_t)c.n * c.K;
  const size_t pbytes = (size_t)c.n * c.D * esz;
  KNND_HIP(hipMemsetAsync(static_cast<char*>(c.P) + pbytes, 0, knnd::HUB_MAXD * esz, c.stream));
  KNND_HIP(hipMemsetAsync(c.L + (size_t)c.n * c.Dp, 0, knnd::HUB_MAXD * sizeof(double), c.stream));
  KNND_HIP(hipMemsetAsync(c.dflag, 0, sizeof(int32_t), c.stream));
  KNND_HIP(knnd::launch_log_table(c, c.dflag));
  if (c.Pw) KNND_HIP(knnd::launch_widen(c));
  if (c.Hrow) KNND_HIP(knnd::launch_hub_rows(c));
  int32_t bad = 0;
  KNND_HIP(hipMemcpyAsync(&bad, c.dflag, sizeof(int32_t), hipMemcpyDeviceToHost, c.stream));
  KNND_HIP(hipStreamSynchronize(c.stream));
  if (bad) return KNND_ERR_DOMAIN;
  if (c.mixed) return prepare_mixed(c, nK);
  return KNND_OK;
}

int create(const void* points, int64_t n, int32_t d, int32_t K, uint64_t seed, const knnd_params* p,
           int32_t on_device, void* stream, Ctx& c) {
  int st = check_shape(n, d, K);
  if (st != KNND_OK) return st;
  knnd_params prm;
  st = resolve_params(p, n, &prm);
  if (st != KNND_OK) return st;
  st = setup(c, n, d, K, seed, prm, stream);
  if (st != KNND_OK) return st;
  const size_t esz = c.dtype == KNND_F32 ? 4 : 8;
  KNND_HIP(hipMemcpyAsync(c.P, points, (size_t)n * c.D * esz,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c.stream));
  st = finish_create(c);
  // neighbourhood tracking: hub form only (k_merge carries the lists over)
  if (st == KNND_OK) c.track_capable = c.use_hub;
  return st;
}

// Split 16-bit operand copies and the error-bound constants of the mixed
// form.  Each operand v (x_i or log c_i) is v = hi + lo + r with
// |r| <= u^2 |v| + 2s and |lo| <= u(1+u)|v| + 3s, where u bounds the relative
// rounding error of one conversion to the 16-bit format (unit roundoff, plus
// 2^-23 in case the conversion rounds through FP32 first) and s is half the
// smallest 16-bit subnormal spacing, likewise inflated.  Dropping lo*lo and
// the residuals costs at most (3u^2 + 3u^3)|x_i||log c_i| + 3s(|x_i| +
// |log c_i|) + 21 s^2 per coordinate.  The products of 16-bit values are
// exact in FP32; the sum of the 3D nonzero products and the accumulator
// chain is charged (3D + 3) 2^-23 times the sum of their magnitudes
// (directed rounding, any order), plus 2^-126 per term for FP32 underflow.
// With every coordinate <= 1, every product x_i log c_i is <= 0, so the sum
// of magnitudes is |C| itself.  Inputs with a coordinate above 1 or outside
// the 16-bit range disable the mixed form (same results, plain speed).
int prepare_mixed(Ctx& c, size_t nK) {
  unsigned long long* dmax = reinterpret_cast<unsigned long long*>(c.dstats);
  KNND_HIP(knnd::launch_zero_i64(c.dstats, knnd::STAT_N, c.stream));
  KNND_HIP(knnd::launch_prep_mixed(c, dmax));
  unsigned long long hmax[2] = {0, 0};
  KNND_HIP(hipMemcpyAsync(hmax, dmax, sizeof hmax, hipMemcpyDeviceToHost, c.stream));
  KNND_HIP(hipStreamSynchronize(c.stream));
  double pmax, lmax;
  std::memcpy(&pmax, &hmax[0], 8);
  std::memcpy(&lmax, &hmax[1], 8);
  const bool bf16 = c.precision == KNND_PREC_MIXED_BF16;
  const double range = bf16 ? 1e38 : 6.0e4;
  if (!(pmax <= 1.0) || !(lmax <= range)) {
    // fall back to the exact hub form
    c.mixed = false;
    (void)hipStreamSynchronize(c.stream);
    if (!c.arena) knnd::pool_free(c.seg32);  // (an arena keeps the space: the bump pointer only grows)
    c.seg32 = nullptr;
    if (!c.plain_ok) {
      const size_t mark = c.arena_used;
      if (dalloc(c, &c.seg, nK * (size_t)(2 * c.Ks + 1)) != hipSuccess ||
          dalloc(c, &c.sl_key, (size_t)c.n * knnd::SHORT_LIST) != hipSuccess) {
        drop_optional(c, mark, &c.seg, &c.sl_key);
        c.use_hub = false;  // pull form: needs neither
      }
      c.plain_ok = c.use_hub;
    }
    return KNND_OK;
  }
  c.mixed_ok = true;
  const double u = (bf16 ? 0x1p-8 : 0x1p-11) + 0x1p-23;
  const double s = bf16 ? 0x1p-133 : 0x1p-24;
  const double m = 3.0 * c.D + 3.0;         // FP32 rounding steps
  const double g = m * 0x1p-23 * 1.0001;    // (1 + 2^-23)^m - 1
  const double grow = std::pow(1 + u, 5);  // sum of |hi*hi|, |hi*lo|, |lo*hi| over |x log c|
  const double opabs = c.D * (3 * s * (pmax + lmax) + 21 * s * s);
  const double e_rel = 3 * u * u + 3 * u * u * u + g * grow;
  c.eps_relq = e_rel / (1 - e_rel) * (1 + 0x1p-50);
  c.eps_abs = opabs * (1 + g) + g * 6 * c.D * s * (pmax + lmax) + 3 * c.D * 0x1p-126;
  return KNND_OK;
}

int read_stats(Ctx& c, knnd_round_stats* st, bool joined) {
  KNND_HIP(hipMemcpyAsync(c.hstats, c.dstats, knnd::STAT_N * sizeof(int64_t), hipMemcpyDeviceToHost, c.stream));
  KNND_HIP(hipStreamSynchronize(c.stream));
  float ms = 0.f, msj = 0.f, msh = 0.f, msr = 0.f;
  if (c.ev0) KNND_HIP(hipEventElapsedTime(&ms, c.ev0, c.ev1));
  if (joined && c.ev0) {
    KNND_HIP(hipEventElapsedTime(&msj, c.evj0, c.evj1));
    KNND_HIP(hipEventElapsedTime(&msh, c.evj0, c.evh));
    KNND_HIP(hipEventElapsedTime(&msr, c.evh, c.evj1));
  }
  if (st) {
    st->updates = c.hstats[knnd::STAT_UPDATES];
    st->fcr_hits = c.hstats[knnd::STAT_HITS];
    st->evals_alg = c.hstats[knnd::STAT_EVALS];
    st->evals_performed = c.hstats[knnd::STAT_PERF];
    st->rescues = c.hstats[knnd::STAT_RESCUES];
    st->carried = c.hstats[knnd::STAT_CARRIED];
    st->evals_carried = c.hstats[knnd::STAT_EVCARRY];
    st->ms = ms;
    st->ms_join = msj;
    st->ms_hub = msh;
    st->ms_recv = msr;
  }
  // an internal consistency check failed on the device (results are unusable)
  if (c.hstats[knnd::STAT_ERR] != 0) return KNND_ERR_DEVICE;
  return KNND_OK;
}

int init_graph(Ctx& c, knnd_round_stats* st) {
  KNND_HIP(knnd::launch_zero_i64(c.dstats, knnd::STAT_N, c.stream));
  KNND_HIP(rec(c.ev0, c.stream));
  KNND_HIP(knnd::launch_init_graph(c));
  KNND_HIP(knnd::launch_fcr(c, c.F[c.cur], 0, c.dstats + knnd::STAT_HITS));
  KNND_HIP(rec(c.ev1, c.stream));
  c.round = 0;
  c.have_graph = true;
  c.track_ok = false;
  return read_stats(c, st, false);
}

// ---------------------------------------------------------------------------
// Autotuner of the join's schedule.  Candidates: the exact hub form with the
// register-staged hub kernel (k_hub_reg, one hub per wave; for small K also
// two or four hubs per wave, k_hub_reg_sub) or the LDS-staged one
// (k_hub_lds), and, under KNND_PREC_AUTO, the BF16 mixed form; then, with
// the fastest of those, the smallest receiver classes one wave per receiver
// (k_recv_wave) for none, one or two classes; then receivers of the
// 8192-slot class whose distinct candidates probably fit a 4096-slot table
// there, guarded (an overflowing receiver is redone in the 8192-slot class).  Every candidate computes
// the same lists, keys and counts, so a choice changes only speed: the join
// of the coming round (binning, hub kernel, receiver pass) is run once per
// candidate from the round-start snapshot, timed with HIP events, and the
// fastest is kept; the round then runs in full with it.  Choices are cached
// by workload shape (K, coordinates, size class, single or batched,
// comparator, precision mode) for the rest of the process and, when
// KNND_TUNE_CACHE names a file, in that file: one line per shape,
// "<shape> | <mixed> <hub_lds> <hubs per wave> <wave receivers> <guarded
// 4096> | <ms of each candidate>".
// ---------------------------------------------------------------------------
struct Sched {
  bool mixed;
  bool hub_lds;
  int hpw;    // hubs per wave of the register hub kernel
  int rwave;  // smallest receiver classes one wave per receiver (0, 1 or 2 classes)
  int opt;    // guarded 4096-slot tables for receivers of the 8192-slot class that probably fit
};

std::mutex g_tune_mu;
std::map<std::string, Sched> g_tune;
bool g_tune_loaded = false;

void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("KNND_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    const char* bar = std::strchr(line, '|');
    int m = 0, h = 0, w = 1, rw = 0, op = 0;
    if (!bar || std::sscanf(bar + 1, "%d %d %d %d %d", &m, &h, &w, &rw, &op) != 5 ||
        (w != 1 && w != 2 && w != 4) || rw < 0 || rw > 2)
      continue;
    std::string key(line, (size_t)(bar - line));
    while (!key.empty() && key.back() == ' ') key.pop_back();
    g_tune[key] = Sched{m != 0, h != 0, w, rw, op != 0 ? 1 : 0};
  }
  std::fclose(f);
}

std::string tune_key(const Ctx& c, bool group) {
  int lg = 0;
  while (((int64_t)1 << lg) < c.n) ++lg;
  char buf[160];
  std::snprintf(buf, sizeof buf, "gfx950 K=%d D=%d log2n=%d batched=%d cmp=%d prec=%d", c.K, c.D, lg, group ? 1 : 0,
                c.cmp, c.auto_prec ? (int)KNND_PREC_AUTO : c.precision);
  return buf;
}

void apply_sched(Ctx& c, Sched s) {
  c.mixed = s.mixed;
  c.hub_lds = s.hub_lds;
  c.hub_hpw = s.hpw;
  c.recv_wave = s.rwave;
  c.opt4096 = s.opt != 0;
}

const char* sched_name(const Sched& s, char* buf, size_t len) {
  std::snprintf(buf, len, "%s%s%s%s", s.mixed ? "mixed" : "exact",
                s.hub_lds ? "/lds" : (s.hpw == 4 ? "/hpw4" : (s.hpw == 2 ? "/hpw2" : "")),
                s.rwave == 2 ? "/wave2" : (s.rwave == 1 ? "/wave1" : ""), s.opt ? "/opt4096" : "");
  return buf;
}

// Choose the join's schedule for context c; its reverse-neighbour lists for
// the coming round must be built.  group: a batched group (its per-instance
// and per-point counters are cleared between trials too).
int tune_join(Ctx& c, bool group) {
  // stage 1: the form and the hub kernel; stage 2: the smallest receiver
  // classes one wave per receiver or not (exact form), with the stage-1
  // choice (the guarded 4096-slot tables are tried on the second round,
  // tune_opt: on the first every distinct candidate is listed)
  Sched cand[8];
  int nc = 0;
  const bool lds_fits = (size_t)(c.K + 1) * c.Ds * sizeof(double) <= 64 * 1024;
  if (c.plain_ok && (c.auto_prec || !c.mixed)) {
    cand[nc++] = Sched{false, false, 1, 0, 0};
    if (c.D <= 24 && c.K <= 32) cand[nc++] = Sched{false, false, 2, 0, 0};  // (the register kernel's row bound)
    if (c.D <= 24 && c.K <= 16) cand[nc++] = Sched{false, false, 4, 0, 0};
    if (lds_fits) cand[nc++] = Sched{false, true, 1, 0, 0};
  }
  if (c.mixed_ok && (c.auto_prec || c.mixed)) cand[nc++] = Sched{true, false, 1, 0, 0};
  if (nc == 0 || !c.evj0) return KNND_OK;
  const bool waves = c.use_hub && c.K < 64;  // (stage 2 applies, to the exact form)
  // KNND_TUNE_FORCE="<mixed> <hub_lds> <hubs per wave> <wave receivers>
  // <guarded 4096>" fixes the schedule when it is a candidate (no trials,
  // nothing cached)
  if (const char* force = std::getenv("KNND_TUNE_FORCE")) {
    int m = 0, h = 0, w = 1, rw = 0, op = 0;
    if (std::sscanf(force, "%d %d %d %d %d", &m, &h, &w, &rw, &op) == 5 && rw >= 0 && rw <= 2 &&
        (rw == 0 || (waves && m == 0)))
      for (int i = 0; i < nc; ++i)
        if (cand[i].mixed == (m != 0) && cand[i].hub_lds == (h != 0) && cand[i].hpw == w) {
          Sched f = cand[i];
          f.rwave = rw;
          f.opt = op != 0 ? 1 : 0;
          apply_sched(c, f);
          return KNND_OK;
        }
  }
  const std::string key = tune_key(c, group);
  // A cached choice applies when it is one of this context's candidates: a
  // context whose optional buffers did not all fit (so that a form is
  // missing) chooses among the forms it has, and its choice is not cached.
  bool cacheable = true;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      const Sched& h = it->second;
      for (int i = 0; i < nc; ++i)
        if (cand[i].mixed == h.mixed && cand[i].hub_lds == h.hub_lds && cand[i].hpw == h.hpw &&
            (h.rwave == 0 || (waves && !h.mixed))) {
          apply_sched(c, h);
          return KNND_OK;
        }
      cacheable = false;
    }
  }
  float ms[10] = {};
  Sched tried[10];
  int nt = 0;
  auto trial = [&](Sched sc, float* out) -> int {
    apply_sched(c, sc);
    KNND_HIP(knnd::launch_zero_i64(c.dstats, knnd::STAT_N, c.stream));
    if (group) {
      KNND_HIP(knnd::launch_zero_i64(c.istats, (int64_t)c.nb * knnd::STAT_N, c.stream));
      KNND_HIP(knnd::launch_zero_i32(c.vcnt, c.n * knnd::VC_N, c.stream));
    }
    KNND_HIP(knnd::launch_bin(c, false));
    KNND_HIP(hipEventRecord(c.evj0, c.stream));
    KNND_HIP(knnd::launch_join_hub(c, c.dstats));
    KNND_HIP(knnd::launch_join_recv(c, c.dstats));
    KNND_HIP(hipEventRecord(c.evj1, c.stream));
    KNND_HIP(hipStreamSynchronize(c.stream));
    KNND_HIP(hipEventElapsedTime(out, c.evj0, c.evj1));
    return KNND_OK;
  };
  int best = 0;
  for (int i = 0; i < nc; ++i) {
    tried[nt] = cand[i];
    const int st = trial(cand[i], &ms[nt]);
    if (st != KNND_OK) return st;
    if (ms[nt] < ms[best]) best = nt;
    ++nt;
  }
  if (waves && !tried[best].mixed)
    for (int rw = 1; rw <= 2; ++rw) {
      Sched sc = tried[best];
      sc.rwave = rw;
      tried[nt] = sc;
      const int st = trial(sc, &ms[nt]);
      if (st != KNND_OK) return st;
      if (ms[nt] < ms[best]) best = nt;
      ++nt;
    }
  apply_sched(c, tried[best]);
  if (!cacheable) return KNND_OK;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = tried[best];
  const char* path = std::getenv("KNND_TUNE_CACHE");
  if (path && *path) {
    if (FILE* f = std::fopen(path, "a")) {
      const Sched& b = tried[best];
      std::fprintf(f, "%s | %d %d %d %d %d |", key.c_str(), b.mixed ? 1 : 0, b.hub_lds ? 1 : 0, b.hpw, b.rwave,
                   b.opt);
      char nm[48];
      for (int i = 0; i < nt; ++i) std::fprintf(f, " %s:%.3f", sched_name(tried[i], nm, sizeof nm), ms[i]);
      std::fprintf(f, "\n");
      std::fclose(f);
    }
  }
  return KNND_OK;
}

// The second tuning point: on the second round (most lists are short from
// there on) time the join with and without guarded 4096-slot tables for the
// receivers of the 8192-slot class that probably fit, and keep the faster.
// Cached per shape like tune_join's choice.
int tune_opt(Ctx& c, bool group) {
  if (!c.use_hub || !c.evj0) return KNND_OK;
  if (const char* force = std::getenv("KNND_TUNE_FORCE")) {
    int m = 0, h = 0, w = 1, rw = 0, op = 0;
    if (std::sscanf(force, "%d %d %d %d %d", &m, &h, &w, &rw, &op) == 5) {
      c.opt4096 = op != 0;
      return KNND_OK;
    }
  }
  const std::string key = tune_key(c, group) + " round=2";
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      c.opt4096 = it->second.opt != 0;
      return KNND_OK;
    }
  }
  float ms[2] = {0.f, 0.f};
  for (int o = 0; o < 2; ++o) {
    c.opt4096 = o != 0;
    KNND_HIP(knnd::launch_zero_i64(c.dstats, knnd::STAT_N, c.stream));
    if (group) {
      KNND_HIP(knnd::launch_zero_i64(c.istats, (int64_t)c.nb * knnd::STAT_N, c.stream));
      KNND_HIP(knnd::launch_zero_i32(c.vcnt, c.n * knnd::VC_N, c.stream));
    }
    KNND_HIP(knnd::launch_bin(c, false));
    KNND_HIP(hipEventRecord(c.evj0, c.stream));
    KNND_HIP(knnd::launch_join_hub(c, c.dstats));
    KNND_HIP(knnd::launch_join_recv(c, c.dstats));
    KNND_HIP(hipEventRecord(c.evj1, c.stream));
    KNND_HIP(hipStreamSynchronize(c.stream));
    KNND_HIP(hipEventElapsedTime(&ms[o], c.evj0, c.evj1));
  }
  c.opt4096 = ms[1] < ms[0];
  Sched rec = Sched{c.mixed, c.hub_lds, c.hub_hpw, c.recv_wave, c.opt4096 ? 1 : 0};
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = rec;
  const char* path = std::getenv("KNND_TUNE_CACHE");
  if (path && *path) {
    if (FILE* f = std::fopen(path, "a")) {
      char nm[48];
      rec.opt = 0;
      std::fprintf(f, "%s | %d %d %d %d %d | %s:%.3f", key.c_str(), c.mixed ? 1 : 0, c.hub_lds ? 1 : 0, c.hub_hpw,
                   c.recv_wave, c.opt4096 ? 1 : 0, sched_name(rec, nm, sizeof nm), ms[0]);
      rec.opt = 1;
      std::fprintf(f, " %s:%.3f\n", sched_name(rec, nm, sizeof nm), ms[1]);
      std::fclose(f);
    }
  }
  return KNND_OK;
}

int run_round(Ctx& c, knnd_round_stats* st) {
  if (!c.have_graph) return KNND_ERR_ARG;
  KNND_HIP(knnd::launch_zero_i64(c.dstats, knnd::STAT_N, c.stream));
  KNND_HIP(rec(c.ev0, c.stream));
  KNND_HIP(knnd::launch_csr(c, c.F[c.cur]));
  if (c.tune && c.own0 == 0 && c.own1 == c.n && (!c.tuned || (c.round == 1 && !c.tuned2))) {
    // (the first and second rounds' times include the trials)
    const int t = c.tuned ? tune_opt(c, false) : tune_join(c, false);
    if (c.tuned) c.tuned2 = true;
    c.tuned = true;
    if (t != KNND_OK) return t;
    KNND_HIP(knnd::launch_zero_i64(c.dstats, knnd::STAT_N, c.stream));
  }
  // receivers whose neighbourhood did not change keep their list and count.
  // A changed list touches about 2K neighbourhoods, so few are unchanged
  // until few lists change: the flags are gathered once the last round
  // changed at most 0.2% of the entries and used once it changed at most
  // 0.1%; using them needs the last round's flags of every receiver and the
  // pair skipping in force
  const bool full = c.own0 == 0 && c.own1 == c.n;
  const int64_t nK = c.n * (int64_t)c.K;
  const bool want = c.track_capable && full && c.last_updates >= 0 && c.last_updates * 500 <= nK;
  if (want && !c.vchg) {  // first use: 24 bytes per point
    const size_t mark = c.arena_used;
    if (dalloc(c, &c.vchg, (size_t)c.n) != hipSuccess || dalloc(c, &c.vev, (size_t)c.n * knnd::VC_N) != hipSuccess) {
      drop_optional(c, mark, &c.vchg, &c.vev);  // no tracking then: every receiver is evaluated, as without it
      c.track_capable = false;
    } else if (knnd::launch_zero_i32(c.vchg, c.n, c.stream) != hipSuccess) {
      (void)hipGetLastError();
      c.track_capable = false;
    }
  }
  c.tracking = want && c.track_capable && c.vchg && c.vev;
  const bool carry = c.tracking && c.track_ok && !c.no_skip_next &&
                     !(c.flags & (KNND_FLAG_NO_SKIP | KNND_FLAG_NO_CARRY)) && c.last_updates * 1000 <= nK;
  KNND_HIP(knnd::launch_bin(c, carry));
  KNND_HIP(rec(c.evj0, c.stream));
  KNND_HIP(knnd::launch_join_hub(c, c.dstats));
  KNND_HIP(rec(c.evh, c.stream));
  KNND_HIP(knnd::launch_join_recv(c, c.dstats));
  KNND_HIP(rec(c.evj1, c.stream));
  if (c.tracking) KNND_HIP(knnd::launch_track(c));
  // (a restricted round copies its receivers' lists back over the
  // round-start ones instead of carrying every other list over)
  if (!full) KNND_HIP(knnd::launch_put_rows(c));
  KNND_HIP(knnd::launch_fcr(c, c.F[full ? c.cur ^ 1 : c.cur], c.round + 1, c.dstats + knnd::STAT_HITS));
  KNND_HIP(rec(c.ev1, c.stream));
  if (full) c.cur ^= 1;
  c.round += 1;
  c.no_skip_next = !full;
  c.track_ok = c.tracking;
  c.tracking = false;
  const int r = read_stats(c, st, true);
  c.last_updates = r == KNND_OK ? c.hstats[knnd::STAT_UPDATES] : -1;
  return r;
}

// One round in which only the receivers [first, first + count) get new lists.
int run_round_share(Ctx& c, int64_t first, int64_t count, knnd_round_stats* st) {
  if (!c.have_graph || first < 0 || count < 1 || first > c.n - count) return KNND_ERR_ARG;
  c.own0 = first;
  c.own1 = first + count;
  const int r = run_round(c, st);
  c.own0 = 0;
  c.own1 = c.n;
  return r;
}

int get_graph(Ctx& c, int32_t* idx, double* kl, int32_t on_device) {
  const size_t nK = (size_t)c.n * c.K;
  if (on_device) {
    KNND_HIP(knnd::launch_strip(c, c.F[c.cur], idx));
    if (kl) KNND_HIP(hipMemcpyAsync(kl, c.keys[c.cur], nK * 8, hipMemcpyDeviceToDevice, c.stream));
  } else {
    // strip into the idle half of the double buffer, then copy out
    int32_t* staging = reinterpret_cast<int32_t*>(c.F[c.cur ^ 1]);
    KNND_HIP(knnd::launch_strip(c, c.F[c.cur], staging));
    KNND_HIP(hipMemcpyAsync(idx, staging, nK * 4, hipMemcpyDeviceToHost, c.stream));
    if (kl) KNND_HIP(hipMemcpyAsync(kl, c.keys[c.cur], nK * 8, hipMemcpyDeviceToHost, c.stream));
  }
  KNND_HIP(hipStreamSynchronize(c.stream));
  return KNND_OK;
}

// Stop test after round r of an instance with n points (Section 1.2, Table 1,
// and Section 1.3, item (b)); *capped tells whether only the round cap stopped it.
bool should_stop(const knnd_params& p, int64_t n, int K, int64_t hits_prev, int64_t hits, int64_t updates,
                 int r, bool* capped) {
  bool rule;
  if (p.stop_rule == KNND_STOP_FIXED_POINT)
    rule = updates == 0;
  else if (p.stop_rule == KNND_STOP_DELTA)
    rule = (double)updates <= p.delta * (double)n * (double)K;
  else
    rule = hits <= hits_prev || updates == 0;
  *capped = !rule && r >= p.max_rounds;
  return rule || r >= p.max_rounds;
}

// ---------------------------------------------------------------------------
// Batched instances.  Instances with the same K and a similar number of
// coordinates form a group: one context whose points are the instances'
// points one after the other, zero-padded to the group's largest d+1 (a
// padded coordinate has log entry 0 and adds exactly nothing to any key).
// Every list stays inside its instance, so a round of the group is a round of
// each instance still running.  The stop test is taken per instance; a
// stopped instance's lists are copied out and it is left out of later rounds
// (its hubs and receivers are skipped).
// ---------------------------------------------------------------------------
int coord_bucket(int D) {
  static const int b[] = {8, 12, 16, 24, 32, 40, 52, 64};
  for (int v : b)
    if (D <= v) return v;
  return (D + 15) / 16 * 16;
}

struct Group {
  Ctx c;
  std::vector<int> members;     // indices into the caller's instance array
  std::vector<int64_t> off;     // [nb+1] first point of each member
  std::vector<int32_t> active;  // host copy of c.iactive
  std::vector<int64_t> hits_prev;
  int32_t* staging = nullptr;   // device [max n_b][K]: host-bound lists
  bool dirty = false;           // active flags changed since the last upload
  int running = 0;
};

void free_group(Group& g) {
  (void)hipStreamSynchronize(g.c.stream);
  knnd::pool_free(g.staging);
  g.staging = nullptr;
  free_ctx(g.c);
}

int create_group(Group& g, const knnd_instance* inst, const knnd_params& prm, int32_t on_device, void* stream) {
  Ctx& c = g.c;
  const int nb = (int)g.members.size();
  const knnd_instance& first = inst[g.members[0]];
  int64_t N = 0, nmax = 0;
  int Dmax = 0;
  g.off.assign(nb + 1, 0);
  for (int j = 0; j < nb; ++j) {
    const knnd_instance& in = inst[g.members[j]];
    g.off[j] = N;
    N += in.n;
    nmax = std::max(nmax, in.n);
    Dmax = std::max(Dmax, in.d + 1);
  }
  g.off[nb] = N;
  if (N >= (int64_t)knnd::IDMASK_HOST) return KNND_ERR_ARG;
  int st = setup(c, N, Dmax - 1, first.K, 0, prm, stream);
  if (st != KNND_OK) return st;
  c.nb = nb;
  c.tune = !(prm.flags & KNND_FLAG_NO_TUNE);
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = dalloc(c, &c.inst_of, (size_t)N);
  if (e == hipSuccess) e = dalloc(c, &c.ioff, (size_t)nb + 1);
  if (e == hipSuccess) e = dalloc(c, &c.iseed, (size_t)nb);
  if (e == hipSuccess) e = dalloc(c, &c.iM, (size_t)nb);
  if (e == hipSuccess) e = dalloc(c, &c.iD, (size_t)nb);
  if (e == hipSuccess) e = dalloc(c, &c.iactive, (size_t)nb);
  if (e == hipSuccess) e = dalloc(c, &c.istats, (size_t)nb * knnd::STAT_N);
  if (e == hipSuccess) e = dalloc(c, &c.vcnt, (size_t)N * knnd::VC_N);
  if (e == hipSuccess && !on_device) e = dalloc(c, &g.staging, (size_t)nmax * c.K);
  if (e != hipSuccess) return map_err(e);

  std::vector<int32_t> inst_of((size_t)N), iD(nb), act(nb, 1);
  std::vector<uint64_t> iseed(nb);
  std::vector<int64_t> iM(nb);
  for (int j = 0; j < nb; ++j) {
    const knnd_instance& in = inst[g.members[j]];
    std::fill(inst_of.begin() + g.off[j], inst_of.begin() + g.off[j + 1], j);
    iD[j] = in.d + 1;
    iseed[j] = in.seed;
    iM[j] = prm.fcr_samples > 0 ? prm.fcr_samples : std::min<int64_t>(in.n, 10000);
    c.Mmax = std::max(c.Mmax, iM[j]);
  }
  KNND_HIP(hipMemcpy(c.inst_of, inst_of.data(), (size_t)N * 4, hipMemcpyHostToDevice));
  KNND_HIP(hipMemcpy(c.ioff, g.off.data(), ((size_t)nb + 1) * 8, hipMemcpyHostToDevice));
  KNND_HIP(hipMemcpy(c.iseed, iseed.data(), (size_t)nb * 8, hipMemcpyHostToDevice));
  KNND_HIP(hipMemcpy(c.iM, iM.data(), (size_t)nb * 8, hipMemcpyHostToDevice));
  KNND_HIP(hipMemcpy(c.iD, iD.data(), (size_t)nb * 4, hipMemcpyHostToDevice));
  KNND_HIP(hipMemcpy(c.iactive, act.data(), (size_t)nb * 4, hipMemcpyHostToDevice));
  g.active = act;
  g.hits_prev.assign(nb, 0);
  g.running = nb;

  // points, zero-padded to Dmax coordinates; host points go through a
  // contiguous device staging copy first (a strided copy straight from
  // pageable host memory would move one row at a time)
  const size_t esz = c.dtype == KNND_F32 ? 4 : 8;
  KNND_HIP(hipMemsetAsync(c.P, 0, (size_t)N * c.D * esz, c.stream));
  void* stage = nullptr;
  if (!on_device) {
    size_t most = 0;
    for (int j = 0; j < nb; ++j) most = std::max(most, (size_t)inst[g.members[j]].n * (inst[g.members[j]].d + 1));
    KNND_HIP(knnd::pool_malloc(&stage, most * esz));
  }
  int rc = KNND_OK;
  for (int j = 0; j < nb && rc == KNND_OK; ++j) {
    const knnd_instance& in = inst[g.members[j]];
    const size_t w = (size_t)(in.d + 1) * esz;
    const void* src = in.points;
    hipError_t e2 = hipSuccess;
    if (!on_device) {
      e2 = hipMemcpyAsync(stage, in.points, w * in.n, hipMemcpyHostToDevice, c.stream);
      src = stage;
    }
    if (e2 == hipSuccess)
      e2 = hipMemcpy2DAsync(static_cast<char*>(c.P) + (size_t)g.off[j] * c.D * esz, (size_t)c.D * esz, src, w, w,
                            (size_t)in.n, hipMemcpyDeviceToDevice, c.stream);
    if (e2 != hipSuccess) rc = map_err(e2);
  }
  if (stage) {
    const hipError_t e3 = hipStreamSynchronize(c.stream);
    knnd::pool_free(stage);
    if (rc == KNND_OK && e3 != hipSuccess) rc = map_err(e3);
  }
  if (rc != KNND_OK) return rc;
  return finish_create(c);
}

// Per-call state of a batched call.  Every group's counters of a round land
// in one device array, copied to the host once per round.  Rounds after the
// second are replayed from two captured graphs (one per parity of the
// double-buffered lists) holding the kernels of every running group; the
// round index the FCR sample hashes is read from the device and advanced by
// the graph's last kernel.  A graph is captured again only when a whole
// group has stopped (a stopped instance inside a running group is skipped by
// the kernels through its device flag).
struct Batch {
  std::vector<Group> groups;
  std::vector<int64_t> slot;   // first row of each group's instances in dall
  int64_t sum_nb = 0;          // rows of instance counters; the group rows follow
  int64_t* dall = nullptr;     // device [sum_nb + groups][STAT_N]
  int64_t* hall = nullptr;     // pinned host copy
  int64_t* dround = nullptr;   // device round index of graph-launched rounds
  hipStream_t cs = nullptr;    // capture stream
  // branch streams of the captured round (each running group's kernels form
  // a branch of their own, forked from and joined into the capture stream)
  std::vector<hipStream_t> bs;
  std::vector<hipEvent_t> bev;  // their join events
  hipEvent_t fork = nullptr;
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  std::vector<char> captured;  // running groups the graphs hold
  hipEvent_t e0 = nullptr, e1 = nullptr;
};

void drop_graphs(Batch& bt) {
  for (int p = 0; p < 2; ++p) {
    if (bt.exec[p]) (void)hipGraphExecDestroy(bt.exec[p]);
    if (bt.graph[p]) (void)hipGraphDestroy(bt.graph[p]);
    bt.exec[p] = nullptr;
    bt.graph[p] = nullptr;
  }
  bt.captured.clear();
}

// Enqueue round r (r = 0: the start graph and its FCR) of group gi on its
// stream, and the copy of its counters into dall.  round_dev: the device
// round index for the FCR sample (graph-launched rounds), else r.
int enqueue_group_round(Batch& bt, size_t gi, int r, const int64_t* round_dev) {
  Group& g = bt.groups[gi];
  Ctx& c = g.c;
  KNND_HIP(knnd::launch_zero_i64(c.istats, (int64_t)c.nb * knnd::STAT_N, c.stream));
  KNND_HIP(knnd::launch_zero_i64(c.dstats, knnd::STAT_N, c.stream));
  if (r == 0) {
    KNND_HIP(knnd::launch_init_graph(c));
    KNND_HIP(knnd::launch_fcr(c, c.F[c.cur], 0, nullptr));
  } else {
    KNND_HIP(knnd::launch_zero_i32(c.vcnt, c.n * knnd::VC_N, c.stream));
    KNND_HIP(knnd::launch_csr(c, c.F[c.cur]));
    KNND_HIP(knnd::launch_bin(c, false));
    KNND_HIP(knnd::launch_join_hub(c, c.dstats));
    KNND_HIP(knnd::launch_join_recv(c, c.dstats));
    KNND_HIP(knnd::launch_fcr(c, c.F[c.cur ^ 1], r, nullptr, round_dev));
    KNND_HIP(knnd::launch_batch_reduce(c));
  }
  KNND_HIP(knnd::launch_copy_i64(bt.dall + bt.slot[gi] * knnd::STAT_N, c.istats, (int64_t)c.nb * knnd::STAT_N,
                                 c.stream));
  KNND_HIP(knnd::launch_copy_i64(bt.dall + (bt.sum_nb + (int64_t)gi) * knnd::STAT_N, c.dstats, knnd::STAT_N,
                                 c.stream));
  return KNND_OK;
}

// The branch streams (one per group, at most 16) and their events.
int make_branches(Batch& bt) {
  if (!bt.fork) KNND_HIP(hipEventCreateWithFlags(&bt.fork, hipEventDisableTiming));
  const size_t nbr = std::min<size_t>(bt.groups.size(), 16);
  while (bt.bs.size() < nbr) {
    hipStream_t s = nullptr;
    hipEvent_t e = nullptr;
    KNND_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));  // (default priority)
    bt.bs.push_back(s);
    KNND_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    bt.bev.push_back(e);
  }
  return KNND_OK;
}

// Capture the round of every running group, for both parities.  On failure
// the call goes on with rounds enqueued one by one.
int capture_graphs(Batch& bt) {
  drop_graphs(bt);
  if (!bt.cs) KNND_HIP(hipStreamCreateWithFlags(&bt.cs, hipStreamNonBlocking));
  if (make_branches(bt) != KNND_OK) return KNND_ERR_DEVICE;
  const size_t nbr = bt.bs.size();
  for (int p = 0; p < 2; ++p) {
    std::vector<std::pair<hipStream_t, int>> saved;
    for (Group& g : bt.groups) {
      saved.emplace_back(g.c.stream, g.c.cur);
      g.c.stream = bt.cs;
      g.c.cur = p;
    }
    int st = KNND_OK;
    if (hipStreamBeginCapture(bt.cs, hipStreamCaptureModeRelaxed) != hipSuccess) st = KNND_ERR_DEVICE;
    if (st == KNND_OK && hipEventRecord(bt.fork, bt.cs) != hipSuccess) st = KNND_ERR_DEVICE;
    size_t used = 0;  // branch streams in use
    for (size_t gi = 0; gi < bt.groups.size() && st == KNND_OK; ++gi) {
      if (bt.groups[gi].running == 0) continue;
      hipStream_t s = bt.bs[used % nbr];
      if (used < nbr && hipStreamWaitEvent(s, bt.fork, 0) != hipSuccess) st = KNND_ERR_DEVICE;
      bt.groups[gi].c.stream = s;
      if (st == KNND_OK) st = enqueue_group_round(bt, gi, 1, bt.dround);
      ++used;
    }
    for (size_t i = 0; i < std::min(used, nbr); ++i)  // (joined on failure too, before the capture ends)
      if (hipEventRecord(bt.bev[i], bt.bs[i]) != hipSuccess || hipStreamWaitEvent(bt.cs, bt.bev[i], 0) != hipSuccess)
        st = KNND_ERR_DEVICE;
    if (st == KNND_OK && knnd::launch_add_i64(bt.dround, 1, bt.cs) != hipSuccess) st = KNND_ERR_DEVICE;
    hipGraph_t gr = nullptr;
    const hipError_t ee = hipStreamEndCapture(bt.cs, &gr);  // (ends a capture that failed midway too)
    bt.graph[p] = gr;
    for (size_t gi = 0; gi < bt.groups.size(); ++gi) {
      bt.groups[gi].c.stream = saved[gi].first;
      bt.groups[gi].c.cur = saved[gi].second;
    }
    if (st == KNND_OK && (ee != hipSuccess || !gr)) st = KNND_ERR_DEVICE;
    if (st == KNND_OK && hipGraphInstantiate(&bt.exec[p], gr, nullptr, nullptr, 0) != hipSuccess) st = KNND_ERR_DEVICE;
    if (st != KNND_OK) {
      (void)hipGetLastError();
      drop_graphs(bt);
      return st;
    }
  }
  bt.captured.clear();
  for (const Group& g : bt.groups) bt.captured.push_back(g.running > 0);
  return KNND_OK;
}

// Copy member j's current lists (and keys) to its outputs.
int group_emit(Group& g, int j, const knnd_instance& in, int32_t on_device) {
  Ctx& c = g.c;
  const int64_t off = g.off[j], cnt = in.n * (int64_t)c.K;
  const double* kl = c.keys[c.cur] + off * c.K;
  if (on_device) {
    KNND_HIP(knnd::launch_emit(c, off, in.n, in.out_idx));
    if (in.out_kl) KNND_HIP(hipMemcpyAsync(in.out_kl, kl, cnt * 8, hipMemcpyDeviceToDevice, c.stream));
  } else {
    KNND_HIP(knnd::launch_emit(c, off, in.n, g.staging));
    KNND_HIP(hipMemcpyAsync(in.out_idx, g.staging, cnt * 4, hipMemcpyDeviceToHost, c.stream));
    if (in.out_kl) KNND_HIP(hipMemcpyAsync(in.out_kl, kl, cnt * 8, hipMemcpyDeviceToHost, c.stream));
  }
  return KNND_OK;
}

int build_batched(knnd_instance* inst, int32_t B, const knnd_params* p, int32_t on_device, void* stream) {
  if (!inst || B < 1) return KNND_ERR_ARG;
  knnd_params prm;
  int st = resolve_params(p, 0, &prm);  // fcr_samples stays 0: per instance min(n, 10000)
  if (st != KNND_OK) return st;
  std::map<std::pair<int, int>, std::vector<int>> by_shape;
  for (int b = 0; b < B; ++b) {
    const knnd_instance& in = inst[b];
    if (!in.points || !in.out_idx || !in.out_rounds) return KNND_ERR_ARG;
    st = check_shape(in.n, in.d, in.K);
    if (st != KNND_OK) return st;
    by_shape[{in.K, coord_bucket(in.d + 1)}].push_back(b);
  }
  hipStream_t strm = reinterpret_cast<hipStream_t>(stream);
  Batch bt;
  std::vector<Group>& groups = bt.groups;
  groups.resize(by_shape.size());
  size_t gi = 0;
  for (auto& kv : by_shape) {
    groups[gi].members = kv.second;
    bt.slot.push_back(bt.sum_nb);
    bt.sum_nb += (int64_t)kv.second.size();
    ++gi;
  }
  int worst = KNND_OK;
  auto fail = [&](int s) {
    (void)hipStreamSynchronize(strm);
    drop_graphs(bt);
    if (bt.cs) (void)hipStreamDestroy(bt.cs);
    for (hipStream_t s : bt.bs) (void)hipStreamDestroy(s);
    for (hipEvent_t e : bt.bev) (void)hipEventDestroy(e);
    if (bt.fork) (void)hipEventDestroy(bt.fork);
    bt.bs.clear();
    bt.bev.clear();
    bt.fork = nullptr;
    for (Group& g : groups) free_group(g);
    knnd::pool_free(bt.dall);
    knnd::pool_free(bt.dround);
    if (bt.hall) (void)hipHostFree(bt.hall);
    if (bt.e0) (void)hipEventDestroy(bt.e0);
    if (bt.e1) (void)hipEventDestroy(bt.e1);
    return s;
  };
  const size_t rows = (size_t)bt.sum_nb + groups.size();
  if (knnd::pmalloc(&bt.dall, rows * knnd::STAT_N * sizeof(int64_t)) != hipSuccess ||
      knnd::pmalloc(&bt.dround, 64) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&bt.hall), rows * knnd::STAT_N * sizeof(int64_t)) != hipSuccess ||
      hipEventCreate(&bt.e0) != hipSuccess || hipEventCreate(&bt.e1) != hipSuccess)
    return fail(KNND_ERR_NOMEM);
  for (Group& g : groups) {
    st = create_group(g, inst, prm, on_device, stream);
    if (st != KNND_OK) return fail(st);
  }
  bool graphs = !(prm.flags & KNND_FLAG_NO_GRAPH);
  bool round_set = false;  // dround holds the index of the next graph-launched round
  int running = B;
  for (int r = 0; running > 0; ++r) {
    if (hipEventRecord(bt.e0, strm) != hipSuccess) return fail(KNND_ERR_DEVICE);
    // (graphs from the third round on, after the tuner's second-round trials)
    bool replay = graphs && r >= 3;
    if (replay) {
      std::vector<char> now;
      for (const Group& g : groups) now.push_back(g.running > 0);
      if (now != bt.captured && capture_graphs(bt) != KNND_OK) graphs = replay = false;
    }
    if (replay) {
      if (!round_set && knnd::launch_set_i64(bt.dround, r, strm) != hipSuccess) return fail(KNND_ERR_DEVICE);
      round_set = true;
      if (hipGraphLaunch(bt.exec[(r - 1) & 1], strm) != hipSuccess) return fail(KNND_ERR_DEVICE);
    } else {
      for (size_t q = 0; q < groups.size(); ++q) {
        Ctx& c = groups[q].c;
        if (groups[q].running == 0) continue;
        if ((r == 1 || r == 2) && c.tune && (r == 1 ? !c.tuned : !c.tuned2)) {
          // the join's schedule, from this round's snapshot (round 0 only builds the initial lists)
          if (knnd::launch_csr(c, c.F[c.cur]) != hipSuccess) return fail(KNND_ERR_DEVICE);
          if ((st = r == 1 ? tune_join(c, true) : tune_opt(c, true)) != KNND_OK) return fail(st);
          (r == 1 ? c.tuned : c.tuned2) = true;
        }
        if ((st = enqueue_group_round(bt, q, r, nullptr)) != KNND_OK) return fail(st);
      }
    }
    for (Group& g : groups)
      if (g.running > 0) {
        if (r > 0) g.c.cur ^= 1;
        g.c.round = r;
      }
    if (hipEventRecord(bt.e1, strm) != hipSuccess ||
        hipMemcpyAsync(bt.hall, bt.dall, rows * knnd::STAT_N * sizeof(int64_t), hipMemcpyDeviceToHost, strm) !=
            hipSuccess ||
        hipStreamSynchronize(strm) != hipSuccess)
      return fail(KNND_ERR_DEVICE);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, bt.e0, bt.e1) != hipSuccess) return fail(KNND_ERR_DEVICE);
    for (size_t q = 0; q < groups.size(); ++q) {
      Group& g = groups[q];
      if (g.running == 0 || g.c.round != r) continue;
      Ctx& c = g.c;
      if (bt.hall[(bt.sum_nb + (int64_t)q) * knnd::STAT_N + knnd::STAT_ERR] != 0) return fail(KNND_ERR_DEVICE);
      for (int j = 0; j < c.nb; ++j) {
        if (!g.active[j]) continue;
        knnd_instance& in = inst[g.members[j]];
        const int64_t* s = bt.hall + (size_t)(bt.slot[q] + j) * knnd::STAT_N;
        knnd_round_stats rs;
        rs.updates = s[knnd::STAT_UPDATES];
        rs.fcr_hits = s[knnd::STAT_HITS];
        rs.evals_alg = s[knnd::STAT_EVALS];
        rs.evals_performed = s[knnd::STAT_PERF];
        rs.rescues = s[knnd::STAT_RESCUES];
        rs.carried = 0;  // (groups evaluate every running receiver)
        rs.evals_carried = 0;
        rs.ms = ms;  // the round of every running group
        rs.ms_join = rs.ms_hub = rs.ms_recv = 0.0;
        if (in.stats) in.stats[r] = rs;
        if (r == 0) {
          g.hits_prev[j] = rs.fcr_hits;
          continue;
        }
        bool capped = false;
        if (should_stop(prm, in.n, in.K, g.hits_prev[j], rs.fcr_hits, rs.updates, r, &capped)) {
          in.status = capped ? KNND_WARN_MAX_ROUNDS : KNND_OK;
          if (capped) worst = KNND_WARN_MAX_ROUNDS;
          *in.out_rounds = r;
          if ((st = group_emit(g, j, in, on_device)) != KNND_OK) return fail(st);
          g.active[j] = 0;
          g.dirty = true;
          --g.running;
          --running;
        } else {
          g.hits_prev[j] = rs.fcr_hits;
        }
      }
      if (g.dirty && g.running > 0) {
        if (hipMemcpyAsync(c.iactive, g.active.data(), (size_t)c.nb * 4, hipMemcpyHostToDevice, c.stream) !=
            hipSuccess)
          return fail(KNND_ERR_DEVICE);
        g.dirty = false;
      }
    }
  }
  (void)fail(KNND_OK);
  return worst;
}

// A whole descent on a created context: start graph, rounds until the stop
// rule, lists (and keys) copied out.
int descend(Ctx& c, const knnd_params* p, int32_t on_device, int32_t* out_idx, double* out_kl,
            knnd_round_stats* stats, int32_t* out_rounds) {
  knnd_params prm;
  (void)resolve_params(p, c.n, &prm);  // already accepted by create
  knnd_round_stats rs;
  int st = init_graph(c, &rs);
  if (st == KNND_OK) {
    if (stats) stats[0] = rs;
    int64_t hits_prev = rs.fcr_hits;
    for (;;) {
      st = run_round(c, &rs);
      if (st != KNND_OK) break;
      if (stats) stats[c.round] = rs;
      bool capped = false;
      if (should_stop(prm, c.n, c.K, hits_prev, rs.fcr_hits, rs.updates, c.round, &capped)) {
        if (capped) st = KNND_WARN_MAX_ROUNDS;
        break;
      }
      hits_prev = rs.fcr_hits;
    }
  }
  if (st == KNND_OK || st == KNND_WARN_MAX_ROUNDS) {
    const int gst = get_graph(c, out_idx, out_kl, on_device);
    if (gst != KNND_OK) st = gst;
    *out_rounds = c.round;
  }
  return st;
}

}  // namespace

// ---------------------------------------------------------------------------
// Fixed device scratch of knnd_build_noalloc: KNND_NOALLOC_MAX_BYTES in the
// library's own code object, so every device the library runs on holds a
// copy of its own until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the device
// symbol): the address of each device's copy is looked up once, with that
// device current, and kept per device.  Every call on a device shares that
// device's copy; calls that overlap on one device race.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[KNND_NOALLOC_MAX_BYTES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// The address of device `dev`'s copy of the scratch array (dev is current).
int scratch_address(int dev, unsigned char** out) {
  *out = nullptr;
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return KNND_ERR_DEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return KNND_ERR_DEVICE;
    }
    g_scratch_ptr[dev] = static_cast<unsigned char*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return KNND_OK;
}
}  // namespace

extern "C" {

void knnd_default_params(knnd_params* p) {
  if (!p) return;
  p->precision = KNND_PREC_FP64;
  p->dtype = KNND_F32;
  p->fcr_samples = 0;
  p->max_rounds = 100;
  p->flags = 0;
  p->stop_rule = KNND_STOP_FCR;
  p->comparator = KNND_CMP_KL;
  p->delta = 0.0;
}

const char* knnd_status_string(int s) {
  switch (s) {
    case KNND_OK: return "KNND_OK";
    case KNND_WARN_MAX_ROUNDS: return "KNND_WARN_MAX_ROUNDS";
    case KNND_ERR_ARG: return "KNND_ERR_ARG";
    case KNND_ERR_DOMAIN: return "KNND_ERR_DOMAIN";
    case KNND_ERR_NOMEM: return "KNND_ERR_NOMEM";
    case KNND_ERR_DEVICE: return "KNND_ERR_DEVICE";
    case KNND_ERR_UNSUPPORTED: return "KNND_ERR_UNSUPPORTED";
    default: return "KNND_UNKNOWN_STATUS";
  }
}

int knnd_abi_version(void) { return KNND_ABI_VERSION; }

int knnd_release_cache(void) {
  knnd::pool_release();
  return KNND_OK;
}

int knnd_memory_stats(int64_t* live, int64_t* cached) {
  knnd::pool_stats(live, cached);
  return KNND_OK;
}

int64_t knnd_test_fail_alloc(int64_t k) {
  const int64_t left = knnd::g_fail_at.exchange(k > 0 ? k : 0);
  return left > 0 ? left : 0;
}

int knnd_ctx_create(const void* points, int64_t n, int32_t d, int32_t K, uint64_t seed, const knnd_params* p,
                    int32_t on_device, void* stream, knnd_ctx** out) {
  if (!points || !out) return KNND_ERR_ARG;
  *out = nullptr;
  knnd_ctx* h = new (std::nothrow) knnd_ctx();
  if (!h) return KNND_ERR_NOMEM;
  const int st = create(points, n, d, K, seed, p, on_device, stream, h->c);
  if (st != KNND_OK) {
    free_ctx(h->c);
    delete h;
    return st;
  }
  *out = h;
  return KNND_OK;
}

int knnd_ctx_init_graph(knnd_ctx* h, knnd_round_stats* st) {
  if (!h) return KNND_ERR_ARG;
  return init_graph(h->c, st);
}

int knnd_ctx_set_graph(knnd_ctx* h, const int32_t* idx, const double* kl, int32_t round, int32_t on_device) {
  if (!h || !idx || !kl || round < 0) return KNND_ERR_ARG;
  Ctx& c = h->c;
  const size_t nK = (size_t)c.n * c.K;
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  int32_t* staging = reinterpret_cast<int32_t*>(c.F[c.cur ^ 1]);
  KNND_HIP(hipMemcpyAsync(staging, idx, nK * 4, kind, c.stream));
  KNND_HIP(hipMemsetAsync(c.dflag, 0, sizeof(int32_t), c.stream));
  KNND_HIP(knnd::launch_load_idx(c, staging, c.F[c.cur], c.dflag));
  KNND_HIP(hipMemcpyAsync(c.keys[c.cur], kl, nK * 8, kind, c.stream));
  int32_t bad = 0;
  KNND_HIP(hipMemcpyAsync(&bad, c.dflag, sizeof(int32_t), hipMemcpyDeviceToHost, c.stream));
  KNND_HIP(hipStreamSynchronize(c.stream));
  if (bad) {
    c.have_graph = false;
    return KNND_ERR_ARG;
  }
  c.round = round;
  c.have_graph = true;
  c.track_ok = false;
  return KNND_OK;
}

int knnd_ctx_round(knnd_ctx* h, knnd_round_stats* st) {
  if (!h) return KNND_ERR_ARG;
  return run_round(h->c, st);
}

int knnd_ctx_round_share(knnd_ctx* h, int64_t first, int64_t count, knnd_round_stats* st) {
  if (!h) return KNND_ERR_ARG;
  return run_round_share(h->c, first, count, st);
}

int knnd_ctx_get_graph(knnd_ctx* h, int32_t* idx, double* kl, int32_t on_device) {
  if (!h || !idx || !h->c.have_graph) return KNND_ERR_ARG;
  return get_graph(h->c, idx, kl, on_device);
}

int knnd_ctx_get_cofriends(knnd_ctx* h, int64_t* rowptr, int32_t* col, int32_t on_device) {
  if (!h || !rowptr || !col || !h->c.have_graph) return KNND_ERR_ARG;
  if (on_device) return KNND_ERR_UNSUPPORTED;
  Ctx& c = h->c;
  const size_t nK = (size_t)c.n * c.K;
  KNND_HIP(knnd::launch_csr(c, c.F[c.cur]));
  KNND_HIP(hipMemcpyAsync(rowptr, c.rowptr, ((size_t)c.n + 1) * 8, hipMemcpyDeviceToHost, c.stream));
  KNND_HIP(hipMemcpyAsync(col, c.col, nK * 4, hipMemcpyDeviceToHost, c.stream));
  KNND_HIP(hipStreamSynchronize(c.stream));
  for (size_t e = 0; e < nK; ++e) col[e] = (int32_t)((uint32_t)col[e] & knnd::IDMASK_HOST);
  for (int64_t y = 0; y < c.n; ++y) std::sort(col + rowptr[y], col + rowptr[y + 1]);
  return KNND_OK;
}

int knnd_ctx_get_log_table(knnd_ctx* h, double* L, int32_t on_device) {
  if (!h || !L) return KNND_ERR_ARG;
  Ctx& c = h->c;
  KNND_HIP(hipMemcpy2DAsync(L, (size_t)c.D * 8, c.L, (size_t)c.Dp * 8, (size_t)c.D * 8, (size_t)c.n,
                            on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c.stream));
  KNND_HIP(hipStreamSynchronize(c.stream));
  return KNND_OK;
}

int knnd_ctx_rounds(const knnd_ctx* h) { return h ? h->c.round : -1; }

int knnd_ctx_destroy(knnd_ctx* h) {
  if (!h) return KNND_ERR_ARG;
  (void)hipStreamSynchronize(h->c.stream);
  free_ctx(h->c);
  delete h;
  return KNND_OK;
}

int knnd_build_ex(const void* points, int64_t n, int32_t d, int32_t K, uint64_t seed, const knnd_params* p,
                  int32_t on_device, void* stream, int32_t* out_idx, double* out_kl, knnd_round_stats* stats,
                  int32_t* out_rounds) {
  if (!points || !out_idx || !out_rounds) return KNND_ERR_ARG;
  knnd_ctx* h = nullptr;
  int st = knnd_ctx_create(points, n, d, K, seed, p, on_device, stream, &h);
  if (st != KNND_OK) return st;
  st = descend(h->c, p, on_device, out_idx, out_kl, stats, out_rounds);
  knnd_ctx_destroy(h);
  return st;
}

int knnd_build_noalloc(const void* points, int64_t n, int32_t d, int32_t K, uint64_t seed, const knnd_params* p,
                       void* stream, int32_t* out_idx, double* out_kl, knnd_round_stats* stats,
                       int32_t* out_rounds) {
  if (!points || !out_idx || !out_rounds) return KNND_ERR_ARG;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return KNND_ERR_DEVICE;
  unsigned char* base = nullptr;
  int st = scratch_address(dev, &base);
  if (st != KNND_OK) return st;
  Ctx c;  // (on the stack: nothing is allocated)
  c.arena = base;
  c.arena_size = (size_t)KNND_NOALLOC_MAX_BYTES;
  st = create(points, n, d, K, seed, p, 1, stream, c);
  if (st == KNND_OK) st = descend(c, p, 1, out_idx, out_kl, stats, out_rounds);
  free_ctx(c);  // (synchronises the stream; an arena gives nothing back)
  return st;
}

int knnd_build_batched(knnd_instance* inst, int32_t B, const knnd_params* p, int32_t on_device, void* stream) {
  return build_batched(inst, B, p, on_device, stream);
}

int knnd_build(const float* points, int64_t n, int32_t d, int32_t K, uint64_t seed, int32_t* out_idx,
               int64_t* out_updates, int32_t max_rounds, int32_t* out_rounds) {
  if (!points || !out_idx || !out_updates || !out_rounds || max_rounds < 1) return KNND_ERR_ARG;
  knnd_params p;
  knnd_default_params(&p);
  p.max_rounds = max_rounds;
  knnd_round_stats* stats = new (std::nothrow) knnd_round_stats[(size_t)max_rounds + 1];
  if (!stats) return KNND_ERR_NOMEM;
  const int st = knnd_build_ex(points, n, d, K, seed, &p, 0, nullptr, out_idx, nullptr, stats, out_rounds);
  if (st == KNND_OK || st == KNND_WARN_MAX_ROUNDS)
    for (int r = 1; r <= *out_rounds; ++r) out_updates[r - 1] = stats[r].updates;
  delete[] stats;
  return st;
}

}  // extern "C"
