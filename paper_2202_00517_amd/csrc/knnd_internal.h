// Internal interface between the host orchestrator and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include <algorithm>

namespace knnd {

// Receiver classes by hash-table capacity, tables in LDS: 512 << k slots for
// classes k = 0..4, MID_CAP slots for class 5 (not a power of two: a 46 KB
// table leaves room for three blocks per CU), 16384 and 32768 slots for
// classes 6 and 7; classes 4..7 (and the exact form's class 3) keep their
// candidate lists in global memory; class 8 has its table there too, for
// very large co-friend lists.
constexpr int NCLASS = 9;
constexpr uint32_t MID_CAP = 11776;
constexpr int BIG_CAND = 24576;  // candidate-list entries per block of the big LDS classes
constexpr int HUB_MAXD = 64;     // register hub kernel up to this many coordinates;
                                 // P and L carry HUB_MAXD zeroed elements of tail padding
constexpr uint32_t IDMASK_HOST = 0x3FFFFFFFu;  // point indices are below this
constexpr uint32_t CLASS_CAP_MIN = 512;
constexpr int SHORT_LIST = 128;  // candidate lists up to this long are merged by k_merge
// Bucketed reverse-neighbour build: at most CSR_MAXB buckets of 256..CSR_MAXTB
// consecutive targets (n <= CSR_MAXB * CSR_MAXTB); larger n uses per-edge atomics.
constexpr int CSR_MAXB = 4096;
constexpr int CSR_MAXTB = 8192;

// Key fold kinds and feature table kinds of the comparators (knnd_comparator):
// KL -> (CK_KL, TK_LOG), reverse KL -> (CK_REV, TK_LOG), Hellinger ->
// (CK_SQ, TK_SQRT), Euclidean -> (CK_SQ, TK_ID).
enum { CK_KL = 0, CK_REV = 1, CK_SQ = 2 };
enum { TK_LOG = 0, TK_SQRT = 1, TK_ID = 2 };
inline int cmp_fold_kind(int cmp) { return cmp == 1 ? CK_REV : (cmp >= 2 ? CK_SQ : CK_KL); }
inline int cmp_table_kind(int cmp) { return cmp == 2 ? TK_SQRT : (cmp == 3 ? TK_ID : TK_LOG); }

// Per-round device counters
// (STAT_CARRIED: receivers whose list and count were carried over unchanged;
// STAT_EVCARRY: the evaluations they add to STAT_EVALS)
enum {
  STAT_UPDATES = 0, STAT_HITS = 1, STAT_EVALS = 2, STAT_PERF = 3, STAT_RESCUES = 4, STAT_ERR = 5,
  STAT_CARRIED = 6, STAT_EVCARRY = 7, STAT_N = 8
};
// Per-point counters of one round in a batched group (summed per instance):
// evaluations and updates of receiver x, keys computed by hub x, keys
// computed by receiver x (pull form and rescues), rescues of receiver x
enum { VC_EVALS = 0, VC_UPD = 1, VC_HUBPERF = 2, VC_RECVPERF = 3, VC_RESC = 4, VC_N = 5 };

struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cu = 0;
  int64_t n = 0;
  int d = 0, D = 0, Dp = 0, Ds = 0, K = 0;
  uint64_t seed = 0;
  int dtype = 0;      // 0 F32, 1 F64
  int precision = 0;
  int flags = 0;
  int cmp = 0;        // knnd_comparator
  int ck = 0;         // its key fold kind (CK_*)
  int tk = 0;         // its feature table kind (TK_*)
  int64_t M = 0;
  int max_rounds = 100;
  int round = 0;      // rounds completed
  bool have_graph = false;
  // receivers whose lists a round updates: [own0, own1) (all of them unless
  // a round is restricted to one share of the receivers)
  int64_t own0 = 0, own1 = 0;
  // the last round updated only a share of the receivers: an edge present a
  // round earlier no longer means that its pairs were evaluated then (a
  // receiver outside the share evaluated nothing), so the next round skips
  // no pair
  bool no_skip_next = false;
  // single descents in the hub form: per point, bit 0 = its list gained an
  // entry in the last round, bit 1 = some list dropped it; and the
  // evaluation count of its last update.  A receiver whose own flags and
  // whose friends' and co-friends' bit 0 are clear has the same candidate
  // set and list as one round earlier (see k_bin).
  int32_t* vchg = nullptr;
  int32_t* vev = nullptr;  // [n][VC_N] per-point counters of the last update (VC_EVALS is used)
  bool track_capable = false; // a single descent in the hub form (arrays allocated on first use)
  bool tracking = false;      // this round gathers the flags and counts
  bool track_ok = false;      // the last round updated every receiver with tracking on
  int64_t last_updates = -1;  // updates of the last round

  // device buffers
  void* P = nullptr;          // [n][D] points (copy owned by the context)
  double* Pw = nullptr;       // FP64 copy of FP32 points, reverse-KL hub form only (the fold weighs by
                              // the candidate's coordinates, read per candidate)
  double* L = nullptr;        // [n][Dp] feature table (log x for the KL comparators)
  // F rows have stride Ks, the power of two >= max(K, 8): a row never
  // straddles more cache lines than its size needs
  uint32_t* F[2] = {nullptr, nullptr};
  int Ks = 0;
  double* keys[2] = {nullptr, nullptr};
  int cur = 0;                // F[cur], keys[cur] hold the current snapshot
  int32_t* deg = nullptr;     // [n]
  int32_t* fill = nullptr;    // [n]
  int64_t* rowptr = nullptr;  // [n+1]
  uint32_t* col = nullptr;    // [nK]
  uint8_t* colslot = nullptr; // [nK] slot of the edge in its source's list
  double* seg = nullptr;      // [nK(K+Ks+1)] candidate keys by snapshot edge (hub form)
  // Exact hub form: each point's D logs, then its D coordinates (the input
  // type), in one row of whole 128-byte lines, hstride bytes apart; the
  // register hub kernel reads these instead of the rows of L and P (which
  // straddle lines).  Optional: null when it did not fit.
  double* Hrow = nullptr;
  int64_t hstride = 0;
  // mixed precision
  bool mixed = false;
  int dk = 0;                 // D padded to 32 or 64 (MFMA K dimension)
  void* Ph = nullptr;         // [n][2 dk] x split in 16-bit high and low parts (rows: dk high, dk low)
  void* Lh = nullptr;         // [n][2 dk] the same split of L
  double* S = nullptr;        // [n] sum_i x_i log x_i
  float* seg32 = nullptr;     // [nK(K+Ks+1)] cross terms C~ by snapshot edge
  double eps_relq = 0.0, eps_abs = 0.0;  // mixed-form error bound: e_rel / (1 - e_rel) and e_abs
  bool use_hub = false;
  // Join schedule (every choice gives the same results; see the tuner in
  // knnd_api.hip): the exact hub form runs k_hub_lds instead of k_hub_reg
  bool hub_lds = false;
  mutable int hub_lds_grid = 0;  // its grid, fixed on first use
  int hub_hpw = 1;               // hubs per wave of the register hub kernel (1, 2 or 4; small K)
  int recv_wave = 0;             // smallest receiver classes one wave per receiver (0: none, 1: 512 slots, 2: and 1024)
  bool opt4096 = false;          // receivers of the 8192-slot class that probably fit try a guarded 4096-slot table
  bool auto_prec = false;        // KNND_PREC_AUTO: the tuner picks exact or mixed
  bool tune = false;             // time the candidate schedules on the first round
  bool tuned = false;
  bool tuned2 = false;           // the second-round trials (guarded 4096-slot tables) are done
  bool mixed_ok = false;         // the mixed form's operands and bound are ready
  bool plain_ok = false;         // the exact hub form's key slots are ready
  // short candidate lists handed from the receiver kernel to k_merge (hub form)
  int32_t* sl_n = nullptr;     // [n] list length, -1 when the receiver kernel merged itself
  uint32_t* sl_id = nullptr;   // [n][SHORT_LIST]
  double* sl_key = nullptr;    // [n][SHORT_LIST] (exact hub form only)
  int64_t* tilesum = nullptr;
  // bucketed CSR build (null when n is too large for it)
  uint64_t* csr_T = nullptr;       // [nK] edges partitioned by target bucket
  int64_t* csr_bcount = nullptr;   // [CSR_MAXB] edges per bucket
  int64_t* csr_bfill = nullptr;    // [CSR_MAXB] reservation cursors
  int64_t* csr_bbase = nullptr;    // [CSR_MAXB + 1] first edge of each bucket
  int csr_shift = 8;               // log2 of the targets per bucket
  int32_t* class_count = nullptr;  // [NCLASS]
  int32_t* class_list = nullptr;   // [NCLASS][n]
  uint32_t* gtab = nullptr;        // [gblocks][gstride]
  uint32_t* gcand = nullptr;       // [gblocks][gstride/2]
  double* gckey = nullptr;         // [gblocks][gstride/2]
  uint32_t* bcand = nullptr;       // [bblocks][BIG_CAND]
  double* bckey = nullptr;         // [bblocks][BIG_CAND]
  int bblocks = 0;
  int64_t gstride = 0;
  int gblocks = 0;
  int64_t* dstats = nullptr;  // [STAT_N] device
  int64_t* hstats = nullptr;  // [STAT_N] pinned host (fixed-scratch mode: hstats_local)
  // Fixed-scratch mode (the entry point that allocates nothing): every device
  // buffer is carved from [arena, arena + arena_size) by a bump pointer
  // instead of coming from the memory cache; no events, no pinned memory
  unsigned char* arena = nullptr;
  size_t arena_size = 0, arena_used = 0;
  int64_t hstats_local[STAT_N] = {};
  int32_t* dflag = nullptr;   // device scratch flag
  hipEvent_t ev0 = nullptr, ev1 = nullptr, evj0 = nullptr, evj1 = nullptr, evh = nullptr;

  // Batched group (nb > 0): nb independent instances laid out one after the
  // other in [0, n); every list stays inside its instance, so one round of
  // the group is one round of each active instance.
  int nb = 0;
  int32_t* inst_of = nullptr;  // [n] instance of each point
  int64_t* ioff = nullptr;     // [nb+1] first point of each instance (ioff[nb] = n)
  uint64_t* iseed = nullptr;   // [nb] seed of each instance
  int64_t* iM = nullptr;       // [nb] FCR samples of each instance
  int32_t* iD = nullptr;       // [nb] coordinates of each instance (<= D; the rest is zero padding)
  int32_t* iactive = nullptr;  // [nb] nonzero while the instance runs
  int64_t* istats = nullptr;   // [nb][STAT_N] per-instance counters of the round
  int64_t* histats = nullptr;  // [nb][STAT_N] pinned host copy
  int32_t* vcnt = nullptr;     // [n][VC_N] per-point counters of the round
  int64_t Mmax = 0;            // largest iM
};

struct JoinArgs {
  const void* P;
  const double* L;
  int64_t n;
  int D, Dp, Ds, K;
  int ck;  // comparator kind of the key fold (CK_*)
  const uint32_t* F;
  const double* keys;
  const int64_t* rowptr;
  const uint32_t* col;
  const uint8_t* colslot;
  int64_t nKK;     // n*K*Ks: offset of the FC part of seg (FF rows of K slots padded to Ks)
  int64_t di_off;  // 2*n*K*Ks: offset of the DI part of seg
  int Ks;          // row stride of F (and of the FC blocks of seg)
  const float* seg32;
  const double* S;
  double eps_relq, eps_abs;
  double* seg;
  uint32_t* Fn;
  double* keysn;
  int64_t* stats;
  int skip;
  uint32_t* gtab;
  uint32_t* gcand;
  double* gckey;
  int64_t gstride;
  uint32_t* bcand;
  double* bckey;
  // batched groups (null otherwise)
  const int32_t* inst_of;
  const int32_t* iactive;
  int32_t* vcnt;
  // short lists (hub form)
  int32_t* sl_n;
  uint32_t* sl_id;
  double* sl_key;
  // receivers whose lists this round updates, [own0, own1)
  int64_t own0, own1;
};

// Device memory of the library comes from a per-process cache of freed
// blocks (see knnd_release_cache): pool_malloc and pool_free stand in for
// hipMalloc and hipFree.  A block goes back to the cache only after the work
// using it has finished (callers synchronise its stream first).
hipError_t pool_malloc(void** p, size_t bytes);
void pool_free(void* p);
void pool_release();
void pool_stats(int64_t* live, int64_t* cached);
extern std::atomic<int64_t> g_fail_at;
template <class T>
hipError_t pmalloc(T** p, size_t bytes) {
  return pool_malloc(reinterpret_cast<void**>(p), bytes);
}

hipError_t launch_zero_i64(int64_t* p, int64_t n, hipStream_t s);
hipError_t launch_log_table(const Ctx& c, int32_t* bad);
hipError_t launch_widen(const Ctx& c);
hipError_t launch_hub_rows(const Ctx& c);
hipError_t launch_init_graph(const Ctx& c);
hipError_t launch_fcr(const Ctx& c, const uint32_t* F, int64_t round, int64_t* hits,
                      const int64_t* round_dev = nullptr);
hipError_t launch_csr(const Ctx& c, const uint32_t* F);
hipError_t launch_bin(const Ctx& c, bool carry);
hipError_t launch_join_hub(const Ctx& c, int64_t* stats);
hipError_t launch_join_recv(const Ctx& c, int64_t* stats);
hipError_t launch_prep_mixed(const Ctx& c, unsigned long long* maxbits);
hipError_t launch_strip(const Ctx& c, const uint32_t* F, int32_t* out);
hipError_t launch_put_rows(const Ctx& c);
hipError_t launch_track(const Ctx& c);
hipError_t launch_load_idx(const Ctx& c, const int32_t* idx, uint32_t* F, int32_t* bad);
// batched groups
hipError_t launch_batch_reduce(const Ctx& c);
hipError_t launch_emit(const Ctx& c, int64_t off, int64_t n_b, int32_t* out_idx);
hipError_t launch_zero_i32(int32_t* p, int64_t n, hipStream_t s);
hipError_t launch_copy_i64(int64_t* dst, const int64_t* src, int64_t cnt, hipStream_t s);
hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t s);
hipError_t launch_add_i64(int64_t* p, int64_t v, hipStream_t s);

}  // namespace knnd
