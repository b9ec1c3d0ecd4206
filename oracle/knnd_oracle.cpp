// CPU oracle for comparator-based K-nearest-neighbor descent (NND) with the
// Kullback-Leibler comparator and a small family of other comparators.
//
// TEST INFRASTRUCTURE ONLY.  This file defines what the GPU library must
// compute, in plain, slow, obviously-correct C++ (FP64, correctly rounded log,
// explicit fma, std::sort).  It shares no code with the GPU library and is loaded only by
// the tests, by the smoke check and by the benchmark's CPU-baseline leg.
//
// Paper: Baron & Darling, "Empirical complexity of comparator-based nearest
// neighbor descent" (arXiv 2202.00517).  Each function below names the passage
// it follows.  Where the paper leaves a detail open, the reading taken is the
// one stated at that function.
//
// Pins (what ties this code to the paper rather than to itself) live in
// tests/test_oracle_*.py: closed-form KL values, the published SplitMix64 test
// vector, brute-force exact K-NN on tiny inputs, a matrix-algebra formulation
// of the candidate set, exhaustive friend-clustering rates, and invariants;
// for the other comparators, closed forms, exact symmetry, acyclic ranking
// digraphs of the metric ones (Section 2.1's theorem) and k-d tree searches.
// Parity unpinned: the round counts, FCR values and update counts at the
// benchmark sizes have no printed value in the paper; only GPU-vs-oracle
// parity and the paper's soft round bound apply there.

#include <quadmath.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <utility>
#include <vector>

namespace {

enum {
  ORC_OK = 0,
  ORC_WARN_MAX_ROUNDS = 1,
  ORC_ERR_ARG = -1,
  ORC_ERR_DOMAIN = -2,
};

// ---------------------------------------------------------------------------
// Counter-based randomness.  The paper only asks for uniform random choices
// (Section 3.2: each point picks K others uniformly at random; Section 3.3:
// sample a point and two of its friends uniformly).  Every draw here is a
// SplitMix64-finalizer hash of (seed, tag, a, b), so the draws do not depend on
// thread count or evaluation order.  Tags: 1 initial graph, 2/3/4 FCR point /
// first slot / second slot.
// ---------------------------------------------------------------------------
uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

uint64_t hash4(uint64_t s, uint64_t t, uint64_t a, uint64_t b) {
  return mix64(mix64(mix64(s ^ (t * 0x9E3779B97F4A7C15ULL)) ^ a) ^ b);
}

// Uniform integer in [0, m): high 64 bits of the 128-bit product h*m.
uint64_t bound(uint64_t h, uint64_t m) {
  return (uint64_t)(((unsigned __int128)h * m) >> 64);
}

int nthreads(int t) {
  if (t > 0) return t;
  unsigned h = std::thread::hardware_concurrency();
  return h ? (int)h : 1;
}

// Run f(lo, hi, tid) over disjoint contiguous ranges of [0, n).
template <class Fn>
void parallel_ranges(int64_t n, int threads, Fn f) {
  int T = nthreads(threads);
  if (T > n) T = (int)std::max<int64_t>(n, 1);
  if (T <= 1) { f(0, n, 0); return; }
  std::vector<std::thread> pool;
  for (int t = 0; t < T; ++t) {
    int64_t lo = n * t / T, hi = n * (t + 1) / T;
    pool.emplace_back([=, &f] { f(lo, hi, t); });
  }
  for (auto& th : pool) th.join();
}

// ---------------------------------------------------------------------------
// The comparator (Section 2.2; Section 4 scaling experiment):
// y ranks before z for x when D(x||y) < D(x||z), with
// D(x||y) = sum_i x_i log(x_i / y_i) summed over every stored coordinate.
// log(x_i / y_i) is written as log x_i - log y_i (exact algebra) with the logs
// taken once per coordinate and rounded correctly to FP64, and the sum is
// folded in ascending coordinate order with one fused multiply-add per term.
// This fixes every rounding, so the value is a reproducible FP64 number that
// does not depend on any math library's accuracy.
// Ties between equal keys go to the lower point index (the paper is silent).
// ---------------------------------------------------------------------------
double kl_key(const double* P, const double* L, int D, int64_t x, int64_t y) {
  const double* px = P + (size_t)x * D;
  const double* lx = L + (size_t)x * D;
  const double* ly = L + (size_t)y * D;
  double acc = 0.0;
  for (int i = 0; i < D; ++i) acc = std::fma(px[i], lx[i] - ly[i], acc);
  return acc;
}

// Other comparators.  The method only needs, for each x, a total order on the
// other points (Section 2.1: a ranking system, one Comparator per x; Section
// 1.3 (a)); these keys give such orders, each with the same (key, index)
// tie rule and the same fixed rounding (ascending fold, one fma per term):
//   CMP_KL          D(x||y) as above;
//   CMP_KL_REVERSE  D(y||x) = sum_i y_i (log y_i - log x_i): KL with the roles
//                   of the two points exchanged (still asymmetric);
//   CMP_HELLINGER   sum_i (sqrt x_i - sqrt y_i)^2, twice the squared Hellinger
//                   distance between the two distributions (a metric after
//                   the square root, so it induces a metric ranking system);
//   CMP_L2          sum_i (x_i - y_i)^2, the squared Euclidean distance.
// Square roots are IEEE (correctly rounded) FP64 square roots of the widened
// coordinates, taken here per pair.
enum { CMP_KL = 0, CMP_KL_REVERSE = 1, CMP_HELLINGER = 2, CMP_L2 = 3 };

double cmp_key(int cmp, const double* P, const double* L, int D, int64_t x, int64_t y) {
  const double* px = P + (size_t)x * D;
  const double* py = P + (size_t)y * D;
  double acc = 0.0;
  if (cmp == CMP_KL) return kl_key(P, L, D, x, y);
  if (cmp == CMP_KL_REVERSE) {
    const double* lx = L + (size_t)x * D;
    const double* ly = L + (size_t)y * D;
    for (int i = 0; i < D; ++i) acc = std::fma(py[i], ly[i] - lx[i], acc);
  } else if (cmp == CMP_HELLINGER) {
    for (int i = 0; i < D; ++i) {
      const double t = std::sqrt(px[i]) - std::sqrt(py[i]);
      acc = std::fma(t, t, acc);
    }
  } else {
    for (int i = 0; i < D; ++i) {
      const double t = px[i] - py[i];
      acc = std::fma(t, t, acc);
    }
  }
  return acc;
}

bool cmp_valid(int cmp) { return cmp >= CMP_KL && cmp <= CMP_L2; }

using Entry = std::pair<double, int32_t>;  // (key, index): lexicographic order

// Reverse neighbors (Section 4.2: the co-friend map is derived from the friend
// map): coF(v) = { x : v is a friend of x }, listed by ascending x.
void build_cofriends(const int32_t* F, int64_t n, int K, std::vector<int64_t>& rowptr,
                     std::vector<int32_t>& col) {
  rowptr.assign((size_t)n + 1, 0);
  for (int64_t x = 0; x < n; ++x)
    for (int j = 0; j < K; ++j) rowptr[(size_t)F[(size_t)x * K + j] + 1]++;
  for (int64_t v = 0; v < n; ++v) rowptr[(size_t)v + 1] += rowptr[(size_t)v];
  std::vector<int64_t> cur(rowptr.begin(), rowptr.end() - 1);
  col.assign((size_t)n * K, 0);
  for (int64_t x = 0; x < n; ++x)
    for (int j = 0; j < K; ++j) {
      int32_t v = F[(size_t)x * K + j];
      col[(size_t)cur[(size_t)v]++] = (int32_t)x;
    }
}

// Candidate set of x (Section 3.1 "Meet"; Section 4.2, proposeNewFriendSet):
// the co-friends of x, the friends of its friends and the friends of its
// co-friends, as a set, without x itself and without the current friends of x.
// Returned sorted by index.
std::vector<int32_t> candidates(const int32_t* F, int K, const std::vector<int64_t>& rowptr,
                                const std::vector<int32_t>& col, int64_t x) {
  std::vector<int32_t> U;
  const int32_t* fx = F + (size_t)x * K;
  for (int64_t q = rowptr[(size_t)x]; q < rowptr[(size_t)x + 1]; ++q) U.push_back(col[(size_t)q]);
  for (int j = 0; j < K; ++j) {
    const int32_t* fv = F + (size_t)fx[j] * K;
    for (int s = 0; s < K; ++s) U.push_back(fv[s]);
  }
  for (int64_t q = rowptr[(size_t)x]; q < rowptr[(size_t)x + 1]; ++q) {
    const int32_t* fw = F + (size_t)col[(size_t)q] * K;
    for (int s = 0; s < K; ++s) U.push_back(fw[s]);
  }
  std::sort(U.begin(), U.end());
  U.erase(std::unique(U.begin(), U.end()), U.end());
  std::vector<int32_t> own(fx, fx + K);
  own.push_back((int32_t)x);
  std::sort(own.begin(), own.end());
  std::vector<int32_t> out;
  std::set_difference(U.begin(), U.end(), own.begin(), own.end(), std::back_inserter(out));
  return out;
}

// Friend set update of one vertex (Section 3.1 "Update"; Section 4.2): the new
// friend list is the best K, in the comparator's order, of the former friends
// and the candidates.  Former friends keep their stored keys (they are the
// same canonical values).  Returns the number of candidate evaluations and
// writes the number of new entries in the list.
int64_t update_vertex(int cmp, const double* P, const double* L, int D, int K, const int32_t* F,
                      const double* keys, const std::vector<int64_t>& rowptr,
                      const std::vector<int32_t>& col, int64_t x, int32_t* outF,
                      double* outKeys, int64_t* updates) {
  std::vector<int32_t> U = candidates(F, K, rowptr, col, x);
  std::vector<Entry> pool;
  pool.reserve(U.size() + K);
  for (int j = 0; j < K; ++j)
    pool.emplace_back(keys[(size_t)x * K + j], F[(size_t)x * K + j]);
  for (int32_t z : U) pool.emplace_back(cmp_key(cmp, P, L, D, x, z), z);
  std::sort(pool.begin(), pool.end());
  std::vector<int32_t> old(F + (size_t)x * K, F + (size_t)x * K + K);
  std::sort(old.begin(), old.end());
  int64_t fresh = 0;
  for (int j = 0; j < K; ++j) {
    outF[j] = pool[(size_t)j].second;
    outKeys[j] = pool[(size_t)j].first;
    if (!std::binary_search(old.begin(), old.end(), outF[j])) ++fresh;
  }
  *updates = fresh;
  return (int64_t)U.size();
}

// Domain of each comparator: the KL forms need every coordinate finite and
// > 0 (points of the open simplex), the Hellinger form finite and >= 0, the
// Euclidean form finite.
bool points_ok(int cmp, const double* P, size_t count) {
  for (size_t i = 0; i < count; ++i) {
    if (!std::isfinite(P[i])) return false;
    if ((cmp == CMP_KL || cmp == CMP_KL_REVERSE) && !(P[i] > 0.0)) return false;
    if (cmp == CMP_HELLINGER && !(P[i] >= 0.0)) return false;
  }
  return true;
}

}  // namespace

extern "C" {

int oracle_abi_version(void) { return 1; }

uint64_t oracle_mix64(uint64_t z) { return mix64(z); }
uint64_t oracle_hash(uint64_t s, uint64_t t, uint64_t a, uint64_t b) { return hash4(s, t, a, b); }
uint64_t oracle_bound(uint64_t h, uint64_t m) { return bound(h, m); }

// L = log(P), elementwise, rounded correctly to FP64: the natural log is taken
// in binary128 (113-bit significand) and rounded once to the nearest double.
void oracle_log_table(const double* P, int64_t count, double* L, int threads) {
  parallel_ranges(count, threads, [&](int64_t lo, int64_t hi, int) {
    for (int64_t i = lo; i < hi; ++i) L[i] = (double)logq((__float128)P[i]);
  });
}

double oracle_key(const double* P, const double* L, int D, int64_t x, int64_t y, int cmp) {
  if (!cmp_valid(cmp)) return std::nan("");
  return cmp_key(cmp, P, L, D, x, y);
}

// Random K-out initial graph (Section 3.2; Section 4.2): each x draws points of
// S \ {x} uniformly, keeping the first K distinct ones (sampling without
// replacement), then orders them by the comparator (the friend sets are
// ordered on insertion).  Draw a of x is r = bound(hash(seed,1,x,a), n-1),
// mapped past x as y = r + (r >= x).
int oracle_initial_graph(const double* P, const double* L, int64_t n, int D, int K,
                         uint64_t seed, int32_t* F, double* keys, int threads, int cmp) {
  if (n < 2 || K < 1 || K > n - 1 || D < 1 || !cmp_valid(cmp)) return ORC_ERR_ARG;
  parallel_ranges(n, threads, [&](int64_t lo, int64_t hi, int) {
    std::vector<Entry> row;
    for (int64_t x = lo; x < hi; ++x) {
      row.clear();
      for (uint64_t a = 0; (int)row.size() < K; ++a) {
        int64_t r = (int64_t)bound(hash4(seed, 1, (uint64_t)x, a), (uint64_t)(n - 1));
        int64_t y = r + (r >= x ? 1 : 0);
        bool seen = false;
        for (const Entry& e : row) seen = seen || e.second == (int32_t)y;
        if (!seen) row.emplace_back(0.0, (int32_t)y);
      }
      for (Entry& e : row) e.first = cmp_key(cmp, P, L, D, x, e.second);
      std::sort(row.begin(), row.end());
      for (int j = 0; j < K; ++j) {
        F[(size_t)x * K + j] = row[(size_t)j].second;
        keys[(size_t)x * K + j] = row[(size_t)j].first;
      }
    }
  });
  return ORC_OK;
}

// Friend clustering rate, sampled (Section 3.3 (i)-(ii)): M samples; sample s
// of round r picks x = bound(hash(seed,2,r,s), n) and two distinct friend slots
// a = bound(hash(seed,3,r,s), K), b = b' + (b' >= a) with
// b' = bound(hash(seed,4,r,s), K-1); with y, z the friends in those slots, it
// is a hit when y is a friend of z or a co-friend of z (z is a friend of y).
// Returns the hit count; the rate is hits / M.
int64_t oracle_fcr(const int32_t* F, int64_t n, int K, uint64_t seed, int64_t round, int64_t M) {
  int64_t hits = 0;
  for (int64_t s = 0; s < M; ++s) {
    int64_t x = (int64_t)bound(hash4(seed, 2, (uint64_t)round, (uint64_t)s), (uint64_t)n);
    int a = (int)bound(hash4(seed, 3, (uint64_t)round, (uint64_t)s), (uint64_t)K);
    int bp = (int)bound(hash4(seed, 4, (uint64_t)round, (uint64_t)s), (uint64_t)(K - 1));
    int b = bp + (bp >= a ? 1 : 0);
    int32_t y = F[(size_t)x * K + a], z = F[(size_t)x * K + b];
    bool hit = false;
    for (int j = 0; j < K; ++j) hit = hit || F[(size_t)z * K + j] == y || F[(size_t)y * K + j] == z;
    hits += hit ? 1 : 0;
  }
  return hits;
}

// Friend clustering rate over every (x, unordered pair of distinct friend
// slots): the population value the sampler estimates.
void oracle_fcr_exhaustive(const int32_t* F, int64_t n, int K, int64_t* hits, int64_t* pairs) {
  int64_t h = 0, p = 0;
  for (int64_t x = 0; x < n; ++x)
    for (int a = 0; a < K; ++a)
      for (int b = a + 1; b < K; ++b) {
        int32_t y = F[(size_t)x * K + a], z = F[(size_t)x * K + b];
        bool yz = false, zy = false;
        for (int j = 0; j < K; ++j) {
          yz = yz || F[(size_t)z * K + j] == y;
          zy = zy || F[(size_t)y * K + j] == z;
        }
        h += (yz || zy) ? 1 : 0;
        ++p;
      }
  *hits = h;
  *pairs = p;
}

// The candidate set of x (sorted by index); returns its size, writes up to cap.
int64_t oracle_candidates(const int32_t* F, int64_t n, int K, int64_t x, int32_t* out, int64_t cap) {
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  build_cofriends(F, n, K, rowptr, col);
  std::vector<int32_t> U = candidates(F, K, rowptr, col, x);
  for (size_t i = 0; i < U.size() && (int64_t)i < cap; ++i) out[i] = U[i];
  return (int64_t)U.size();
}

// One synchronous round (Section 4.2): every vertex's new list is computed
// from the same round-start snapshot (F, keys), which is never written while
// the round runs; the outputs become the next snapshot.
int oracle_round(const double* P, const double* L, int64_t n, int D, int K, const int32_t* F,
                 const double* keys, int32_t* Fn, double* keysn, int64_t* updates,
                 int64_t* evals, int threads, int cmp) {
  if (!cmp_valid(cmp)) return ORC_ERR_ARG;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  build_cofriends(F, n, K, rowptr, col);
  int T = nthreads(threads);
  std::vector<int64_t> upd(T + 1, 0), ev(T + 1, 0);
  parallel_ranges(n, T, [&](int64_t lo, int64_t hi, int t) {
    for (int64_t x = lo; x < hi; ++x) {
      int64_t u = 0;
      ev[t] += update_vertex(cmp, P, L, D, K, F, keys, rowptr, col, x, Fn + (size_t)x * K,
                             keysn + (size_t)x * K, &u);
      upd[t] += u;
    }
  });
  int64_t su = 0, se = 0;
  for (int t = 0; t <= T; ++t) { su += upd[t]; se += ev[t]; }
  *updates = su;
  *evals = se;
  return ORC_OK;
}

// The same update for a chosen subset of vertices (used to check large runs on
// a sample of vertices).  Row i of the outputs belongs to xs[i].
int oracle_round_subset(const double* P, const double* L, int64_t n, int D, int K,
                        const int32_t* F, const double* keys, const int64_t* xs, int64_t m,
                        int32_t* Fout, double* keysout, int64_t* upd, int64_t* evals,
                        int threads, int cmp) {
  if (!cmp_valid(cmp)) return ORC_ERR_ARG;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  build_cofriends(F, n, K, rowptr, col);
  parallel_ranges(m, threads, [&](int64_t lo, int64_t hi, int) {
    for (int64_t i = lo; i < hi; ++i)
      evals[i] = update_vertex(cmp, P, L, D, K, F, keys, rowptr, col, xs[i], Fout + (size_t)i * K,
                               keysout + (size_t)i * K, &upd[i]);
  });
  return ORC_OK;
}

// Exact K-NN of the query points qs under the comparator, by sorting all of
// S \ {q} (Section 2.3: the naive computation).
int oracle_bruteforce(const double* P, const double* L, int64_t n, int D, int K,
                      const int64_t* qs, int64_t m, int32_t* out, double* keys, int threads,
                      int cmp) {
  if (K > n - 1 || !cmp_valid(cmp)) return ORC_ERR_ARG;
  parallel_ranges(m, threads, [&](int64_t lo, int64_t hi, int) {
    std::vector<Entry> all;
    for (int64_t i = lo; i < hi; ++i) {
      int64_t q = qs[i];
      all.clear();
      for (int64_t y = 0; y < n; ++y)
        if (y != q) all.emplace_back(cmp_key(cmp, P, L, D, q, y), (int32_t)y);
      std::partial_sort(all.begin(), all.begin() + K, all.end());
      for (int j = 0; j < K; ++j) {
        out[(size_t)i * K + j] = all[(size_t)j].second;
        keys[(size_t)i * K + j] = all[(size_t)j].first;
      }
    }
  });
  return ORC_OK;
}

// The stop rule (Section 3.3 (iv)): stop after round r when the clustering
// rate did not increase (hits_r <= hits_{r-1}; M is fixed so counts compare
// exactly).  Also stop at a fixed point (no update this round) and at the
// round cap.  Returns 1 to stop, 0 to continue.
int oracle_should_stop(int64_t hits_prev, int64_t hits_cur, int64_t updates, int round,
                       int max_rounds) {
  if (hits_cur <= hits_prev) return 1;
  if (updates == 0) return 1;
  if (round >= max_rounds) return 1;
  return 0;
}

// The other terminations the paper names among K-NN descent implementations
// (Section 1.2, Table 1, and Section 1.3, item (b)):
//   rule 1, "no possible update": stop after the first round that changed no
//           list (a fixed point of the round map);
//   rule 2, the delta-proportion rule of Dong et al.: stop after the first
//           round whose update count is at most delta * n * K (the product
//           taken in FP64, left to right);
// and rule 0 is the statistical criterion above.  Every rule also stops at
// the round cap.  Returns 1 to stop; *capped is set when only the cap
// stopped the run.
int oracle_stop_rule(int rule, double delta, int64_t n, int K, int64_t hits_prev, int64_t hits_cur,
                     int64_t updates, int round, int max_rounds, int* capped) {
  bool rule_stops;
  if (rule == 1)
    rule_stops = updates == 0;
  else if (rule == 2)
    rule_stops = (double)updates <= delta * (double)n * (double)K;
  else
    rule_stops = hits_cur <= hits_prev || updates == 0;
  if (capped) *capped = !rule_stops && round >= max_rounds;
  return rule_stops || round >= max_rounds;
}

// Whole descent: validate, log table, random K-out graph, FCR of the initial
// graph, then synchronous rounds until the stop rule fires.
//   points: [n][d+1] row-major, FP32 (dtype 0) or FP64 (dtype 1); widened to
//           FP64 exactly, never renormalised; every coordinate must be finite
//           and > 0 (the paper's points lie in the open simplex), or for the
//           other comparators lie in their domain (points_ok).
//   M <= 0 selects the default sample size min(n, 10000).
//   Per-round outputs have max_rounds+1 entries; entry 0 is the initial graph.
// Returns 0, 1 when the round cap stopped the run, or a negative error.
//   stop_rule / delta: see oracle_stop_rule (0 = the paper's criterion).
//   cmp: the comparator (CMP_KL is the paper's).
int oracle_build(const void* points, int dtype, int64_t n, int d, int K, uint64_t seed,
                 int64_t M, int max_rounds, int threads, int32_t* out_idx, double* out_keys,
                 int64_t* out_updates, int64_t* out_hits, int64_t* out_evals,
                 int32_t* out_rounds, double* out_seconds, int stop_rule, double delta, int cmp) {
  if (!points || !out_idx || n < 2 || d < 1 || K < 2 || K > n - 1 || max_rounds < 1 ||
      (dtype != 0 && dtype != 1) || n > ((int64_t)1 << 30) || stop_rule < 0 || stop_rule > 2 ||
      !(delta >= 0.0) || !std::isfinite(delta) || !cmp_valid(cmp))
    return ORC_ERR_ARG;
  const int D = d + 1;
  const size_t cnt = (size_t)n * D;
  auto t0 = std::chrono::steady_clock::now();
  std::vector<double> P(cnt), L(cnt);
  if (dtype == 0) {
    const float* p = (const float*)points;
    for (size_t i = 0; i < cnt; ++i) P[i] = (double)p[i];
  } else {
    std::memcpy(P.data(), points, cnt * sizeof(double));
  }
  if (!points_ok(cmp, P.data(), cnt)) return ORC_ERR_DOMAIN;
  if (M <= 0) M = std::min<int64_t>(n, 10000);
  if (cmp == CMP_KL || cmp == CMP_KL_REVERSE) oracle_log_table(P.data(), (int64_t)cnt, L.data(), threads);

  std::vector<int32_t> F((size_t)n * K), Fn((size_t)n * K);
  std::vector<double> keys((size_t)n * K), keysn((size_t)n * K);
  oracle_initial_graph(P.data(), L.data(), n, D, K, seed, F.data(), keys.data(), threads, cmp);
  int64_t hits_prev = oracle_fcr(F.data(), n, K, seed, 0, M);
  auto secs = [](std::chrono::steady_clock::time_point a) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - a).count();
  };
  if (out_updates) out_updates[0] = 0;
  if (out_hits) out_hits[0] = hits_prev;
  if (out_evals) out_evals[0] = 0;
  if (out_seconds) out_seconds[0] = secs(t0);

  int status = ORC_OK;
  int r = 0;
  for (;;) {
    ++r;
    auto tr = std::chrono::steady_clock::now();
    int64_t upd = 0, ev = 0;
    oracle_round(P.data(), L.data(), n, D, K, F.data(), keys.data(), Fn.data(), keysn.data(),
                 &upd, &ev, threads, cmp);
    F.swap(Fn);
    keys.swap(keysn);
    int64_t hits = oracle_fcr(F.data(), n, K, seed, r, M);
    if (out_updates) out_updates[r] = upd;
    if (out_hits) out_hits[r] = hits;
    if (out_evals) out_evals[r] = ev;
    if (out_seconds) out_seconds[r] = secs(tr);
    int capped = 0;
    if (oracle_stop_rule(stop_rule, delta, n, K, hits_prev, hits, upd, r, max_rounds, &capped)) {
      if (capped) status = ORC_WARN_MAX_ROUNDS;
      break;
    }
    hits_prev = hits;
  }
  std::memcpy(out_idx, F.data(), F.size() * sizeof(int32_t));
  if (out_keys) std::memcpy(out_keys, keys.data(), keys.size() * sizeof(double));
  if (out_rounds) *out_rounds = r;
  return status;
}

}  // extern "C"
