// Exact K nearest neighbours of query points by exhaustive comparison: the
// problem statement itself (Section 2.3), used to measure the descent's
// accuracy (Section 4.4: the share of true nearest neighbours found).
//
// For each query q every other point p gets its canonical key k(q, p) under
// the comparator (the same FP64 fold as the descent; D(q||p) for KL) and the
// K smallest (key, index) pairs are returned in order.  Three kernels:
//   bound    (when the caller gives no bound) each thread keeps the best
//            pair of its share of the points; the K-th smallest of those
//            minima is a pair that K distinct points reach, so it bounds the
//            K-th smallest pair from above;
//   collect  every pair at or below the bound goes to the query's buffer;
//            a full buffer tightens the bound to the K-th smallest pair it
//            holds (strictly smaller, since pairs are distinct) and the
//            query is collected again;
//   select   the buffer is sorted down to its K smallest pairs.
// Eight queries share a block: their rows are staged in LDS and each point's
// log row is read once for all of them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "knnd.h"
#include "knnd_device.h"
#include "knnd_internal.h"

namespace knnd {

constexpr int XQ = 8;          // queries per block
constexpr int XCAP = 4096;     // collected pairs per query
constexpr int XMAXD = 256;     // coordinates supported
constexpr int XROW = XMAXD + 16;

__device__ __forceinline__ bool pair_le(uint64_t ka, uint32_t ia, uint64_t kb, uint32_t ib) {
  return ka < kb || (ka == kb && ia <= ib);
}

// Stage the rows of queries qb..qb+XQ-1 (as FP64) and their logs in LDS.
template <typename PT>
__device__ void stage_queries(const PT* P, const double* L, int D, int Dp, const int32_t* queries, int64_t nq,
                              int64_t qb, double (*sx)[XROW], double (*sl)[XROW], int32_t* sq) {
  for (int t = threadIdx.x; t < XQ * XROW; t += blockDim.x) {
    const int j = t / XROW, i = t - j * XROW;
    const int64_t qi = qb + j;
    double xv = 0.0, lv = 0.0;
    if (qi < nq && i < D) {
      const int64_t q = queries[qi];
      xv = (double)P[q * D + i];
      lv = L[q * Dp + i];
    }
    sx[j][i] = xv;
    sl[j][i] = lv;
  }
  if (threadIdx.x < XQ) sq[threadIdx.x] = qb + threadIdx.x < nq ? queries[qb + threadIdx.x] : -1;
  __syncthreads();
}

// Keys of point p for the XQ staged queries, fold kind CK (CK_KL:
// acc_j = fold_i fma(x_j,i, l_j,i - L_p,i)).  The point's feature row lp (and
// for CK_REV its point row pp) is read 8 coordinates at a time (rows stay
// inside the arrays' tail padding).
template <int CK, typename PT>
__device__ __forceinline__ void point_keys(const double* __restrict__ lp, const PT* __restrict__ pp, int D,
                                           const double (*sx)[XROW], const double (*sl)[XROW], double (&acc)[XQ]) {
#pragma unroll
  for (int j = 0; j < XQ; ++j) acc[j] = 0.0;
  for (int c0 = 0; c0 < D; c0 += 8) {
    double z[8], w[8];
    const double2* l2 = reinterpret_cast<const double2*>(lp + c0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double2 v = l2[k];
      z[2 * k] = v.x;
      z[2 * k + 1] = v.y;
    }
    if constexpr (CK == CK_REV) {
#pragma unroll
      for (int k = 0; k < 8; ++k) w[k] = (double)pp[c0 + k];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (c0 + k < D) {
#pragma unroll
        for (int j = 0; j < XQ; ++j) {
          if constexpr (CK == CK_KL)
            acc[j] = key_term<CK>(sx[j][c0 + k], sl[j][c0 + k], z[k], acc[j]);
          else
            acc[j] = key_term<CK>(w[k], sl[j][c0 + k], z[k], acc[j]);
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < XQ; ++j) acc[j] = acc[j] + 0.0;
}

// The K smallest of one (key, id) per thread of a 256-thread block, merged
// into wave 0 (ascending across its lanes).
__device__ void block_smallest(uint64_t k, uint32_t id, uint64_t (*sk)[WAVE], uint32_t (*si)[WAVE],
                               uint64_t& lk, uint32_t& li) {
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  wave_sort(k, id);
  if (wave > 0) {
    sk[wave - 1][lane] = k;
    si[wave - 1][lane] = id;
  }
  __syncthreads();
  lk = k;
  li = id;
  if (wave == 0)
    for (int w = 0; w < 3; ++w) wave_merge(lk, li, sk[w][lane], si[w][lane]);
  __syncthreads();
}

template <typename PT, int CK>
__global__ __launch_bounds__(256) void k_exact_bound(const PT* __restrict__ P, const double* __restrict__ L,
                                                     int64_t n, int D, int Dp, int K,
                                                     const int32_t* __restrict__ queries, int64_t nq,
                                                     uint64_t* __restrict__ tk, uint32_t* __restrict__ ti) {
  __shared__ double sx[XQ][XROW], sl[XQ][XROW];
  __shared__ int32_t sq[XQ];
  __shared__ uint64_t sk[3][WAVE];
  __shared__ uint32_t si[3][WAVE];
  const int64_t qb = (int64_t)blockIdx.x * XQ;
  stage_queries(P, L, D, Dp, queries, nq, qb, sx, sl, sq);
  uint64_t mk[XQ];
  uint32_t mi[XQ];
#pragma unroll
  for (int j = 0; j < XQ; ++j) {
    mk[j] = KEY_SENTINEL;
    mi[j] = IDMASK;
  }
  for (int64_t p = threadIdx.x; p < n; p += blockDim.x) {
    double acc[XQ];
    point_keys<CK>(L + p * Dp, P + p * D, D, sx, sl, acc);
#pragma unroll
    for (int j = 0; j < XQ; ++j) {
      const uint64_t kb = key_bits(acc[j]);
      if (p != sq[j] && ke_less(kb, (uint32_t)p, mk[j], mi[j])) {
        mk[j] = kb;
        mi[j] = (uint32_t)p;
      }
    }
  }
  for (int j = 0; j < XQ; ++j) {
    uint64_t lk;
    uint32_t li;
    block_smallest(mk[j], mi[j], sk, si, lk, li);
    if ((int)threadIdx.x == K - 1 && qb + j < nq) {  // lane K-1 of wave 0
      tk[qb + j] = lk;
      ti[qb + j] = li;
    }
  }
}

// Collect the pairs at or below each query's bound.  `sel` lists the
// positions (in queries) still to collect; cnt[q] receives the number of
// pairs at or below the bound (possibly more than XCAP: then only XCAP kept).
template <typename PT, int CK>
__global__ __launch_bounds__(256) void k_exact_collect(const PT* __restrict__ P, const double* __restrict__ L,
                                                       int64_t n, int D, int Dp,
                                                       const int32_t* __restrict__ queries,
                                                       const int32_t* __restrict__ sel, int64_t nsel,
                                                       const uint64_t* __restrict__ tk,
                                                       const uint32_t* __restrict__ ti, uint64_t* __restrict__ ck,
                                                       uint32_t* __restrict__ ci, int32_t* __restrict__ cnt) {
  __shared__ double sx[XQ][XROW], sl[XQ][XROW];
  __shared__ int32_t sq[XQ];
  __shared__ int32_t spos[XQ];
  __shared__ int s_cnt[XQ];
  __shared__ uint64_t s_tk[XQ];
  __shared__ uint32_t s_ti[XQ];
  const int64_t qb = (int64_t)blockIdx.x * XQ;
  // gather this block's query positions into a contiguous staging list
  if (threadIdx.x < XQ) {
    const int64_t s = qb + threadIdx.x;
    const int pos = s < nsel ? sel[s] : -1;
    spos[threadIdx.x] = pos;
    s_cnt[threadIdx.x] = 0;
    s_tk[threadIdx.x] = pos >= 0 ? tk[pos] : 0;
    s_ti[threadIdx.x] = pos >= 0 ? ti[pos] : 0;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < XQ * XROW; t += blockDim.x) {
    const int j = t / XROW, i = t - j * XROW;
    double xv = 0.0, lv = 0.0;
    if (spos[j] >= 0 && i < D) {
      const int64_t q = queries[spos[j]];
      xv = (double)P[q * D + i];
      lv = L[q * Dp + i];
    }
    sx[j][i] = xv;
    sl[j][i] = lv;
  }
  if (threadIdx.x < XQ) sq[threadIdx.x] = spos[threadIdx.x] >= 0 ? queries[spos[threadIdx.x]] : -1;
  __syncthreads();
  for (int64_t p = threadIdx.x; p < n; p += blockDim.x) {
    double acc[XQ];
    point_keys<CK>(L + p * Dp, P + p * D, D, sx, sl, acc);
#pragma unroll
    for (int j = 0; j < XQ; ++j) {
      if (spos[j] < 0 || p == sq[j]) continue;
      const uint64_t kb = key_bits(acc[j]);
      if (pair_le(kb, (uint32_t)p, s_tk[j], s_ti[j])) {
        const int at = atomicAdd(&s_cnt[j], 1);
        if (at < XCAP) {
          ck[(int64_t)spos[j] * XCAP + at] = kb;
          ci[(int64_t)spos[j] * XCAP + at] = (uint32_t)p;
        }
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < XQ && spos[threadIdx.x] >= 0) cnt[spos[threadIdx.x]] = s_cnt[threadIdx.x];
}

// The K smallest pairs of each selected query's buffer (count capped at
// XCAP); `tighten` != 0: only the K-th of them is stored, as the new bound.
__global__ __launch_bounds__(256) void k_exact_select(const int32_t* __restrict__ sel, int64_t nsel, int K,
                                                      const uint64_t* __restrict__ ck,
                                                      const uint32_t* __restrict__ ci,
                                                      const int32_t* __restrict__ cnt, int tighten,
                                                      uint64_t* __restrict__ tk, uint32_t* __restrict__ ti,
                                                      int32_t* __restrict__ out_idx, double* __restrict__ out_kl) {
  __shared__ uint64_t sk[3][WAVE];
  __shared__ uint32_t si[3][WAVE];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  for (int64_t s = blockIdx.x; s < nsel; s += gridDim.x) {
    const int pos = sel[s];
    const int c = min(cnt[pos], XCAP);
    uint64_t lk = KEY_SENTINEL;
    uint32_t li = IDMASK;
    for (int b0 = wave * WAVE; b0 < c; b0 += 4 * WAVE) {
      const bool ok = b0 + lane < c;
      uint64_t bk = ok ? ck[(int64_t)pos * XCAP + b0 + lane] : KEY_SENTINEL;
      uint32_t bi = ok ? ci[(int64_t)pos * XCAP + b0 + lane] : IDMASK;
      wave_sort(bk, bi);
      wave_merge(lk, li, bk, bi);
    }
    if (wave > 0) {
      sk[wave - 1][lane] = lk;
      si[wave - 1][lane] = li;
    }
    __syncthreads();
    if (wave == 0) {
      for (int w = 0; w < 3; ++w) wave_merge(lk, li, sk[w][lane], si[w][lane]);
      if (tighten) {
        if (lane == K - 1) {
          tk[pos] = lk;
          ti[pos] = li;
        }
      } else if (lane < K) {
        out_idx[(int64_t)pos * K + lane] = (int32_t)li;
        if (out_kl) out_kl[(int64_t)pos * K + lane] = bits_key(lk);
      }
    }
    __syncthreads();
  }
}

__global__ void k_bound_from_keys(const double* __restrict__ tau, int64_t nq, uint64_t* __restrict__ tk,
                                  uint32_t* __restrict__ ti) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q < nq) {
    tk[q] = key_bits(tau[q] + 0.0);
    ti[q] = IDMASK;
  }
}

__global__ void k_check_queries(const int32_t* __restrict__ queries, int64_t nq, int64_t n, int32_t* bad) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q < nq && (queries[q] < 0 || queries[q] >= n)) atomicOr(bad, 1);
}

}  // namespace knnd

namespace {

int map_err_x(hipError_t e) { return e == hipErrorOutOfMemory ? KNND_ERR_NOMEM : KNND_ERR_DEVICE; }

#define KNND_XHIP(x)                           \
  do {                                         \
    hipError_t e_ = (x);                       \
    if (e_ != hipSuccess) return map_err_x(e_); \
  } while (0)

struct XBufs {
  void* P = nullptr;
  double* L = nullptr;
  int32_t* q = nullptr;
  double* tau = nullptr;
  uint64_t* tk = nullptr;
  uint32_t* ti = nullptr;
  uint64_t* ck = nullptr;
  uint32_t* ci = nullptr;
  int32_t* cnt = nullptr;
  int32_t* sel = nullptr;
  int32_t* idx = nullptr;
  double* kl = nullptr;
  int32_t* flag = nullptr;
  hipStream_t st = nullptr;
  ~XBufs() {
    void* b[] = {P, L, q, tau, tk, ti, ck, ci, cnt, sel, idx, kl, flag};
    (void)hipStreamSynchronize(st);  // the blocks go back to the cache
    for (void* p : b) knnd::pool_free(p);
  }
};

template <typename PT, int CK>
int exact_knn(const void* points, int64_t n, int32_t d, int32_t K, int tk, const int32_t* queries, int64_t nq,
              const double* tau, int32_t on_device, hipStream_t st, int32_t* out_idx, double* out_kl) {
  using namespace knnd;
  const int D = d + 1, Dp = (D + 1) & ~1;
  const size_t esz = sizeof(PT);
  const hipMemcpyKind h2d = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  const hipMemcpyKind d2h = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  XBufs b;
  b.st = st;
  KNND_XHIP(knnd::pmalloc(&b.P, ((size_t)n * D + HUB_MAXD) * esz));
  KNND_XHIP(knnd::pmalloc(&b.L, ((size_t)n * Dp + HUB_MAXD) * 8));
  KNND_XHIP(knnd::pmalloc(&b.q, (size_t)nq * 4));
  KNND_XHIP(knnd::pmalloc(&b.tk, (size_t)nq * 8));
  KNND_XHIP(knnd::pmalloc(&b.ti, (size_t)nq * 4));
  KNND_XHIP(knnd::pmalloc(&b.ck, (size_t)nq * XCAP * 8));
  KNND_XHIP(knnd::pmalloc(&b.ci, (size_t)nq * XCAP * 4));
  KNND_XHIP(knnd::pmalloc(&b.cnt, (size_t)nq * 4));
  KNND_XHIP(knnd::pmalloc(&b.sel, (size_t)nq * 4));
  KNND_XHIP(knnd::pmalloc(&b.flag, 16));
  if (!on_device) {
    KNND_XHIP(knnd::pmalloc(&b.idx, (size_t)nq * K * 4));
    if (out_kl) KNND_XHIP(knnd::pmalloc(&b.kl, (size_t)nq * K * 8));
  }
  int32_t* didx = on_device ? out_idx : b.idx;
  double* dkl = on_device ? out_kl : b.kl;
  KNND_XHIP(hipMemcpyAsync(b.P, points, (size_t)n * D * esz, h2d, st));
  KNND_XHIP(hipMemsetAsync(static_cast<char*>(b.P) + (size_t)n * D * esz, 0, HUB_MAXD * esz, st));
  KNND_XHIP(hipMemsetAsync(b.L + (size_t)n * Dp, 0, HUB_MAXD * 8, st));
  KNND_XHIP(hipMemcpyAsync(b.q, queries, (size_t)nq * 4, h2d, st));
  KNND_XHIP(hipMemsetAsync(b.flag, 0, 16, st));
  // log table and domain check (the descent's kernel), query range check
  Ctx c;
  c.P = b.P;
  c.L = b.L;
  c.n = n;
  c.D = D;
  c.Dp = Dp;
  c.dtype = sizeof(PT) == 4 ? KNND_F32 : KNND_F64;
  c.tk = tk;
  c.stream = st;
  KNND_XHIP(launch_log_table(c, b.flag));
  hipLaunchKernelGGL(k_check_queries, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, st, b.q, nq, n,
                     b.flag + 1);
  KNND_XHIP(hipGetLastError());
  int32_t bad[2] = {0, 0};
  KNND_XHIP(hipMemcpyAsync(bad, b.flag, 8, hipMemcpyDeviceToHost, st));
  KNND_XHIP(hipStreamSynchronize(st));
  c.P = nullptr;  // owned by b
  c.L = nullptr;
  if (bad[0]) return KNND_ERR_DOMAIN;
  if (bad[1]) return KNND_ERR_ARG;

  const unsigned qblocks = (unsigned)((nq + XQ - 1) / XQ);
  if (tau) {
    KNND_XHIP(knnd::pmalloc(&b.tau, (size_t)nq * 8));
    KNND_XHIP(hipMemcpyAsync(b.tau, tau, (size_t)nq * 8, h2d, st));
    hipLaunchKernelGGL(k_bound_from_keys, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, st, b.tau, nq, b.tk,
                       b.ti);
  } else {
    hipLaunchKernelGGL((k_exact_bound<PT, CK>), dim3(qblocks), dim3(256), 0, st, (const PT*)b.P, b.L, n, D, Dp, K, b.q,
                       nq, b.tk, b.ti);
  }
  KNND_XHIP(hipGetLastError());
  // collect every query, then again those whose buffer overflowed (with a
  // tightened bound) until none does
  std::vector<int32_t> sel((size_t)nq), cnt((size_t)nq);
  for (int64_t i = 0; i < nq; ++i) sel[i] = (int32_t)i;
  int64_t nsel = nq;
  for (int pass = 0; nsel > 0; ++pass) {
    if (pass > 64) return KNND_ERR_DEVICE;  // cannot happen: each pass strictly lowers the bound
    KNND_XHIP(hipMemcpyAsync(b.sel, sel.data(), (size_t)nsel * 4, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL((k_exact_collect<PT, CK>), dim3((unsigned)((nsel + XQ - 1) / XQ)), dim3(256), 0, st,
                       (const PT*)b.P, b.L, n, D, Dp, b.q, b.sel, nsel, b.tk, b.ti, b.ck, b.ci, b.cnt);
    KNND_XHIP(hipGetLastError());
    KNND_XHIP(hipMemcpyAsync(cnt.data(), b.cnt, (size_t)nq * 4, hipMemcpyDeviceToHost, st));
    KNND_XHIP(hipStreamSynchronize(st));
    std::vector<int32_t> over;
    for (int64_t s = 0; s < nsel; ++s)
      if (cnt[sel[s]] > XCAP) over.push_back(sel[s]);
    if (over.empty()) break;
    KNND_XHIP(hipMemcpyAsync(b.sel, over.data(), over.size() * 4, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_exact_select, dim3((unsigned)std::min<size_t>(over.size(), 4096)), dim3(256), 0, st, b.sel,
                       (int64_t)over.size(), K, b.ck, b.ci, b.cnt, 1, b.tk, b.ti, nullptr, nullptr);
    KNND_XHIP(hipGetLastError());
    KNND_XHIP(hipStreamSynchronize(st));  // `over` is read by the copy above
    sel = over;
    nsel = (int64_t)over.size();
  }
  // a bound below the K-th key leaves fewer than K pairs: not a bound
  for (int64_t i = 0; i < nq; ++i)
    if (cnt[i] < K) return KNND_ERR_ARG;
  for (int64_t i = 0; i < nq; ++i) sel[i] = (int32_t)i;
  KNND_XHIP(hipMemcpyAsync(b.sel, sel.data(), (size_t)nq * 4, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_exact_select, dim3((unsigned)std::min<int64_t>(nq, 8192)), dim3(256), 0, st, b.sel, nq, K,
                     b.ck, b.ci, b.cnt, 0, b.tk, b.ti, didx, dkl);
  KNND_XHIP(hipGetLastError());
  if (!on_device) {
    KNND_XHIP(hipMemcpyAsync(out_idx, b.idx, (size_t)nq * K * 4, d2h, st));
    if (out_kl) KNND_XHIP(hipMemcpyAsync(out_kl, b.kl, (size_t)nq * K * 8, d2h, st));
  }
  KNND_XHIP(hipStreamSynchronize(st));
  return KNND_OK;
}

}  // namespace

extern "C" int knnd_exact_knn(const void* points, int64_t n, int32_t d, int32_t K, int32_t dtype,
                              int32_t comparator, const int32_t* queries, int64_t nq, const double* tau,
                              int32_t on_device, void* stream, int32_t* out_idx, double* out_kl) {
  if (!points || !queries || !out_idx || nq < 1) return KNND_ERR_ARG;
  if (comparator < KNND_CMP_KL || comparator > KNND_CMP_L2) return KNND_ERR_ARG;
  if (n < 2 || d < 1 || K < 1 || K > 64 || K > n - 1 || n >= (int64_t)knnd::IDMASK_HOST) return KNND_ERR_ARG;
  if (d + 1 > knnd::XMAXD) return KNND_ERR_UNSUPPORTED;
  if (dtype != KNND_F32 && dtype != KNND_F64) return KNND_ERR_ARG;
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return KNND_ERR_DEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return KNND_ERR_DEVICE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int ck = knnd::cmp_fold_kind(comparator), tk = knnd::cmp_table_kind(comparator);
  if (dtype == KNND_F32) {
    if (ck == knnd::CK_REV) return exact_knn<float, knnd::CK_REV>(points, n, d, K, tk, queries, nq, tau, on_device, st, out_idx, out_kl);
    if (ck == knnd::CK_SQ) return exact_knn<float, knnd::CK_SQ>(points, n, d, K, tk, queries, nq, tau, on_device, st, out_idx, out_kl);
    return exact_knn<float, knnd::CK_KL>(points, n, d, K, tk, queries, nq, tau, on_device, st, out_idx, out_kl);
  }
  if (ck == knnd::CK_REV) return exact_knn<double, knnd::CK_REV>(points, n, d, K, tk, queries, nq, tau, on_device, st, out_idx, out_kl);
  if (ck == knnd::CK_SQ) return exact_knn<double, knnd::CK_SQ>(points, n, d, K, tk, queries, nq, tau, on_device, st, out_idx, out_kl);
  return exact_knn<double, knnd::CK_KL>(points, n, d, K, tk, queries, nq, tau, on_device, st, out_idx, out_kl);
}
