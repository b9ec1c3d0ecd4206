// Device-side building blocks for gfx950 (wave64): counter-based hashing, the
// correctly rounded FP64 log, the canonical KL key, order-preserving key bits
// and wave-level bitonic sort/merge of (key, index) pairs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "knnd_internal.h"

namespace knnd {

constexpr int WAVE = 64;
constexpr uint32_t IDMASK = 0x3FFFFFFFu;   // point index (n < 2^30)
constexpr uint32_t EXCLBIT = 0x40000000u;  // hash-table entry: x itself or a current friend
constexpr uint32_t NEWBIT = 0x80000000u;   // list entry / edge that is new this round
constexpr uint32_t EMPTY = 0xFFFFFFFFu;    // free hash-table slot
constexpr uint64_t KEY_SENTINEL = ~0ull;   // sorts after every finite key

// ---------------------------------------------------------------------------
// Counter-based randomness: SplitMix64 finalizer (Steele, Lea & Flood 2014;
// Stafford's variant-13 constants) chained over (seed, tag, a, b).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t hash4(uint64_t s, uint64_t t, uint64_t a, uint64_t b) {
  return mix64(mix64(mix64(s ^ (t * 0x9E3779B97F4A7C15ull)) ^ a) ^ b);
}

// floor(h * m / 2^64)
__device__ __forceinline__ uint64_t bound(uint64_t h, uint64_t m) { return __umul64hi(h, m); }

// ---------------------------------------------------------------------------
// Correctly rounded natural log in FP64.
// x = 2^e * m with m in [sqrt(2)/2, sqrt(2)]; log m = 2 atanh(s),
// s = (m-1)/(m+1), |s| <= 0.1716, and 2 atanh(s) = 2 s sum_k s^(2k)/(2k+1).
// Everything after the exact reduction runs in double-double (about 104
// significant bits), so the final rounding to FP64 is the correct one unless
// log x lies within ~2^-100 (relative) of a rounding boundary.
// ---------------------------------------------------------------------------
struct dd {
  double h, l;
};

__device__ __forceinline__ dd two_sum(double a, double b) {
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}
__device__ __forceinline__ dd quick_two_sum(double a, double b) {
  double s = a + b;
  return {s, b - (s - a)};
}
__device__ __forceinline__ dd two_prod(double a, double b) {
  double p = a * b;
  return {p, fma(a, b, -p)};
}
__device__ __forceinline__ dd dd_add(dd a, dd b) {
  dd s = two_sum(a.h, b.h);
  dd t = two_sum(a.l, b.l);
  double e = s.l + t.h;
  s = quick_two_sum(s.h, e);
  return quick_two_sum(s.h, s.l + t.l);
}
__device__ __forceinline__ dd dd_mul(dd a, dd b) {
  dd p = two_prod(a.h, b.h);
  double e = p.l + (a.h * b.l + a.l * b.h);
  return quick_two_sum(p.h, e);
}
__device__ __forceinline__ dd dd_mul_d(dd a, double b) {
  dd p = two_prod(a.h, b);
  return quick_two_sum(p.h, p.l + a.l * b);
}

// 1/(2k+1) for k = 0..22 as double-double pairs: hi = 1/(2k+1) rounded, lo =
// (1 - hi (2k+1)) / (2k+1) rounded (1 - hi (2k+1) is exact), the values the
// series below would otherwise form with two divisions per term.
static __constant__ const dd kOddRecip[23] = {
    {0x1.0000000000000p+0, 0.0},
    {0x1.5555555555555p-2, 0x1.5555555555555p-56},
    {0x1.999999999999ap-3, -0x1.999999999999ap-57},
    {0x1.2492492492492p-3, 0x1.2492492492492p-57},
    {0x1.c71c71c71c71cp-4, 0x1.c71c71c71c71cp-58},
    {0x1.745d1745d1746p-4, -0x1.745d1745d1746p-59},
    {0x1.3b13b13b13b14p-4, -0x1.3b13b13b13b14p-58},
    {0x1.1111111111111p-4, 0x1.1111111111111p-60},
    {0x1.e1e1e1e1e1e1ep-5, 0x1.e1e1e1e1e1e1ep-61},
    {0x1.af286bca1af28p-5, 0x1.af286bca1af28p-59},
    {0x1.8618618618618p-5, 0x1.8618618618618p-59},
    {0x1.642c8590b2164p-5, 0x1.642c8590b2164p-60},
    {0x1.47ae147ae147bp-5, -0x1.eb851eb851eb8p-61},
    {0x1.2f684bda12f68p-5, 0x1.2f684bda12f68p-59},
    {0x1.1a7b9611a7b96p-5, 0x1.1a7b9611a7b96p-61},
    {0x1.0842108421084p-5, 0x1.0842108421084p-60},
    {0x1.f07c1f07c1f08p-6, -0x1.f07c1f07c1f08p-61},
    {0x1.d41d41d41d41dp-6, 0x1.0750750750750p-60},
    {0x1.bacf914c1bad0p-6, -0x1.bacf914c1bad0p-60},
    {0x1.a41a41a41a41ap-6, 0x1.0690690690690p-60},
    {0x1.8f9c18f9c18fap-6, -0x1.f3831f3831f38p-61},
    {0x1.7d05f417d05f4p-6, 0x1.7d05f417d05f4p-62},
    {0x1.6c16c16c16c17p-6, -0x1.f49f49f49f49fp-61},
};

__device__ inline double crlog(double x) {
  // x is finite and > 0 (validated by the caller).
  int e = 0;
  if (x < 0x1p-1022) {  // subnormal: scale into the normal range first
    x *= 0x1p54;
    e = -54;
  }
  uint64_t b = (uint64_t)__double_as_longlong(x);
  e += (int)((b >> 52) & 0x7ff) - 1023;
  double m = __longlong_as_double((long long)((b & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull));
  if (m > 0x1.6a09e667f3bcdp+0) {  // sqrt(2)
    m *= 0.5;
    e += 1;
  }
  const double f = m - 1.0;       // exact (Sterbenz)
  const dd den = two_sum(m, 1.0);  // m + 1 exactly
  // s = f / (m+1) in double-double
  const double q1 = f / den.h;
  const dd p = dd_mul_d(den, q1);
  const dd r = dd_add(dd{f, 0.0}, dd{-p.h, -p.l});
  const double q2 = r.h / den.h;
  const dd s = quick_two_sum(q1, q2);
  const dd w = dd_mul(s, s);
  // Horner on sum_{k=0}^{22} w^k / (2k+1); w <= 0.0295, so the first omitted
  // term is below 2^-114 of the sum.
  const int N = 22;
  dd acc = kOddRecip[N];
  for (int k = N - 1; k >= 0; --k) acc = dd_add(dd_mul(acc, w), kOddRecip[k]);
  dd y = dd_mul(s, acc);
  y.h *= 2.0;
  y.l *= 2.0;
  // ln 2 as the nearest double plus the nearest double to the remainder
  const dd ln2 = {0x1.62e42fefa39efp-1, 0x1.abc9e3b39803fp-56};
  const dd E = dd_mul_d(ln2, (double)e);
  const dd t = dd_add(E, y);
  return t.h + t.l;
}

// ---------------------------------------------------------------------------
// Comparator kinds of the key fold (each point has its own order on the
// others, Section 2.1).  L is the comparator's feature table: log x for the
// two KL kinds, sqrt x for the Hellinger comparator, x itself for the
// Euclidean one.  With x the receiver (first argument) and z the candidate:
//   CK_KL   acc = fma(x_i, Lx_i - Lz_i, acc)    D(x||z)
//   CK_REV  acc = fma(z_i, Lz_i - Lx_i, acc)    D(z||x)
//   CK_SQ   t = Lx_i - Lz_i; acc = fma(t, t, acc)   squared distance of the features
// i ascending, from +0.0.
// ---------------------------------------------------------------------------
// (CK_* and the table kinds TK_* are declared in knnd_internal.h)

// One term; w is the weighing coordinate (x_i for CK_KL, z_i for CK_REV,
// unused for CK_SQ).
template <int CK>
__device__ __forceinline__ double key_term(double w, double lx, double lz, double acc) {
  if constexpr (CK == CK_KL) {
    return fma(w, lx - lz, acc);
  } else if constexpr (CK == CK_REV) {
    return fma(w, lz - lx, acc);
  } else {
    const double t = lx - lz;
    return fma(t, t, acc);
  }
}

// ---------------------------------------------------------------------------
// Canonical key of comparator kind CK (CK_KL: acc = fma(x_i, Lx_i - Lz_i,
// acc), i ascending, from +0.0).
// Adding +0.0 at the end turns a -0.0 into +0.0 so that the bit order below
// agrees with FP64 comparison.
// The rows are read in chunks of 8 coordinates, the next chunk requested
// before the current one is used, every read unconditional (so that no read
// waits for the one before it).  Reads reach element D + 22 of each row: the
// arrays must stay readable that far past their last row (P and L carry 64
// elements of tail padding).  lx and lz must be 16-byte aligned.  pw is the
// weighing point row (x's for CK_KL, z's for CK_REV; not read for CK_SQ).
// ---------------------------------------------------------------------------
template <typename PT, int CK = CK_KL>
struct KeyChunk {
  double w[8], l[8], z[8];
  __device__ __forceinline__ void load(const PT* __restrict__ pw, const double* __restrict__ lx,
                                       const double* __restrict__ lz, int c0) {
    const double2* lx2 = reinterpret_cast<const double2*>(lx + c0);
    const double2* lz2 = reinterpret_cast<const double2*>(lz + c0);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double2 a = lx2[j], b = lz2[j];
      l[2 * j] = a.x;
      l[2 * j + 1] = a.y;
      z[2 * j] = b.x;
      z[2 * j + 1] = b.y;
    }
    if constexpr (CK != CK_SQ) {
#pragma unroll
      for (int j = 0; j < 8; ++j) w[j] = (double)pw[c0 + j];
    }
  }
  __device__ __forceinline__ double fold(double acc, int c0, int D) const {
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (c0 + j < D) acc = key_term<CK>(w[j], l[j], z[j], acc);
    return acc;
  }
};

template <typename PT, int CK = CK_KL>
__device__ __forceinline__ double canonical_key(const PT* __restrict__ pw,
                                                const double* __restrict__ lx,
                                                const double* __restrict__ lz, int D) {
  double acc = 0.0;
  KeyChunk<PT, CK> a, b;
  a.load(pw, lx, lz, 0);
  for (int c0 = 0; c0 < D; c0 += 16) {
    b.load(pw, lx, lz, c0 + 8);
    acc = a.fold(acc, c0, D);
    a.load(pw, lx, lz, c0 + 16);
    acc = b.fold(acc, c0 + 8, D);
  }
  return acc + 0.0;
}

// Key of x against z for a comparator kind known only at run time (uniform
// across the wave): rows of P [n][D] and of the feature table L [n][Dp].
template <typename PT>
__device__ __forceinline__ double key_of_kind(int ck, const PT* __restrict__ P, int64_t x, int64_t z,
                                              const double* __restrict__ L, int D, int Dp) {
  const double* lx = L + x * Dp;
  const double* lz = L + z * Dp;
  if (ck == CK_REV) return canonical_key<PT, CK_REV>(P + z * D, lx, lz, D);
  if (ck == CK_SQ) return canonical_key<PT, CK_SQ>(P + x * D, lx, lz, D);
  return canonical_key<PT, CK_KL>(P + x * D, lx, lz, D);
}

// The same key with x's row (as FP64) and its logs staged in LDS: sx and sl
// must hold at least D + 16 readable entries (those past D are never used).
__device__ __forceinline__ double canonical_key_lds(const double* sx, const double* sl,
                                                    const double* __restrict__ lz, int D) {
  double acc = 0.0;
  double za[8], zb[8];
  auto load = [&](double* z, int c0) {
    const double2* lz2 = reinterpret_cast<const double2*>(lz + c0);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double2 v = lz2[j];
      z[2 * j] = v.x;
      z[2 * j + 1] = v.y;
    }
  };
  auto fold = [&](const double* z, int c0) {
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (c0 + j < D) acc = fma(sx[c0 + j], sl[c0 + j] - z[j], acc);
  };
  load(za, 0);
  for (int c0 = 0; c0 < D; c0 += 16) {
    load(zb, c0 + 8);
    fold(za, c0);
    load(za, c0 + 16);
    fold(zb, c0 + 8);
  }
  return acc + 0.0;
}

// Order-preserving map FP64 -> uint64 (for non-NaN values, with -0 == +0
// already canonicalised): a < b  <=>  key_bits(a) < key_bits(b).
__device__ __forceinline__ uint64_t key_bits(double k) {
  const uint64_t u = (uint64_t)__double_as_longlong(k);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double bits_key(uint64_t u) {
  return __longlong_as_double((long long)((u >> 63) ? (u & 0x7FFFFFFFFFFFFFFFull) : ~u));
}

// (key, index) order; flag bits above IDMASK are ignored.
__device__ __forceinline__ bool ke_less(uint64_t ka, uint32_t ia, uint64_t kb, uint32_t ib) {
  return ka < kb || (ka == kb && (ia & IDMASK) < (ib & IDMASK));
}

// ---------------------------------------------------------------------------
// Wave-level primitives (64 lanes).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint32_t rank_in(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
  const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src, WAVE);
  const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src, WAVE);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m, WAVE);
  const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m, WAVE);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint32_t shfl_u32(uint32_t v, int src) {
  return (uint32_t)__shfl((int)v, src, WAVE);
}
__device__ __forceinline__ uint32_t shfl_xor_u32(uint32_t v, int m) {
  return (uint32_t)__shfl_xor((int)v, m, WAVE);
}

// One compare-exchange step between lane and lane^stride; `keep_min` says
// whether this lane keeps the smaller element.
__device__ __forceinline__ void cx_step(uint64_t& k, uint32_t& id, int stride, bool keep_min) {
  const uint64_t pk = shfl_xor_u64(k, stride);
  const uint32_t pid = shfl_xor_u32(id, stride);
  const bool take = keep_min ? ke_less(pk, pid, k, id) : ke_less(k, id, pk, pid);
  if (take) {
    k = pk;
    id = pid;
  }
}

// Ascending bitonic sort of one (key, id) per lane across the wave.
__device__ __forceinline__ void wave_sort(uint64_t& k, uint32_t& id) {
  const int lane = lane_id();
#pragma unroll
  for (int size = 2; size <= WAVE; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const bool asc = (lane & size) == 0;
      const bool lower = (lane & stride) == 0;
      cx_step(k, id, stride, lower == asc);
    }
  }
}

// a (ascending across lanes) <- the 64 smallest of a and b (b ascending).
__device__ __forceinline__ void wave_merge(uint64_t& ak, uint32_t& aid, uint64_t bk, uint32_t bid) {
  const int lane = lane_id();
  const uint64_t rk = shfl_u64(bk, WAVE - 1 - lane);
  const uint32_t rid = shfl_u32(bid, WAVE - 1 - lane);
  if (ke_less(rk, rid, ak, aid)) {
    ak = rk;
    aid = rid;
  }
#pragma unroll
  for (int stride = WAVE / 2; stride > 0; stride >>= 1) cx_step(ak, aid, stride, (lane & stride) == 0);
}

// Insert one wave-uniform entry (ck, ci) into the ascending list held one
// entry per lane; the last lane's entry drops out.
__device__ __forceinline__ void wave_insert(uint64_t& lk, uint32_t& li, uint64_t ck, uint32_t ci) {
  const int lane = lane_id();
  const bool move = ke_less(ck, ci, lk, li);  // the new entry goes before mine
  const uint64_t pk = shfl_u64(lk, lane > 0 ? lane - 1 : 0);
  const uint32_t pi = shfl_u32(li, lane > 0 ? lane - 1 : 0);
  const int pos = (int)__popcll(__ballot(!move));
  if (move) {
    if (lane == pos) {
      lk = ck;
      li = ci;
    } else {
      lk = pk;
      li = pi;
    }
  }
}

}  // namespace knnd
