// gfx950 kernels for one round of comparator-based K-NN descent with the
// Kullback-Leibler comparator (Baron & Darling, arXiv 2202.00517).
//
// Data layout in HBM (all row-major):
//   P     [n][D]   points as given (FP32 or FP64), D = d+1
//   L     [n][Dp]  FP64 correctly rounded log of P, Dp = D rounded up to even
//                  (16-byte aligned rows for dwordx4 gathers), pad = 0
//   F     [n][K]   uint32: point index | NEWBIT when the edge is new this round
//   keys  [n][K]   FP64 canonical keys of F, ascending per row
//   rowptr[n+1]    int64, col[nK] uint32: co-friend (reverse) lists; col holds
//                  the source index | NEWBIT of that edge
#include "knnd_device.h"
#include "knnd_internal.h"

namespace knnd {

// ---------------------------------------------------------------------------
// Small utility kernels
// ---------------------------------------------------------------------------
__global__ void k_zero_i32(int32_t* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}
__global__ void k_zero_i64(int64_t* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}
// out = F without flag bits
__global__ void k_strip(const uint32_t* __restrict__ F, int64_t cnt, int32_t* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (int32_t)(F[i] & IDMASK);
}
// F = idx | NEWBIT (an externally supplied snapshot: every edge counts as new)
__global__ void k_load_idx(const int32_t* __restrict__ idx, int64_t cnt, uint32_t* __restrict__ F) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x)
    F[i] = ((uint32_t)idx[i] & IDMASK) | NEWBIT;
}

// ---------------------------------------------------------------------------
// a0: log table (and domain check of every coordinate)
// ---------------------------------------------------------------------------
template <typename PT>
__global__ void k_log_table(const PT* __restrict__ P, int64_t n, int D, int Dp, double* __restrict__ L,
                            int32_t* __restrict__ bad) {
  const int64_t total = n * Dp;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = t / Dp;
    const int i = (int)(t - j * Dp);
    double out = 0.0;
    if (i < D) {
      const double v = (double)P[j * D + i];
      if (!(v > 0.0) || isinf(v)) {
        atomicOr(bad, 1);
      } else {
        out = crlog(v);
      }
    }
    L[t] = out;
  }
}

// ---------------------------------------------------------------------------
// a0: random K-out start, one wave per point (Section 3.2).  Draw a of x is
// y = r + (r >= x), r = bound(H(seed,1,x,a), n-1); the first K distinct draws
// are kept, 64 draws at a time (one per lane), then sorted by (key, index).
// ---------------------------------------------------------------------------
template <typename PT>
__global__ __launch_bounds__(256) void k_init_graph(const PT* __restrict__ P, const double* __restrict__ L,
                                                    int64_t n, int D, int Dp, int K, uint64_t seed,
                                                    uint32_t* __restrict__ F, double* __restrict__ keys) {
  __shared__ uint32_t slot[4][WAVE];
  const int wave = threadIdx.x >> 6;
  const int lane = lane_id();
  const int64_t x = (int64_t)blockIdx.x * 4 + wave;
  if (x >= n) return;  // whole wave; no block-level barrier follows
  uint32_t mine = IDMASK;
  int count = 0;
  for (uint64_t a0 = 0; count < K; a0 += WAVE) {
    const uint64_t r = bound(hash4(seed, 1, (uint64_t)x, a0 + lane), (uint64_t)(n - 1));
    const uint32_t y = (uint32_t)(r + (r >= (uint64_t)x ? 1 : 0));
    bool dup = false;
    for (int j = 0; j < count; ++j) dup |= (shfl_u32(mine, j) == y);
    for (int l = 0; l < WAVE - 1; ++l) {
      const uint32_t yl = shfl_u32(y, l);
      dup |= (l < lane) && (yl == y);
    }
    const uint64_t ok = __ballot(!dup);
    const int pos = count + (int)rank_in(ok);
    if (!dup && pos < K) slot[wave][pos] = y;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int nc = min(K, count + (int)__popcll(ok));
    if (lane >= count && lane < nc) mine = slot[wave][lane];
    count = nc;
  }
  uint64_t kb = KEY_SENTINEL;
  uint32_t id = IDMASK;
  if (lane < K) {
    kb = key_bits(canonical_key(P + x * D, L + x * Dp, L + (int64_t)mine * Dp, D));
    id = mine;
  }
  wave_sort(kb, id);
  if (lane < K) {
    F[x * K + lane] = id | NEWBIT;
    keys[x * K + lane] = bits_key(kb);
  }
}

// ---------------------------------------------------------------------------
// a6: friend clustering rate sample (Section 3.3), one thread per sample.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fcr(const uint32_t* __restrict__ F, int64_t n, int K, uint64_t seed,
                                             int64_t round, int64_t M, int64_t* __restrict__ hits) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  bool hit = false;
  if (s < M) {
    const int64_t x = (int64_t)bound(hash4(seed, 2, (uint64_t)round, (uint64_t)s), (uint64_t)n);
    const int av = (int)bound(hash4(seed, 3, (uint64_t)round, (uint64_t)s), (uint64_t)K);
    const int bp = (int)bound(hash4(seed, 4, (uint64_t)round, (uint64_t)s), (uint64_t)(K - 1));
    const int bv = bp + (bp >= av ? 1 : 0);
    const uint32_t y = F[x * K + av] & IDMASK;
    const uint32_t z = F[x * K + bv] & IDMASK;
    for (int j = 0; j < K; ++j)
      hit |= ((F[(int64_t)z * K + j] & IDMASK) == y) || ((F[(int64_t)y * K + j] & IDMASK) == z);
  }
  const uint64_t m = __ballot(hit);
  if (lane_id() == 0 && m) atomicAdd((unsigned long long*)hits, (unsigned long long)__popcll(m));
}

// ---------------------------------------------------------------------------
// a1: reverse neighbors by counting sort: in-degree histogram, exclusive scan,
// scatter.  The order inside a co-friend list is arbitrary (the round's result
// does not depend on it).
// ---------------------------------------------------------------------------
__global__ void k_degree(const uint32_t* __restrict__ F, int64_t nK, int32_t* __restrict__ deg) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nK; e += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&deg[F[e] & IDMASK], 1);
}

constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = 256 * SCAN_ITEMS;

// Block-wide exclusive scan of one int64 per thread (256 threads).
__device__ __forceinline__ int64_t block_exscan(int64_t v, int64_t* sh /*[4]*/, int64_t& total) {
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  int64_t incl = v;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const int64_t t = (int64_t)shfl_u64((uint64_t)incl, max(lane - o, 0));
    if (lane >= o) incl += t;
  }
  if (lane == WAVE - 1) sh[wave] = incl;
  __syncthreads();
  int64_t off = 0;
  for (int w = 0; w < wave; ++w) off += sh[w];
  total = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return off + incl - v;
}

// Exclusive scan of deg[i] * a + b (a = 1, b = 0: reverse-neighbor offsets;
// a = K+1, b = K*K: offsets of the per-receiver candidate segments).
__global__ __launch_bounds__(256) void k_scan_tiles(const int32_t* __restrict__ deg, int64_t n, int64_t a,
                                                    int64_t b, int64_t* __restrict__ rowptr,
                                                    int64_t* __restrict__ tilesum) {
  __shared__ int64_t sh[4];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  int64_t v[SCAN_ITEMS];
  int64_t sum = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    v[k] = (base + k < n) ? (int64_t)deg[base + k] * a + b : 0;
    sum += v[k];
  }
  int64_t total;
  int64_t run = block_exscan(sum, sh, total);
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    if (base + k < n) rowptr[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) tilesum[blockIdx.x] = total;
}

// Exclusive scan of the tile sums in place (one block), total into rowptr[n].
__global__ __launch_bounds__(256) void k_scan_top(int64_t* __restrict__ tilesum, int64_t ntiles,
                                                  int64_t* __restrict__ rowptr, int64_t n) {
  __shared__ int64_t sh[4];
  int64_t carry = 0;
  for (int64_t b = 0; b < ntiles; b += 256) {
    const int64_t i = b + threadIdx.x;
    const int64_t v = i < ntiles ? tilesum[i] : 0;
    int64_t total;
    const int64_t ex = block_exscan(v, sh, total);
    if (i < ntiles) tilesum[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) rowptr[n] = carry;
}

__global__ void k_scan_add(int64_t* __restrict__ rowptr, int64_t n, const int64_t* __restrict__ tilesum) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    rowptr[i] += tilesum[i / SCAN_TILE];
}

// Edge e = x*K + j (x -> v = F[x][j]) lands at position q of coF(v):
// col[rowptr[v] + q] = x | new-flag, colslot[...] = j, revpos[e] = q.
__global__ void k_scatter(const uint32_t* __restrict__ F, int64_t nK, int K, const int64_t* __restrict__ rowptr,
                          int32_t* __restrict__ fill, uint32_t* __restrict__ col, uint8_t* __restrict__ colslot,
                          int32_t* __restrict__ revpos) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nK; e += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t raw = F[e];
    const uint32_t v = raw & IDMASK;
    const int q = atomicAdd(&fill[v], 1);
    const int64_t pos = rowptr[v] + q;
    const int64_t x = e / K;
    col[pos] = (uint32_t)x | (raw & NEWBIT);
    colslot[pos] = (uint8_t)(e - x * K);
    revpos[e] = q;
  }
}

// ---------------------------------------------------------------------------
// Receiver binning by hash-table size.  A receiver with c co-friends has at
// most T = c + K*K + c*K candidate occurrences; its table must hold the
// distinct candidates plus x and its K friends at load <= 1/2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t table_need(int64_t c, int K, int64_t n) {
  const int64_t T = c + (int64_t)K * K + c * K;
  return min(T, n - 1 - K) + K + 1;
}

__global__ __launch_bounds__(256) void k_bin(const int64_t* __restrict__ rowptr, int64_t n, int K,
                                             int32_t* __restrict__ counts, int32_t* __restrict__ lists) {
  const int lane = lane_id();
  // uniform trip count so that every lane takes part in the ballots
  for (int64_t x0 = blockIdx.x * (int64_t)blockDim.x; x0 < n; x0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = x0 + threadIdx.x;
    int cls = -1;
    if (x < n) {
      const int64_t need2 = 2 * table_need(rowptr[x + 1] - rowptr[x], K, n);
      cls = NCLASS - 1;
      for (int k = 0; k < NCLASS - 1; ++k)
        if (need2 <= (int64_t)(CLASS_CAP_MIN << k)) {
          cls = k;
          break;
        }
    }
    for (int k = 0; k < NCLASS; ++k) {
      const uint64_t m = __ballot(cls == k);
      if (!m) continue;
      int base = 0;
      if (lane == 0) base = atomicAdd(&counts[k], (int)__popcll(m));
      base = __shfl(base, 0, WAVE);
      if (cls == k) lists[(int64_t)k * n + base + (int)rank_in(m)] = (int32_t)x;
    }
  }
}

__device__ __forceinline__ int64_t block_sum(int64_t v, int64_t* sh /*[4]*/) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) v += (int64_t)shfl_xor_u64((uint64_t)v, o);
  if (lane_id() == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  const int64_t t = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return t;
}

// ---------------------------------------------------------------------------
// a2+a3, hub form: every point v is a hub whose friends F(v) (and v itself)
// are candidates for the receivers R(v) = coF(v) u F(v):
//   r in coF(v):      friends of a friend      -> F(v)
//   r in F(v):        friends of a co-friend   -> F(v) \ {r}, and the co-friend v
// The K+1 candidate log rows are staged in LDS once per hub; each wave takes
// floor(64/(K+1)) receivers at a time, one lane per candidate, and folds the
// canonical FP64 key.  Keys go to fixed slots of the receiver's segment, laid
// out in the receiver's own enumeration order:
//   [c co-friends][K x K friends of friends][c x K friends of co-friends]
// Pairs whose two edges were both present one round earlier are skipped
// (their candidate cannot enter, see the receiver kernel).
// ---------------------------------------------------------------------------
template <typename PT>
__global__ __launch_bounds__(256) void k_hub_lds(JoinArgs a) {
  extern __shared__ double s_cand[];  // (K+1) rows of Ds doubles
  __shared__ uint32_t s_fv[2 * WAVE];
  const int K = a.K, K1 = a.K + 1, D = a.D, Dp = a.Dp, Ds = a.Ds;
  const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
  const PT* P = reinterpret_cast<const PT*>(a.P);
  int G, g, ci0, cstep;
  if (K1 <= WAVE) {
    G = WAVE / K1;
    g = lane / K1;
    ci0 = lane - g * K1;
    cstep = K1;
  } else {
    G = 1;
    g = 0;
    ci0 = lane;
    cstep = WAVE;
  }
  const bool lane_on = g < G;
  int64_t my_perf = 0;

  for (int64_t v = blockIdx.x; v < a.n; v += gridDim.x) {
    const int64_t rp = a.rowptr[v];
    const int cv = (int)(a.rowptr[v + 1] - rp);
    bool anynew = !a.skip;
    if (tid < K) {
      const uint32_t e = a.F[v * K + tid];
      s_fv[tid] = e;
      anynew |= (e & NEWBIT) != 0;
    }
    for (int q = tid; q < cv; q += 256) anynew |= (a.col[rp + q] & NEWBIT) != 0;
    if (!__syncthreads_or(anynew)) continue;
    for (int idx = tid; idx < K1 * D; idx += 256) {
      const int j = idx / D, i = idx - j * D;
      const int64_t c = (j < K) ? (int64_t)(s_fv[j] & IDMASK) : v;
      s_cand[j * Ds + i] = a.L[c * Dp + i];
    }
    __syncthreads();
    const int nR = cv + K;
    for (int kb = wave * G; kb < nR; kb += 4 * G) {
      const int k = kb + g;
      if (!lane_on || k >= nR) continue;
      int64_t r, b0, b1 = -1;
      uint32_t rnew;
      int excl = -1;
      if (k < cv) {
        const uint32_t e = a.col[rp + k];
        r = e & IDMASK;
        rnew = e & NEWBIT;
        const int64_t cr = a.rowptr[r + 1] - a.rowptr[r];
        b0 = a.segbase[r] + cr + (int64_t)a.colslot[rp + k] * K;
      } else {
        const int sp = k - cv;
        const uint32_t e = s_fv[sp];
        r = e & IDMASK;
        rnew = e & NEWBIT;
        excl = sp;
        const int64_t q = a.revpos[v * K + sp];
        const int64_t cr = a.rowptr[r + 1] - a.rowptr[r];
        b0 = a.segbase[r] + cr + (int64_t)K * K + q * K;
        b1 = a.segbase[r] + q;
      }
      const PT* pr = P + r * D;
      const double* lr = a.L + r * Dp;
      for (int ci = ci0; ci < K1; ci += cstep) {
        int64_t pos;
        bool isnew;
        if (ci < K) {
          if (ci == excl) continue;
          pos = b0 + ci;
          isnew = (rnew | (s_fv[ci] & NEWBIT)) != 0;
        } else {
          if (b1 < 0) continue;
          pos = b1;
          isnew = rnew != 0;
        }
        if (a.skip && !isnew) continue;
        const double* lc = s_cand + ci * Ds;
        double acc = 0.0;
        for (int i = 0; i < D; ++i) acc = fma((double)pr[i], lr[i] - lc[i], acc);
        a.seg[pos] = acc + 0.0;
        ++my_perf;
      }
    }
    __syncthreads();
  }
  __shared__ int64_t s_red[4];
  const int64_t pf = block_sum(my_perf, s_red);
  if (tid == 0 && pf) atomicAdd((unsigned long long*)&a.stats[STAT_PERF], (unsigned long long)pf);
}

// Register form of the hub kernel for D <= MAXD (the common case): one wave
// per hub, one lane per receiver.  The receiver's coordinates and logs live in
// VGPRs; each candidate's log row is wave-uniform and is read with scalar
// loads, so the fold is two FP64 VALU operations per coordinate with no
// vector memory traffic.  Same output as k_hub_lds.
template <int MAXD, typename PT>
__global__ __launch_bounds__(256) void k_hub_reg(JoinArgs a, const double* __restrict__ L,
                                                 const PT* __restrict__ P) {
  const int K = a.K, K1 = a.K + 1, D = a.D, Dp = a.Dp;
  const int lane = lane_id();
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  int64_t my_perf = 0;
  for (int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); v < a.n; v += nwaves) {
    const int64_t rp = a.rowptr[v];
    const int cv = (int)(a.rowptr[v + 1] - rp);
    const uint32_t fv = lane < K ? a.F[v * K + lane] : 0u;  // lane j holds F(v)[j]
    const uint64_t cand_new = __ballot((fv & NEWBIT) != 0);
    const int nR = cv + K;
    for (int k0 = 0; k0 < nR; k0 += WAVE) {
      const int k = k0 + lane;
      const bool on = k < nR;
      // all lanes take part in the shuffle (a disabled source lane reads as 0)
      const uint32_t fsp = (uint32_t)__shfl((int)fv, (k >= cv && k < nR) ? k - cv : 0, WAVE);
      int64_t r = 0, b0 = 0, b1 = -1;
      uint32_t rnew = 0;
      int excl = -1;
      if (on) {
        if (k < cv) {
          const uint32_t e = a.col[rp + k];
          r = e & IDMASK;
          rnew = e & NEWBIT;
          const int64_t cr = a.rowptr[r + 1] - a.rowptr[r];
          b0 = a.segbase[r] + cr + (int64_t)a.colslot[rp + k] * K;
        } else {
          const int sp = k - cv;
          r = fsp & IDMASK;
          rnew = fsp & NEWBIT;
          excl = sp;
          const int64_t q = a.revpos[v * K + sp];
          const int64_t cr = a.rowptr[r + 1] - a.rowptr[r];
          b0 = a.segbase[r] + cr + (int64_t)K * K + q * K;
          b1 = a.segbase[r] + q;
        }
      }
      const bool want_any = on && (!a.skip || rnew != 0);
      if (a.skip && cand_new == 0 && __ballot(want_any) == 0) continue;
      // Receiver row in registers; coordinates beyond D are zero, so the
      // extra terms fma(0, y, acc) (y finite) leave acc unchanged.  Rows are
      // read past their end into the zeroed tail padding of P and L.
      double pr[MAXD], lr[MAXD];
      const PT* prow = P + (on ? r : 0) * D;
      const double* lrow = L + (on ? r : 0) * Dp;
#pragma unroll
      for (int i = 0; i < MAXD; ++i) {
        const double pv = (double)prow[i];
        const double lv = lrow[i];
        pr[i] = i < D ? pv : 0.0;
        lr[i] = i < D ? lv : 0.0;
      }
      for (int ci = 0; ci < K1; ++ci) {
        const bool cnew = ci < K && ((cand_new >> ci) & 1);
        bool need;
        int64_t pos;
        if (ci < K) {
          need = on && ci != excl && (!a.skip || rnew || cnew);
          pos = b0 + ci;
        } else {
          need = on && b1 >= 0 && (!a.skip || rnew);
          pos = b1;
        }
        if (__ballot(need) == 0) continue;
        const uint32_t craw = ci < K ? (uint32_t)__shfl((int)fv, ci, WAVE) : (uint32_t)v;
        const int64_t cidx = (int64_t)__builtin_amdgcn_readfirstlane(craw & IDMASK);
        const double* lc = L + cidx * Dp;  // wave-uniform: scalar loads
        double acc = 0.0;
#pragma unroll
        for (int i0 = 0; i0 < MAXD; i0 += 16) {
          double cv16[16];
#pragma unroll
          for (int i = 0; i < 16; ++i)
            if (i0 + i < MAXD) cv16[i] = lc[i0 + i];
#pragma unroll
          for (int i = 0; i < 16; ++i)
            if (i0 + i < MAXD) acc = fma(pr[i0 + i], lr[i0 + i] - cv16[i], acc);
        }
        if (need) {
          a.seg[pos] = acc + 0.0;
          ++my_perf;
        }
      }
    }
  }
  __shared__ int64_t s_red[4];
  const int64_t pf = block_sum(my_perf, s_red);
  if (threadIdx.x == 0 && pf) atomicAdd((unsigned long long*)&a.stats[STAT_PERF], (unsigned long long)pf);
}

// ---------------------------------------------------------------------------
// a2..a5, receiver side: one 256-thread block per receiver x.
//  B  insert x and F(x) into the block's hash set, marked excluded
//  C  enumerate every candidate occurrence (co-friends, friends of friends,
//     friends of co-friends) and insert it.  A first insertion is one
//     algorithmic evaluation.  The occurrence that first marks a candidate as
//     reached through a new edge appends it to the candidate list (with its
//     key from the segment in the hub form).
//  D  each wave takes 64 listed candidates at a time (the pull form computes
//     their canonical keys here, gathering log rows), drops those that cannot
//     beat the current K-th (the paper's compare-to-last, Section 4.2) and
//     merges the rest into its sorted list held in registers
//  E  wave 0 merges the four lists and writes the first K
// A candidate reached only through edges already present one round earlier
// was a candidate then too and lost to K entries that are still at least as
// good, so it cannot enter: it is counted but not evaluated.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int tab_insert(uint32_t* tab, uint32_t mask, uint32_t z, uint32_t flag) {
  // returns bit 0: first insertion of z; bit 1: this call marked z NEW first
  uint32_t h = z * 0x9E3779B1u;
  h = (h ^ (h >> 15)) & mask;
  for (;;) {
    const uint32_t old = atomicCAS(&tab[h], EMPTY, z | flag);
    if (old == EMPTY) return 1 | ((flag & NEWBIT) ? 2 : 0);
    if ((old & IDMASK) == z) {
      if ((flag & NEWBIT) && !(old & (NEWBIT | EXCLBIT))) {
        const uint32_t prev = atomicOr(&tab[h], NEWBIT);
        if (!(prev & NEWBIT)) return 2;
      }
      return 0;
    }
    h = (h + 1) & mask;
  }
}

template <int CAP, typename PT, bool SEG>
__global__ __launch_bounds__(256) void k_recv(JoinArgs a, const int32_t* __restrict__ list,
                                              const int32_t* __restrict__ count) {
  constexpr bool GLOB = (CAP == 0);
  constexpr bool BIG = (CAP > 8192);  // table in LDS, candidate list in global memory
  constexpr int CC = (GLOB || BIG) ? 1 : CAP / 2;
  __shared__ uint32_t s_tab[GLOB ? 1 : CAP];
  __shared__ uint32_t s_cid[CC];
  __shared__ double s_ckey[SEG ? CC : 1];
  __shared__ uint32_t s_fx[WAVE];
  __shared__ uint64_t s_lk[3][WAVE];
  __shared__ uint32_t s_li[3][WAVE];
  __shared__ uint64_t s_tau;
  __shared__ int s_ncand;
  __shared__ int64_t s_red[4];

  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wave = tid >> 6;
  const int K = a.K;
  const int D = a.D, Dp = a.Dp;
  const int64_t n = a.n;
  const int64_t half = a.gstride / 2;
  uint32_t* tab = GLOB ? a.gtab + (int64_t)blockIdx.x * a.gstride : s_tab;
  uint32_t* cid = GLOB ? a.gcand + (int64_t)blockIdx.x * half
                       : (BIG ? a.bcand + (int64_t)blockIdx.x * BIG_CAND : s_cid);
  double* ckey = SEG ? (GLOB ? a.gckey + (int64_t)blockIdx.x * half
                             : (BIG ? a.bckey + (int64_t)blockIdx.x * BIG_CAND : s_ckey))
                     : nullptr;
  const PT* P = reinterpret_cast<const PT*>(a.P);
  const int nitems = *count;
  int64_t my_evals = 0, my_perf = 0, my_upd = 0;

  for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
    const int64_t x = list[item];
    const int64_t rp = a.rowptr[x];
    const int64_t c = a.rowptr[x + 1] - rp;
    const int64_t KK = (int64_t)K * K;
    const int64_t T = c + KK + c * K;
    const int64_t sbase = SEG ? a.segbase[x] : 0;
    uint32_t cap = (uint32_t)CAP;
    if (GLOB) {
      const int64_t need2 = 2 * table_need(c, K, n);
      cap = CLASS_CAP_MIN;
      while ((int64_t)cap < need2) cap <<= 1;
    }
    const uint32_t mask = cap - 1;

    // A: clear
    for (uint32_t s = tid; s < cap; s += 256) tab[s] = EMPTY;
    if (tid == 0) {
      s_ncand = 0;
      s_tau = key_bits(a.keys[x * K + K - 1]);
    }
    __syncthreads();
    // B: excluded entries
    if (tid < K) {
      const uint32_t raw = a.F[x * K + tid];
      s_fx[tid] = raw;
      tab_insert(tab, mask, raw & IDMASK, EXCLBIT);
    } else if (tid == K) {
      tab_insert(tab, mask, (uint32_t)x, EXCLBIT);
    }
    __syncthreads();
    // C: enumerate candidate occurrences, four per thread in flight (uniform
    // trip count across the block)
    for (int64_t t0 = 0; t0 < T; t0 += 4 * 256) {
      uint32_t z[4], nw[4];
      int res[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t t = t0 + tid + 256 * u;
        z[u] = 0;
        nw[u] = 0;
        if (t < c) {
          const uint32_t w = a.col[rp + t];
          z[u] = w & IDMASK;
          nw[u] = w & NEWBIT;
        } else if (t < c + KK) {
          const int uu = (int)(t - c);
          const int j = uu / K;
          const int s = uu - j * K;
          const uint32_t v = s_fx[j];
          const uint32_t zr = a.F[(int64_t)(v & IDMASK) * K + s];
          z[u] = zr & IDMASK;
          nw[u] = (v | zr) & NEWBIT;
        } else if (t < T) {
          const int64_t uu = t - c - KK;
          const int64_t q = uu / K;
          const int s = (int)(uu - q * K);
          const uint32_t w = a.col[rp + q];
          const uint32_t zr = a.F[(int64_t)(w & IDMASK) * K + s];
          z[u] = zr & IDMASK;
          nw[u] = (w | zr) & NEWBIT;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        res[u] = 0;
        if (t0 + tid + 256 * u < T) {
          res[u] = tab_insert(tab, mask, z[u], a.skip ? nw[u] : NEWBIT);
          my_evals += res[u] & 1;
        }
      }
      double kv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) kv[u] = (SEG && (res[u] & 2)) ? a.seg[sbase + t0 + tid + 256 * u] : 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool app = (res[u] & 2) != 0;
        const uint64_t m = __ballot(app);
        if (m) {
          int base = 0;
          if (lane == 0) base = atomicAdd(&s_ncand, (int)__popcll(m));
          base = __shfl(base, 0, WAVE);
          if (app) {
            const int at = base + (int)rank_in(m);
            cid[at] = z[u];
            if (SEG) ckey[at] = kv[u];
          }
        }
      }
    }
    __syncthreads();
    // D: keys, compare-to-last filter, wave merges
    const int ncand = s_ncand;
    uint64_t lk = KEY_SENTINEL;
    uint32_t li = IDMASK;
    if (wave == 0 && lane < K) {
      lk = key_bits(a.keys[x * K + lane]);
      li = s_fx[lane] & IDMASK;
    }
    const PT* px = P + x * D;
    const double* lx = a.L + x * Dp;
    for (int i0 = wave * WAVE; i0 < ncand; i0 += 256) {
      const int i = i0 + lane;
      const bool valid = i < ncand;
      uint64_t kb = KEY_SENTINEL;
      uint32_t z = IDMASK;
      if (valid) {
        z = cid[i];
        if (SEG)
          kb = key_bits(ckey[i]);
        else
          kb = key_bits(canonical_key(px, lx, a.L + (int64_t)z * Dp, D));
      }
      my_perf += (!SEG && valid) ? 1 : 0;
      const uint64_t kk = shfl_u64(lk, K - 1);
      const uint32_t ki = shfl_u32(li, K - 1);
      const uint64_t tau = *(volatile uint64_t*)&s_tau;
      const bool surv = valid && kb <= tau && ke_less(kb, z, kk, ki);
      const uint64_t sm = __ballot(surv);
      if (sm) {
        if (__popcll(sm) <= 8) {
          // few survivors: insert them one by one
          uint64_t mm = sm;
          while (mm) {
            const int src = __ffsll((unsigned long long)mm) - 1;
            mm &= mm - 1;
            const uint64_t ck = shfl_u64(kb, src);
            const uint32_t cz = shfl_u32(z, src) | NEWBIT;
            if (ke_less(ck, cz, shfl_u64(lk, K - 1), shfl_u32(li, K - 1))) wave_insert(lk, li, ck, cz);
          }
        } else {
          uint64_t bk = surv ? kb : KEY_SENTINEL;
          uint32_t bi = surv ? (z | NEWBIT) : IDMASK;
          wave_sort(bk, bi);
          wave_merge(lk, li, bk, bi);
        }
        const uint64_t nk = shfl_u64(lk, K - 1);
        if (lane == 0 && nk < tau) atomicMin((unsigned long long*)&s_tau, (unsigned long long)nk);
      }
    }
    // E: combine the four wave lists
    if (wave > 0) {
      s_lk[wave - 1][lane] = lk;
      s_li[wave - 1][lane] = li;
    }
    __syncthreads();
    if (wave == 0) {
      for (int w = 0; w < 3; ++w) wave_merge(lk, li, s_lk[w][lane], s_li[w][lane]);
      if (lane < K) {
        a.Fn[x * K + lane] = li;
        a.keysn[x * K + lane] = bits_key(lk);
      }
      const uint64_t um = __ballot(lane < K && (li & NEWBIT));
      if (lane == 0) my_upd += (int64_t)__popcll(um);
    }
    __syncthreads();
  }
  const int64_t ev = block_sum(my_evals, s_red);
  const int64_t pf = block_sum(my_perf, s_red);
  const int64_t up = block_sum(my_upd, s_red);
  if (tid == 0) {
    if (ev) atomicAdd((unsigned long long*)&a.stats[STAT_EVALS], (unsigned long long)ev);
    if (pf) atomicAdd((unsigned long long*)&a.stats[STAT_PERF], (unsigned long long)pf);
    if (up) atomicAdd((unsigned long long*)&a.stats[STAT_UPDATES], (unsigned long long)up);
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline int grid_for(int64_t work, int block, int cap_blocks) {
  int64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap_blocks) g = cap_blocks;
  return (int)g;
}

hipError_t launch_zero_i64(int64_t* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_i64, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_log_table(const Ctx& c, int32_t* bad) {
  const int64_t total = c.n * c.Dp;
  const int g = grid_for(total, 256, 65536);
  if (c.dtype == 0)
    hipLaunchKernelGGL(k_log_table<float>, dim3(g), dim3(256), 0, c.stream, (const float*)c.P, c.n, c.D, c.Dp,
                       c.L, bad);
  else
    hipLaunchKernelGGL(k_log_table<double>, dim3(g), dim3(256), 0, c.stream, (const double*)c.P, c.n, c.D, c.Dp,
                       c.L, bad);
  return hipGetLastError();
}

hipError_t launch_init_graph(const Ctx& c) {
  const int g = (int)((c.n + 3) / 4);
  uint32_t* F = c.F[c.cur];
  double* keys = c.keys[c.cur];
  if (c.dtype == 0)
    hipLaunchKernelGGL(k_init_graph<float>, dim3(g), dim3(256), 0, c.stream, (const float*)c.P, c.L, c.n, c.D,
                       c.Dp, c.K, c.seed, F, keys);
  else
    hipLaunchKernelGGL(k_init_graph<double>, dim3(g), dim3(256), 0, c.stream, (const double*)c.P, c.L, c.n, c.D,
                       c.Dp, c.K, c.seed, F, keys);
  return hipGetLastError();
}

hipError_t launch_fcr(const Ctx& c, const uint32_t* F, int64_t round, int64_t* hits) {
  const int g = grid_for(c.M, 256, 1 << 30);
  hipLaunchKernelGGL(k_fcr, dim3(g), dim3(256), 0, c.stream, F, c.n, c.K, c.seed, round, c.M, hits);
  return hipGetLastError();
}

static void launch_scan(const Ctx& c, int64_t a, int64_t b, int64_t* out) {
  const int64_t ntiles = (c.n + SCAN_TILE - 1) / SCAN_TILE;
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(256), 0, c.stream, c.deg, c.n, a, b, out,
                     c.tilesum);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, c.stream, c.tilesum, ntiles, out, c.n);
  hipLaunchKernelGGL(k_scan_add, dim3(grid_for(c.n, 256, 8192)), dim3(256), 0, c.stream, out, c.n, c.tilesum);
}

hipError_t launch_csr(const Ctx& c, const uint32_t* F) {
  const int64_t nK = c.n * c.K;
  hipLaunchKernelGGL(k_zero_i32, dim3(grid_for(c.n, 256, 4096)), dim3(256), 0, c.stream, c.deg, c.n);
  hipLaunchKernelGGL(k_zero_i32, dim3(grid_for(c.n, 256, 4096)), dim3(256), 0, c.stream, c.fill, c.n);
  hipLaunchKernelGGL(k_degree, dim3(grid_for(nK, 256, 8192)), dim3(256), 0, c.stream, F, nK, c.deg);
  launch_scan(c, 1, 0, c.rowptr);
  if (c.use_hub) launch_scan(c, c.K + 1, (int64_t)c.K * c.K, c.segbase);
  hipLaunchKernelGGL(k_scatter, dim3(grid_for(nK, 256, 8192)), dim3(256), 0, c.stream, F, nK, c.K, c.rowptr,
                     c.fill, c.col, c.colslot, c.revpos);
  return hipGetLastError();
}

hipError_t launch_bin(const Ctx& c) {
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, c.stream, c.class_count, (int64_t)NCLASS);
  hipLaunchKernelGGL(k_bin, dim3(grid_for(c.n, 256, 8192)), dim3(256), 0, c.stream, c.rowptr, c.n, c.K,
                     c.class_count, c.class_list);
  return hipGetLastError();
}

template <int CAP, typename PT, bool SEG>
static hipError_t launch_recv_class(const Ctx& c, const JoinArgs& a, int cls) {
  auto kern = k_recv<CAP, PT, SEG>;
  int grid;
  if (CAP == 0) {
    grid = c.gblocks;
  } else {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0) != hipSuccess || per_cu < 1)
      per_cu = 1;
    grid = (int)std::min<int64_t>(c.n, (int64_t)per_cu * c.num_cu);
    if (CAP > 8192) grid = std::min(grid, c.bblocks);
  }
  hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, c.stream, a, c.class_list + (int64_t)cls * c.n,
                     c.class_count + cls);
  return hipGetLastError();
}

template <typename PT, bool SEG>
static hipError_t launch_recv_all(const Ctx& c, const JoinArgs& a) {
  hipError_t e;
  if ((e = launch_recv_class<CLASS_CAP_MIN << 0, PT, SEG>(c, a, 0)) != hipSuccess) return e;
  if ((e = launch_recv_class<CLASS_CAP_MIN << 1, PT, SEG>(c, a, 1)) != hipSuccess) return e;
  if ((e = launch_recv_class<CLASS_CAP_MIN << 2, PT, SEG>(c, a, 2)) != hipSuccess) return e;
  if ((e = launch_recv_class<CLASS_CAP_MIN << 3, PT, SEG>(c, a, 3)) != hipSuccess) return e;
  if ((e = launch_recv_class<CLASS_CAP_MIN << 4, PT, SEG>(c, a, 4)) != hipSuccess) return e;
  if ((e = launch_recv_class<CLASS_CAP_MIN << 5, PT, SEG>(c, a, 5)) != hipSuccess) return e;
  if ((e = launch_recv_class<CLASS_CAP_MIN << 6, PT, SEG>(c, a, 6)) != hipSuccess) return e;
  return launch_recv_class<0, PT, SEG>(c, a, 7);
}

template <int MAXD, typename PT>
static hipError_t launch_hub_reg(const Ctx& c, const JoinArgs& a) {
  auto kern = k_hub_reg<MAXD, PT>;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0) != hipSuccess || per_cu < 1) per_cu = 1;
  const int grid = (int)std::min<int64_t>((c.n + 3) / 4, (int64_t)per_cu * c.num_cu * 4);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, c.stream, a, c.L, (const PT*)c.P);
  return hipGetLastError();
}

template <typename PT>
static hipError_t launch_hub(const Ctx& c, const JoinArgs& a) {
  if (c.D <= 8) return launch_hub_reg<8, PT>(c, a);
  if (c.D <= 12) return launch_hub_reg<12, PT>(c, a);
  if (c.D <= 16) return launch_hub_reg<16, PT>(c, a);
  if (c.D <= 24) return launch_hub_reg<24, PT>(c, a);
  if (c.D <= 32) return launch_hub_reg<32, PT>(c, a);
  if (c.D <= 40) return launch_hub_reg<40, PT>(c, a);
  if (c.D <= 52) return launch_hub_reg<52, PT>(c, a);
  if (c.D <= HUB_MAXD) return launch_hub_reg<HUB_MAXD, PT>(c, a);
  const size_t lds = (size_t)(c.K + 1) * c.Ds * sizeof(double);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_hub_lds<PT>, 256, lds) != hipSuccess || per_cu < 1)
    per_cu = 1;
  const int grid = (int)std::min<int64_t>(c.n, (int64_t)per_cu * c.num_cu * 2);
  hipLaunchKernelGGL(k_hub_lds<PT>, dim3(grid), dim3(256), lds, c.stream, a);
  return hipGetLastError();
}

hipError_t launch_join(const Ctx& c, int64_t* stats) {
  JoinArgs a;
  a.P = c.P;
  a.L = c.L;
  a.n = c.n;
  a.D = c.D;
  a.Dp = c.Dp;
  a.Ds = c.Ds;
  a.K = c.K;
  a.F = c.F[c.cur];
  a.keys = c.keys[c.cur];
  a.rowptr = c.rowptr;
  a.col = c.col;
  a.colslot = c.colslot;
  a.revpos = c.revpos;
  a.segbase = c.segbase;
  a.seg = c.seg;
  a.Fn = c.F[c.cur ^ 1];
  a.keysn = c.keys[c.cur ^ 1];
  a.stats = stats;
  a.skip = (c.flags & 1) ? 0 : 1;
  a.gtab = c.gtab;
  a.gcand = c.gcand;
  a.gckey = c.gckey;
  a.gstride = c.gstride;
  a.bcand = c.bcand;
  a.bckey = c.bckey;
  hipError_t e;
  if (c.use_hub) {
    e = c.dtype == 0 ? launch_hub<float>(c, a) : launch_hub<double>(c, a);
    if (e != hipSuccess) return e;
    return c.dtype == 0 ? launch_recv_all<float, true>(c, a) : launch_recv_all<double, true>(c, a);
  }
  return c.dtype == 0 ? launch_recv_all<float, false>(c, a) : launch_recv_all<double, false>(c, a);
}

hipError_t launch_strip(const Ctx& c, const uint32_t* F, int32_t* out) {
  const int64_t cnt = c.n * c.K;
  hipLaunchKernelGGL(k_strip, dim3(grid_for(cnt, 256, 8192)), dim3(256), 0, c.stream, F, cnt, out);
  return hipGetLastError();
}

hipError_t launch_load_idx(const Ctx& c, const int32_t* idx, uint32_t* F) {
  const int64_t cnt = c.n * c.K;
  hipLaunchKernelGGL(k_load_idx, dim3(grid_for(cnt, 256, 8192)), dim3(256), 0, c.stream, idx, cnt, F);
  return hipGetLastError();
}

}  // namespace knnd
