// Segmented stable LSD radix sort of order-preserving float keys, and the
// order-statistic estimators computed on the sorted segments:
//   * univariate reweighted MCD (Sec. 3.1), used for the standardisation and
//     inside the refinement (Sec. 3.3 steps 3-4);
//   * median and MAD (DetMCD's standardisation, Sec. 2.2 step 1);
//   * the GSSCM cutoffs A, B of the linearly redescending weight (eq. LR).
#include "common.h"
#include "sortseg.h"
#include "wave.h"

#include <type_traits>

namespace rtd {

namespace {


constexpr int RS_NT = 256;           // threads per tile
constexpr int RS_ITEMS = 16;         // keys per thread
constexpr int RS_TILE = RS_NT * RS_ITEMS;
constexpr int RS_WAVES = RS_NT / 64;

template <typename K>
__device__ inline int digit_of(K k, int shift) { return (int)((k >> shift) & (K)0xFF); }

// Per-tile digit counts of the pass at `shift`.  PEEL (the top digit of
// double keys: very few distinct values) adds one count per distinct digit
// of a wave's 64 keys instead of one atomic per key on one or two counters.
template <typename K, bool PEEL>
__global__ __launch_bounds__(RS_NT) void k_rs_count(const K* __restrict__ keys,
                                                    const SegTile* __restrict__ tiles,
                                                    const int64_t* __restrict__ seg_off,
                                                    const int64_t* __restrict__ seg_len,
                                                    int shift, int32_t* __restrict__ counts) {
  __shared__ int hist[256];
  const SegTile t = tiles[blockIdx.x];
  const int64_t base = seg_off[t.seg] + (int64_t)t.tile * RS_TILE;
  const int64_t end = seg_off[t.seg] + seg_len[t.seg];
  hist[threadIdx.x] = 0;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < RS_ITEMS; ++i) {
    const int64_t k = base + i * RS_NT + threadIdx.x;
    if constexpr (PEEL) {
      const bool valid = k < end;
      const int d = valid ? digit_of(keys[k], shift) : 0;
      uint64_t left = __ballot(valid);
      while (left) {
        const int lead = __ffsll((long long)left) - 1;
        const int dl = __builtin_amdgcn_readlane(d, lead);
        const uint64_t mm = __ballot(valid && d == dl);
        if ((int)(threadIdx.x & 63) == lead) atomicAdd(&hist[dl], __popcll(mm));
        left &= ~mm;
      }
    } else {
      if (k < end) atomicAdd(&hist[digit_of(keys[k], shift)], 1);
    }
  }
  __syncthreads();
  counts[(size_t)blockIdx.x * 256 + threadIdx.x] = hist[threadIdx.x];
}

// Per segment: offsets[tile][d] = base(d) + counts of digit d in earlier tiles.
// Thread (g, d) walks a quarter g of the segment's tiles for digit d, eight
// independent loads at a time; digit bases come from a wave scan.
constexpr int SCAN_NT = 1024;
constexpr int SCAN_U = 8;

__global__ __launch_bounds__(SCAN_NT) void k_rs_scan(const int32_t* __restrict__ counts,
                                                     const int32_t* __restrict__ seg_tile0,
                                                     int tile_first, int32_t* __restrict__ offs) {
  __shared__ int gt[4][256];
  __shared__ int wsum[4];
  const int s = blockIdx.x;
  const int t0 = seg_tile0[s] - tile_first, t1 = seg_tile0[s + 1] - tile_first;
  const int tid = threadIdx.x, d = tid & 255, g = tid >> 8, lane = tid & 63, w = tid >> 6;
  const int nt = t1 - t0;
  const int a = t0 + (nt * g) / 4, b = t0 + (nt * (g + 1)) / 4;
  int tot = 0;
  for (int t = a; t < b; t += SCAN_U) {
    int c[SCAN_U];
#pragma unroll
    for (int u = 0; u < SCAN_U; ++u) c[u] = (t + u < b) ? counts[(size_t)(t + u) * 256 + d] : 0;
#pragma unroll
    for (int u = 0; u < SCAN_U; ++u) tot += c[u];
  }
  gt[g][d] = tot;
  __syncthreads();
  if (tid < 256) {   // digit d = tid: total over groups, scan over digits
    const int g0 = gt[0][d], g1 = gt[1][d], g2 = gt[2][d], g3 = gt[3][d];
    const int T = g0 + g1 + g2 + g3;
    int x = T;
    x = wave_incl_sum(x);
    if (lane == 63) wsum[w] = x;
    const int ex = x - T;
    gt[0][d] = ex;
    gt[1][d] = ex + g0;
    gt[2][d] = ex + g0 + g1;
    gt[3][d] = ex + g0 + g1 + g2;
  }
  __syncthreads();
  int run = gt[g][d];
  for (int k = 0; k < (d >> 6); ++k) run += wsum[k];
  for (int t = a; t < b; t += SCAN_U) {
    int c[SCAN_U];
#pragma unroll
    for (int u = 0; u < SCAN_U; ++u) c[u] = (t + u < b) ? counts[(size_t)(t + u) * 256 + d] : 0;
#pragma unroll
    for (int u = 0; u < SCAN_U; ++u) {
      if (t + u < b) offs[(size_t)(t + u) * 256 + d] = run;
      run += c[u];
    }
  }
}

// Stable scatter of one tile.  Wave w owns keys [w*1024, (w+1)*1024) of the
// tile, visited 64 at a time in index order.  Equal digits are ranked within
// a wave by LDS atomics on per-(wave, digit) counters (their results follow
// lane order on this hardware) or, with SAFE, by eight ballots (stable by
// construction).  PEEL ranks the top digit (few distinct values, so atomics
// would serialise) with one ballot per distinct digit.  The tile is then
// ordered by digit in LDS, so that the global writes of each digit run are
// contiguous.
template <typename K, bool SAFE, bool PEEL>
__global__ __launch_bounds__(RS_NT) void k_rs_scatter(const K* __restrict__ kin,
                                                      K* __restrict__ kout,
                                                      const SegTile* __restrict__ tiles,
                                                      const int64_t* __restrict__ seg_off,
                                                      const int64_t* __restrict__ seg_len,
                                                      int shift,
                                                      const int32_t* __restrict__ offs,
                                                      int32_t* __restrict__ zero_after) {
  __shared__ int wc[RS_WAVES][256];
  __shared__ int td[256];            // tile-local start of each digit
  __shared__ int go[256];            // global position of a tile slot: go[d] + slot
  __shared__ int wtot[RS_WAVES];
  __shared__ K sl[RS_TILE];
  const SegTile t = tiles[blockIdx.x];
  const int64_t so = seg_off[t.seg];
  const int64_t base = so + (int64_t)t.tile * RS_TILE;
  const int64_t end = so + seg_len[t.seg];
  const int nvalid = (int)min((int64_t)RS_TILE, end - base);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (zero_after != nullptr && blockIdx.x == 0 && tid == 0) *zero_after = 0;   // (no longer read)
  for (int d = tid; d < RS_WAVES * 256; d += RS_NT) (&wc[0][0])[d] = 0;
  __syncthreads();
  K kv[RS_ITEMS];
  int dg[RS_ITEMS], rk[RS_ITEMS];
  const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll
  for (int i = 0; i < RS_ITEMS; ++i) {
    const int q = w * (RS_ITEMS * 64) + i * 64 + lane;
    const bool valid = q < nvalid;
    kv[i] = valid ? kin[base + q] : (K)0;
    const int d = digit_of(kv[i], shift);
    dg[i] = d;
    if constexpr (SAFE) {
      uint64_t match = __ballot(valid);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const uint64_t bb = __ballot((d >> b) & 1);
        match &= ((d >> b) & 1) ? bb : ~bb;
      }
      const int before = __popcll(match & below);
      const int cur = wc[w][d];
      rk[i] = cur + before;
      if (valid && before == 0) wc[w][d] = cur + __popcll(match);
    } else if constexpr (PEEL) {
      uint64_t left = __ballot(valid);
      int rank = 0;
      while (left) {
        const int lead = __ffsll((long long)left) - 1;
        const int dl = __builtin_amdgcn_readlane(d, lead);
        const uint64_t mm = __ballot(valid && d == dl);
        const int cur = wc[w][dl];
        if (valid && d == dl) rank = cur + __popcll(mm & below);
        if (lane == lead) wc[w][dl] = cur + __popcll(mm);
        left &= ~mm;
      }
      rk[i] = rank;
    } else {
      rk[i] = valid ? atomicAdd(&wc[w][d], 1) : 0;
    }
  }
  __syncthreads();
  // per digit d = tid: exclusive scan over waves, then over digits
  {
    const int d = tid;
    int acc = 0;
#pragma unroll
    for (int k = 0; k < RS_WAVES; ++k) {
      const int v = wc[k][d];
      wc[k][d] = acc;
      acc += v;
    }
    int x = acc;
    x = wave_incl_sum(x);
    if (lane == 63) wtot[w] = x;
    __syncthreads();
    int ex = x - acc;
    for (int k = 0; k < w; ++k) ex += wtot[k];
    td[d] = ex;
    go[d] = offs[(size_t)blockIdx.x * 256 + d] - ex;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < RS_ITEMS; ++i) {
    const int q = w * (RS_ITEMS * 64) + i * 64 + lane;
    if (q < nvalid) sl[td[dg[i]] + wc[w][dg[i]] + rk[i]] = kv[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < RS_ITEMS; ++i) {
    const int q = i * RS_NT + tid;
    if (q < nvalid) {
      const K k = sl[q];
      kout[so + go[digit_of(k, shift)] + q] = k;
    }
  }
}

// Order check of sorted segments: any adjacent pair out of order sets *flag.
template <typename K>
__global__ __launch_bounds__(RS_NT) void k_rs_check(const K* __restrict__ keys,
                                                    const SegTile* __restrict__ tiles,
                                                    const int64_t* __restrict__ seg_off,
                                                    const int64_t* __restrict__ seg_len,
                                                    int32_t* __restrict__ flag) {
  const SegTile t = tiles[blockIdx.x];
  const int64_t so = seg_off[t.seg];
  const int64_t base = so + (int64_t)t.tile * RS_TILE;
  const int64_t end = so + seg_len[t.seg];
  bool bad = false;
#pragma unroll 4
  for (int i = 0; i < RS_ITEMS; ++i) {
    const int64_t k = base + i * RS_NT + threadIdx.x;
    if (k + 1 < end) bad = bad || keys[k] > keys[k + 1];
  }
  if (bad) *flag = 1;
}

// After passes on the high 48 bits of 64-bit keys (stable, so keys equal
// there keep their order of arrival): runs of equal high bits that hold a
// descent of the full key are listed, each from its first descent (the walks
// only read: another run's fix-up never touches this run), as (start << 12
// | length) in list[1..cap] with the count in list[0] (as int32, zero on
// entry).  A run longer than FIXUP_RUN, or more runs than cap, sets *flag
// (the fit is then run again with the full-width sort).
constexpr int GRUN_MAX = 256;   // longest run fixed in place
template <typename K>
__global__ __launch_bounds__(RS_NT) void k_rs_runs(const K* __restrict__ keys,
                                                   const SegTile* __restrict__ tiles,
                                                   const int64_t* __restrict__ seg_off,
                                                   const int64_t* __restrict__ seg_len,
                                                   uint64_t* __restrict__ list, int cap,
                                                   int32_t* __restrict__ flag) {
  const SegTile t = tiles[blockIdx.x];
  const int64_t so = seg_off[t.seg];
  const int64_t base = so + (int64_t)t.tile * RS_TILE;
  const int64_t end = so + seg_len[t.seg];
  auto hi = [](K k) { return (uint64_t)(k >> 16); };
#pragma unroll 4
  for (int i = 0; i < RS_ITEMS; ++i) {
    const int64_t q = base + i * RS_NT + threadIdx.x;
    if (q + 1 >= end) continue;
    const K a = keys[q], b = keys[q + 1];
    if (!(hi(a) == hi(b) && a > b)) continue;
    const uint64_t hq = hi(a);
    int64_t s0 = q;
    bool first = true, over = false;
    K right = a;
    while (s0 > so) {
      if (q - s0 >= GRUN_MAX) { over = true; break; }
      const K left = keys[s0 - 1];
      if (hi(left) != hq) break;
      if (left > right) { first = false; break; }   // an earlier descent takes the run
      right = left;
      --s0;
    }
    if (!first) continue;
    int64_t e = q + 2;
    while (!over && e < end && hi(keys[e]) == hq) {
      if (e - s0 >= GRUN_MAX) over = true;
      ++e;
    }
    if (over) {
      *flag = 1;
      continue;
    }
    const int slot = atomicAdd(reinterpret_cast<int32_t*>(list), 1);
    if (slot < cap) list[1 + slot] = ((uint64_t)s0 << 12) | (uint64_t)(e - s0);
    else *flag = 1;
  }
}

// Insertion sort of each listed run, one thread per run.
template <typename K>
__global__ __launch_bounds__(256) void k_rs_fixup(K* __restrict__ keys,
                                                  const uint64_t* __restrict__ list, int cap) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  const int n = min(*reinterpret_cast<const int32_t*>(list), cap);
  if (r >= n) return;
  const uint64_t e = list[1 + r];
  const int64_t s0 = (int64_t)(e >> 12), len = (int64_t)(e & 0xFFF);
  for (int64_t a = s0 + 1; a < s0 + len; ++a) {
    const K x = keys[a];
    int64_t b = a;
    while (b > s0 && keys[b - 1] > x) {
      keys[b] = keys[b - 1];
      --b;
    }
    keys[b] = x;
  }
}

// ---------------------------------------------------------------------------
// Estimators on sorted segments.  One block per segment.
// ---------------------------------------------------------------------------
constexpr int SS_NT = 1024;

template <typename K>
__device__ inline double val_of(K k);
template <>
__device__ inline double val_of<uint32_t>(uint32_t k) {
  const uint32_t b = (k & 0x80000000u) ? (k ^ 0x80000000u) : ~k;
  return (double)__uint_as_float(b);
}
template <>
__device__ inline double val_of<uint64_t>(uint64_t k) {
  const uint64_t b = (k & 0x8000000000000000ull) ? (k ^ 0x8000000000000000ull) : ~k;
  return __longlong_as_double((long long)b);
}
// segments already converted back to values
template <>
__device__ inline double val_of<float>(float k) {
  return (double)k;
}
template <>
__device__ inline double val_of<double>(double k) {
  return k;
}

constexpr int SS_WV = SS_NT / 64;

// Exclusive prefix sums in thread order of NV doubles per thread (wave scans,
// then the totals of earlier waves) over a block of NW waves.  red: NV * NW
// doubles.  TRAIL: end with a barrier, so that red may be written again.
template <int NV, bool TRAIL = true, int NW = SS_WV>
__device__ inline void block_excl_prefix(double (&v)[NV], double* __restrict__ red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double ex[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double x = wave_incl_sum(v[k]);
    if (lane == 63) red[k * NW + w] = x;
    ex[k] = dpp_d<0x138, 0xf>(x, 0.0);   // wave_shr 1: the previous lane's, 0 in lane 0
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double off = 0.0;
    for (int q = 0; q < w; ++q) off += red[k * NW + q];
    v[k] = off + ex[k];
  }
  if (TRAIL) __syncthreads();
}

// Sums over a block of NW waves of NV doubles per thread, in a fixed order
// (xor tree in each wave, then the waves in index order); every thread
// receives them.  red: NV * NW doubles; ends with a barrier.
template <int NV, int NW>
__device__ inline void block_sums(double (&v)[NV], double* __restrict__ red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double x = wave_sum(v[k]);
    if (lane == 0) red[k * NW + w] = x;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) t += red[k * NW + q];
    v[k] = t;
  }
  __syncthreads();
}

// k-th smallest (0-based) of |v_i - c| for a sorted segment v, by bisection on
// the count of values within the band [c - t, c + t]; the answer is one of
// the deviations, found exactly by searching over the two monotone runs.
template <typename K>
__device__ double kth_abs_dev(const K* __restrict__ v, int64_t L, double c, int64_t k) {
  // split point: first index with v >= c
  int64_t lo = 0, hi = L;
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    if (val_of<K>(v[mid]) < c) lo = mid + 1;
    else hi = mid;
  }
  const int64_t s = lo;            // left run: c - v[s-1], c - v[s-2], ... (increasing)
  const int64_t nl = s, nr = L - s;  // right run: v[s] - c, v[s+1] - c, ... (increasing)
  // k-th smallest of two sorted sequences A (len nl) and B (len nr)
  int64_t a_lo = k + 1 > nr ? k + 1 - nr : 0;
  int64_t a_hi = k + 1 < nl ? k + 1 : nl;
  // choose i elements from A, k+1-i from B
  while (a_lo < a_hi) {
    const int64_t i = (a_lo + a_hi) / 2;
    const int64_t j = k + 1 - i;
    const double Ai = (i < nl) ? c - val_of<K>(v[s - 1 - i]) : INFINITY;   // A[i]
    const double Bj1 = (j > 0) ? val_of<K>(v[s + j - 1]) - c : -INFINITY; // B[j-1]
    if (Ai < Bj1) a_lo = i + 1;
    else a_hi = i;
  }
  const int64_t i = a_lo, j = k + 1 - i;
  const double Ai1 = (i > 0) ? c - val_of<K>(v[s - i]) : -INFINITY;       // A[i-1]
  const double Bj1 = (j > 0) ? val_of<K>(v[s + j - 1]) - c : -INFINITY;   // B[j-1]
  return Ai1 > Bj1 ? Ai1 : Bj1;
}

template <typename K>
__device__ inline double median_sorted(const K* __restrict__ v, int64_t L) {
  const double a = val_of<K>(v[(L - 1) / 2]), b = val_of<K>(v[L / 2]);
  return 0.5 * (a + b);
}

// Order-statistic estimators of a sorted segment v[0..L), L > 0, computed by
// one thread: median/MAD and the GSSCM cutoffs.  Kept out of line: it is
// cold next to the univariate MCD.
template <typename K>
__device__ __noinline__ SegStat segstat_order(const K* __restrict__ v, int64_t L, int mode) {
  SegStat r{};
  if (mode == SEGSTAT_MEDMAD) {
    const double med = median_sorted(v, L);
    const double a = kth_abs_dev(v, L, med, (L - 1) / 2);
    const double b = kth_abs_dev(v, L, med, L / 2);
    r.mu = r.mu_raw = med;
    const double mad = 1.4826 * 0.5 * (a + b);
    r.var = r.var_raw = mad * mad;
    r.n_kept = L;
    return r;
  }
  if (mode == SEGSTAT_GSSCM) {
    // norms r sorted; s = r^(2/3) is sorted as well
    const double A = median_sorted(v, L);
    const double sa = pow(val_of<K>(v[(L - 1) / 2]), 2.0 / 3.0);
    const double sb = pow(val_of<K>(v[L / 2]), 2.0 / 3.0);
    const double ms = 0.5 * (sa + sb);
    // median of |s_i - ms| over the two monotone runs of s
    int64_t lo = 0, hi = L;
    while (lo < hi) {
      const int64_t mid = (lo + hi) / 2;
      if (pow(val_of<K>(v[mid]), 2.0 / 3.0) < ms) lo = mid + 1;
      else hi = mid;
    }
    const int64_t s0 = lo, nl = s0, nr = L - s0;
    double dev[2];
    for (int q = 0; q < 2; ++q) {
      const int64_t k = q == 0 ? (L - 1) / 2 : L / 2;
      int64_t a_lo = k + 1 > nr ? k + 1 - nr : 0;
      int64_t a_hi = k + 1 < nl ? k + 1 : nl;
      while (a_lo < a_hi) {
        const int64_t i = (a_lo + a_hi) / 2, j = k + 1 - i;
        const double Ai = (i < nl) ? ms - pow(val_of<K>(v[s0 - 1 - i]), 2.0 / 3.0) : INFINITY;
        const double Bj1 = (j > 0) ? pow(val_of<K>(v[s0 + j - 1]), 2.0 / 3.0) - ms : -INFINITY;
        if (Ai < Bj1) a_lo = i + 1;
        else a_hi = i;
      }
      const int64_t i = a_lo, j = k + 1 - i;
      const double Ai1 = (i > 0) ? ms - pow(val_of<K>(v[s0 - i]), 2.0 / 3.0) : -INFINITY;
      const double Bj1 = (j > 0) ? pow(val_of<K>(v[s0 + j - 1]), 2.0 / 3.0) - ms : -INFINITY;
      dev[q] = Ai1 > Bj1 ? Ai1 : Bj1;
    }
    const double mad = 0.5 * (dev[0] + dev[1]);
    r.mu = A;
    r.var = pow(ms + mad, 1.5);
    return r;
  }
  return r;
}

// Estimator over one sorted segment v[0..L) (global or LDS memory), computed
// by the whole block; the result is valid in thread 0.  Scratch: red, pfa,
// pfb hold SS_NT doubles each.
template <typename K>
__device__ __forceinline__ SegStat segstat_body(const K* __restrict__ v, int64_t L, double craw,
                                                double q1, double crew, int mode, double* red,
                                                double* pfa, double* pfb) {
  const int tid = threadIdx.x;
  SegStat r{};
  if (L <= 0) return r;
  if (mode != SEGSTAT_UNIMCD) {
    if (tid == 0) r = segstat_order<K>(v, L, mode);
    return r;
  }
  // ---- univariate reweighted MCD (Sec. 3.1)
  // red is split so that no region is written again after its barrier:
  // [0, 2 SS_WV) prefix totals, [64, 128) best windows, [128, 176) sums.
  const int lane = tid & 63, w = tid >> 6;
  const int64_t hh = L / 2 + 1;
  const double hd = (double)hh;
  const double c = val_of<K>(v[L / 2]);
  const int64_t a0 = (L * tid) / SS_NT, a1 = (L * (tid + 1)) / SS_NT;
  double pa[2] = {0.0, 0.0};
  for (int64_t k = a0; k < a1; ++k) {
    const double d = val_of<K>(v[k]) - c;
    pa[0] += d;
    pa[1] = fma(d, d, pa[1]);
  }
  block_excl_prefix<2, false>(pa, red);
  const double P1a = pa[0], P2a = pa[1];
  // prefix at a0 + hh: the owner thread's prefix plus part of its range
  double P1b = 0.0, P2b = 0.0;
  const int64_t nw = L - hh + 1;             // number of windows
  const int64_t j0 = a0, j1 = a1 < nw ? a1 : nw;
  pfa[tid] = P1a;
  pfb[tid] = P2a;
  __syncthreads();
  if (j0 < j1) {
    const int64_t pos = j0 + hh;             // <= L
    // owner of pos: the estimate is off by at most one either way
    int ow = (int)((double)pos * ((double)SS_NT / (double)L));
    if (ow > SS_NT - 1) ow = SS_NT - 1;
    while (ow > 0 && (L * ow) / SS_NT > pos) --ow;
    while (ow < SS_NT - 1 && (L * (ow + 1)) / SS_NT <= pos) ++ow;
    const int64_t ob = (L * ow) / SS_NT;
    P1b = pfa[ow];
    P2b = pfb[ow];
    for (int64_t k = ob; k < pos; ++k) {
      const double d = val_of<K>(v[k]) - c;
      P1b += d;
      P2b = fma(d, d, P2b);
    }
  }
  // windows are ranked by hd * s2 - s1^2 = hd (hd - 1) var (no division in
  // the loop); the variance itself is formed from the best window's sums
  double best = INFINITY, b1 = 0.0, b2 = 0.0;
  int64_t bj = -1;
  {
    double q1l = P1a, q2l = P2a, q1h = P1b, q2h = P2b;
    for (int64_t j = j0; j < j1; ++j) {
      const double s1 = q1h - q1l, s2 = q2h - q2l;
      const double cr = fma(s2, hd, -(s1 * s1));
      if (cr < best) { best = cr; bj = j; b1 = s1; b2 = s2; }
      const double dl = val_of<K>(v[j]) - c;
      q1l += dl;
      q2l = fma(dl, dl, q2l);
      if (j + hh < L) {
        const double dh = val_of<K>(v[j + hh]) - c;
        q1h += dh;
        q2h = fma(dh, dh, q2h);
      }
    }
  }
  // smallest criterion, ties to the lowest start (an exact min, so every
  // lane of the xor tree agrees); the lane that owns the winning window
  // publishes its variance and window sum
  double* __restrict__ rb = red + 64;
  {
    const int64_t own = bj;
    wave_argmin(best, bj);
    if (own >= 0 && own == bj) {
      rb[SS_WV + w] = (b2 - b1 * b1 / hd) / (hd - 1.0);
      rb[2 * SS_WV + w] = b1;
    }
    if (lane == 0) {
      rb[w] = best;
      reinterpret_cast<int64_t*>(rb)[3 * SS_WV + w] = bj;
    }
  }
  __syncthreads();
  double cmin = INFINITY, wmin = INFINITY, s1w = 0.0;
  int64_t js = -1;
  for (int q = 0; q < SS_WV; ++q) {
    const double c2 = rb[q];
    const int64_t j2 = reinterpret_cast<const int64_t*>(rb)[3 * SS_WV + q];
    if (j2 >= 0 && (js < 0 || c2 < cmin)) {   // waves hold increasing starts
      cmin = c2;
      wmin = rb[SS_WV + q];
      s1w = rb[2 * SS_WV + q];
      js = j2;
    }
  }
  const double mu_raw = c + s1w / hd;
  const double var_raw = wmin * craw;
  // reweighting: keep (v - mu_raw)^2 <= q1 var_raw
  const double lim = q1 * var_raw;
  double cs[3] = {0.0, 0.0, 0.0};
  for (int64_t k = a0; k < a1; ++k) {
    const double x = val_of<K>(v[k]);
    const double e = x - mu_raw;
    if (e * e <= lim) {
      const double d = x - c;
      cs[0] += 1.0;
      cs[1] += d;
      cs[2] = fma(d, d, cs[2]);
    }
  }
  // sums over the block (xor tree in each wave, then the waves in order),
  // needed by thread 0 only
  double* __restrict__ rs = red + 128;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double x = wave_sum(cs[k]);
    if (lane == 0) rs[k * SS_WV + w] = x;
  }
  __syncthreads();
  if (tid == 0) {
    double N = 0.0, S1 = 0.0, S2 = 0.0;
    for (int q = 0; q < SS_WV; ++q) {
      N += rs[q];
      S1 += rs[SS_WV + q];
      S2 += rs[2 * SS_WV + q];
    }
    r.mu_raw = mu_raw;
    r.var_raw = var_raw;
    r.start = js;
    r.n_kept = (int64_t)N;
    r.mu = N > 0 ? c + S1 / N : NAN;
    r.var = N > 1 ? (S2 - S1 * S1 / N) / (N - 1.0) * crew : 0.0;
  }
  return r;
}

// Estimator over segments already sorted in global memory.
template <typename K>
__global__ __launch_bounds__(SS_NT) void k_segstats(const K* __restrict__ keys,
                                                    const int64_t* __restrict__ seg_off,
                                                    const int64_t* __restrict__ seg_len,
                                                    const double* __restrict__ seg_craw,
                                                    double q1, double crew, int mode,
                                                    SegStat* __restrict__ out) {
  __shared__ double red[SS_NT], pfa[SS_NT], pfb[SS_NT];
  const int sg = blockIdx.x;
  const SegStat r = segstat_body<K>(keys + seg_off[sg], seg_len[sg], seg_craw[sg], q1, crew, mode,
                                    red, pfa, pfb);
  if (threadIdx.x == 0) out[sg] = r;
}

// Sort one segment of at most LDS_KEYS keys entirely in LDS (LSD radix on
// 8-bit digits), then run the estimator on the sorted LDS copy.  With KPT
// keys per thread, wave w holds the keys at positions w*KPT*64 + i*64 + lane,
// i < KPT, so ranks follow position order; KPT is the smallest even number
// from 4 to 16 that holds the segment, so little padding is sorted.
//
// The three passes run on a 24-bit key normalised to the segment's value
// range (DigitNorm): a monotone function of the value, so its order never
// contradicts the order of the values, and all of its digits spread over the
// values (the high bits of the order key hold the sign and exponent, which
// take few distinct values).  The last pass scatters the values themselves,
// so the buffer then holds the values ordered on the key.
//
// Ranks within a wave come from LDS atomics on per-(wave, digit) counters;
// those ranks follow lane order on this hardware, which keeps each pass
// stable.  Nothing is taken on trust: the estimator's threads load their
// contiguous ranges of the result and compare every adjacent pair
// (check_fix).  A descent between equal keys (values closer than the key's
// resolution: a few pairs per segment of continuous data) puts its run on a
// list, found from the run's first descent; each listed run is then put in
// order by insertion sort by one thread.  Runs of equal values hold no
// descent and are never walked.  A descent between unequal keys or a padding
// value inside the segment fails the check; so do too many descents, or a
// run too long or too costly for the fix-up (values crowded into a few keys:
// heavy tails, far outliers).  Such a segment is left to k_seg_lds_slow:
// passes on the high 32 bits of the order key (resolution relative to each
// value) with the same check, and failing that the full-width sort with
// ballot ranking only.
constexpr int LDS_KEYS = SS_NT * 16;
constexpr int FIXUP_RUN = 256;      // longest run finished by insertion sort
constexpr int FIXUP_MOVES = 2048;   // insertion-sort budget per run
constexpr int FIXUP_LIST = 1024;    // runs fixed per segment
constexpr int NORM_MAX_DESC = 512;  // descents fixed after the normalised-key passes
constexpr int64_t SEG_REDO = -2;    // SegStat.start of a segment left to k_seg_lds_slow

// How a pass ranks keys within a wave (all three follow lane order).
constexpr int RK_ATOM = 0;     // LDS atomics on per-(wave, digit) counters
constexpr int RK_BALLOT = 1;   // match by eight bit ballots: any digit mix
constexpr int RK_PEEL = 2;     // one ballot per distinct digit in the wave

// Digits of a pass: 8 bits at `shift` of the item's sort key.
struct DigitFull {   // the key itself
  template <typename K>
  __device__ int operator()(K k, int shift) const { return (int)((k >> shift) & (K)0xFF); }
};
struct DigitKey32 {   // the high 32 bits of the key (all of a float key)
  template <typename K>
  __device__ int operator()(K k, int shift) const {
    return (int)(((uint32_t)(k >> (8 * sizeof(K) - 32)) >> shift) & 0xFFu);
  }
};
// Padding of a block's key slots beyond the segment: slot q holds the order
// key ~0 - q (a NaN pattern, above every real key), so padded slots spread
// over the digits instead of all ranking on one counter.
template <typename K>
__device__ inline K pad_key(int q) { return ~(K)0 - (K)q; }
template <typename K>
__device__ inline bool is_pad(K k) { return k > ~(K)0 - (K)65536; }
constexpr uint32_t NORM_TOP = 16777216u - 4096u;   // real keys below, padding from here

// The segment-normalised 24-bit key floor((x - lo) T / (hi - lo)) of the
// item's value x, T = 2^24 - 2^12, clamped to [0, T - 1]; padding slot q
// takes T + (q mod 2^12).  Each step (fma with a positive scale, clamps,
// truncation) is monotone in x, so its order never contradicts the order of
// the values; unlike the high bits of the order key, all three digits
// spread over the segment's values.
struct DigitNorm {
  double sc, off;   // T / (hi - lo), -lo sc
  // From per-wave bounds of the high 32 bits of the order keys, rr[0..16)
  // (minima) and rr[16..32) (maxima), read after a barrier: 16 lanes of
  // every wave reduce them, so every lane gets the same values, kept in
  // scalar registers.  lo and hi are the smallest and largest values with
  // those high halves, so lo <= every value <= hi.  A range that is empty or
  // too narrow to scale gives one key to all values (a single run of equal
  // keys).
  template <typename K>
  __device__ void finish(const uint32_t* rr) {
    const int l = threadIdx.x & 15;
    uint32_t mn = rr[l], mx = rr[16 + l];
    mn = min(mn, (uint32_t)dpp_i<0x111, 0xf>((int)mn, -1));   // row_shr 1, 2, 4, 8
    mx = max(mx, (uint32_t)dpp_i<0x111, 0xf>((int)mx, 0));
    mn = min(mn, (uint32_t)dpp_i<0x112, 0xf>((int)mn, -1));
    mx = max(mx, (uint32_t)dpp_i<0x112, 0xf>((int)mx, 0));
    mn = min(mn, (uint32_t)dpp_i<0x114, 0xf>((int)mn, -1));
    mx = max(mx, (uint32_t)dpp_i<0x114, 0xf>((int)mx, 0));
    mn = min(mn, (uint32_t)dpp_i<0x118, 0xf>((int)mn, -1));
    mx = max(mx, (uint32_t)dpp_i<0x118, 0xf>((int)mx, 0));
    mn = (uint32_t)__builtin_amdgcn_readlane((int)mn, 15);
    mx = (uint32_t)__builtin_amdgcn_readlane((int)mx, 15);
    double lo, hi;
    if constexpr (sizeof(K) == 8) {
      lo = val_of<K>((K)mn << 32);
      hi = val_of<K>(((K)mx << 32) | 0xFFFFFFFFull);
    } else {
      lo = val_of<K>((K)mn);
      hi = val_of<K>((K)mx);
    }
    const double s = (double)NORM_TOP / (hi - lo);
    sc = uniform_d((hi > lo && s < 1e300) ? s : 0.0);
    off = uniform_d(-lo * sc);
  }
  __device__ uint32_t of_val(double x) const {
    const double t = fmin(fmax(fma(x, sc, off), 0.0), (double)(NORM_TOP - 1u));
    return (uint32_t)t;
  }
  template <typename K>
  __device__ uint32_t of_key(K k) const {
    return is_pad<K>(k) ? NORM_TOP + ((uint32_t)~k & 4095u) : of_val(val_of<K>(k));
  }
  template <typename K>
  __device__ int operator()(K k, int shift) const { return (int)((of_key<K>(k) >> shift) & 0xFFu); }
};

// One LSD pass over the block's keys (kv in position order on entry and on
// exit).  RK: how ranks are found (RK_*).  dg: the digit of an item; with
// PREP, dg.finish(prep) runs after the pass's first barrier (it may read
// what the block wrote to prep before the pass).  wc: [16][256] ints, gs: [4][256] ints, wt: [4].  TOVAL (the last
// pass): the values of the keys are scattered instead (double for double
// keys, float for float keys, in the same buffer) and kv is left as it was.
template <typename K, int RK, typename DG, int KPT, bool TOVAL = false, bool PREP = false>
__device__ inline void lds_radix_pass(K (&kv)[KPT], int shift, DG& dg, K* __restrict__ sk,
                                      int* __restrict__ wc, int* __restrict__ gs,
                                      int* __restrict__ wt, const uint32_t* prep = nullptr) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint64_t below = (1ull << lane) - 1ull;
  for (int e = tid; e < 16 * 256; e += SS_NT) wc[e] = 0;
  __syncthreads();
  if constexpr (PREP) dg.template finish<K>(prep);
  int dr[KPT];   // digit << 16 | rank within (wave, digit)
#pragma unroll
  for (int i = 0; i < KPT; ++i) {
    const int d = dg(kv[i], shift);
    if constexpr (RK == RK_ATOM) {
      dr[i] = (d << 16) | atomicAdd(&wc[w * 256 + d], 1);
    } else if constexpr (RK == RK_PEEL) {
      // every lane is active here; each round takes the lanes that share the
      // lowest remaining lane's digit
      uint64_t left = ~0ull;
      int rank = 0;
      while (left) {
        const int lead = __ffsll((long long)left) - 1;
        const int dl = __builtin_amdgcn_readlane(d, lead);
        const uint64_t m = __ballot(d == dl);
        const int cur = wc[w * 256 + dl];
        if (d == dl) rank = cur + __popcll(m & below);
        if (lane == lead) wc[w * 256 + dl] = cur + __popcll(m);
        left &= ~m;
      }
      dr[i] = (d << 16) | rank;
    } else {
      uint64_t match = ~0ull;
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const uint64_t bb = __ballot((d >> b) & 1);
        match &= ((d >> b) & 1) ? bb : ~bb;
      }
      const int before = __popcll(match & below);
      const int cur = wc[w * 256 + d];
      dr[i] = (d << 16) | (cur + before);
      if (before == 0) wc[w * 256 + d] = cur + __popcll(match);
    }
  }
  __syncthreads();
  // offsets of (wave, digit): digit base + earlier waves of the same digit.
  // Thread (g, d) scans waves 4g..4g+3 of digit d.
  const int d = tid & 255, g = tid >> 8;
  int c[4];
  {
    int run = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      c[k] = run;
      run += wc[(g * 4 + k) * 256 + d];
    }
    gs[g * 256 + d] = run;
  }
  __syncthreads();
  if (tid < 256) {   // waves 0..3: digit d = tid, scan of digit totals
    const int t0 = gs[d], t1 = gs[256 + d], t2 = gs[512 + d], t3 = gs[768 + d];
    const int tot = t0 + t1 + t2 + t3;
    int x = tot;
    x = wave_incl_sum(x);
    if (lane == 63) wt[w] = x;
    const int ex = x - tot;   // exclusive within this wave's 64 digits
    gs[d] = ex;
    gs[256 + d] = ex + t0;
    gs[512 + d] = ex + t0 + t1;
    gs[768 + d] = ex + t0 + t1 + t2;
  }
  __syncthreads();
  {
    int base = gs[g * 256 + d];
    for (int k = 0; k < (d >> 6); ++k) base += wt[k];
#pragma unroll
    for (int k = 0; k < 4; ++k) wc[(g * 4 + k) * 256 + d] = base + c[k];
  }
  __syncthreads();
  if constexpr (TOVAL) {
    using V = typename std::conditional<sizeof(K) == 8, double, float>::type;
    V* __restrict__ sv = reinterpret_cast<V*>(sk);
#pragma unroll
    for (int i = 0; i < KPT; ++i) {
      const int di = dr[i] >> 16;
      sv[wc[w * 256 + di] + (dr[i] & 0xFFFF)] = (V)val_of<K>(kv[i]);
    }
    __syncthreads();
    return;
  }
#pragma unroll
  for (int i = 0; i < KPT; ++i) {
    const int di = dr[i] >> 16;
    sk[wc[w * 256 + di] + (dr[i] & 0xFFFF)] = kv[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < KPT; ++i) kv[i] = sk[w * KPT * 64 + i * 64 + lane];
}

// Sort key of a value under the order-key passes: the high half of a double's
// order key, or a float's order key (for float data it is the whole key).
struct Key32 {
  __device__ uint32_t of_val(double x) const {
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    return (uint32_t)(((b >> 63) ? ~b : (b | 0x8000000000000000ull)) >> 32);
  }
  __device__ uint32_t of_val(float x) const {
    const uint32_t b = __float_as_uint(x);
    return (b >> 31) ? ~b : (b | 0x80000000u);
  }
};
struct KeyNormV {   // the normalised key of a value (see DigitNorm)
  DigitNorm dn;
  __device__ uint32_t of_val(double x) const { return dn.of_val(x); }
  __device__ uint32_t of_val(float x) const { return dn.of_val((double)x); }
};

// Check of sv[0..L) after passes that ordered it on the key kf (a monotone
// function of the value), and the fix-up of runs of equal keys.  Thread t
// reads its range [a0, a0 + n) into x and compares every adjacent pair.  A
// descent between unequal keys, or a padding value (NaN) inside the segment,
// fails the check; a descent between equal keys marks its run.  When there
// are at most max_desc descents, each run that holds one is listed from its
// first descent (the walks only read) and then put in order by insertion
// sort by one thread; runs longer than FIXUP_RUN or costlier than
// FIXUP_MOVES fail.  Returns true (the same in every thread) on failure;
// otherwise x holds the sorted range.  flg[0..3) must be zero on entry and
// no thread may still read them from an earlier use.
template <typename V, int RN, typename KF>
__device__ bool check_fix(V* __restrict__ sv, int L, int a0, int n, V (&x)[RN], KF kf,
                          int max_desc, int* flg, int* runs) {
#pragma unroll
  for (int k = 0; k < RN; ++k) {   // a0 + RN <= CAP + RN: no branches
    const V t = sv[a0 + k];
    x[k] = k < n ? t : (V)0;
  }
  uint32_t desc = 0;
  bool bad = false;
  {
    const V nxt = sv[a0 + n];   // a0 + n <= L
#pragma unroll
    for (int k = 0; k < RN; ++k) {
      if (k < n) {
        const V a = x[k];
        const V b2 = (k + 1 < n) ? x[k + 1] : nxt;
        bad = bad || !(a == a);
        if (a0 + k + 1 < L && a > b2) {
          if (kf.of_val(a) != kf.of_val(b2)) bad = true;
          else desc |= 1u << k;
        }
      }
    }
  }
  if (bad) atomicOr(&flg[1], 1);
  if (desc) atomicAdd(&flg[0], __popc(desc));
  __syncthreads();
  if (flg[1] || flg[0] > max_desc) return true;
  if (!flg[0]) return false;
  for (uint32_t dm = desc; dm; dm &= dm - 1u) {
    const int q = a0 + __ffs(dm) - 1;
    const V vq = sv[q];
    const uint32_t kq = kf.of_val(vq);
    int s0 = q;
    bool first = true, over = false;
    V right = vq;
    while (s0 > 0) {
      if (q - s0 >= FIXUP_RUN) { over = true; break; }
      const V left = sv[s0 - 1];
      if (kf.of_val(left) != kq) break;
      if (left > right) { first = false; break; }   // an earlier descent takes the run
      right = left;
      --s0;
    }
    if (!first) continue;
    int e = q + 2;
    while (!over && e < L && kf.of_val(sv[e]) == kq) {
      if (e - s0 >= FIXUP_RUN) over = true;
      ++e;
    }
    if (over) {
      atomicOr(&flg[1], 1);
      continue;
    }
    const int slot = atomicAdd(&flg[2], 1);
    if (slot < FIXUP_LIST) {
      runs[2 * slot] = s0;
      runs[2 * slot + 1] = e;
    } else {
      atomicOr(&flg[1], 1);
    }
  }
  __syncthreads();
  const int nr = min(flg[2], FIXUP_LIST);
  for (int t = threadIdx.x; t < nr && !flg[1]; t += SS_NT) {
    const int s0 = runs[2 * t], e = runs[2 * t + 1];
    int moves = 0;
    for (int a = s0 + 1; a < e && moves <= FIXUP_MOVES; ++a) {
      const V xa = sv[a];
      int b = a;
      while (b > s0 && sv[b - 1] > xa && moves <= FIXUP_MOVES) {
        sv[b] = sv[b - 1];
        --b;
        ++moves;
      }
      sv[b] = xa;
    }
    if (moves > FIXUP_MOVES) atomicOr(&flg[1], 1);
  }
  __syncthreads();
  if (flg[1]) return true;
#pragma unroll
  for (int k = 0; k < RN; ++k) {
    const V t = sv[a0 + k];
    x[k] = k < n ? t : (V)0;
  }
  return false;
}

// Univariate reweighted MCD (Sec. 3.1) of a sorted LDS segment v[0..L), with
// RN readable slots past L.  Thread t takes the positions [t S, t S + S) of
// the segment (clipped to L), S odd (so that the threads of a wave start
// their ranges in different LDS banks) and S <= RN, so every loop is unrolled
// over RN with its reads issued together; no value is held across a
// barrier.  The operations are those of segstat_body (prefix sums of the
// values centred at the middle order statistic, windows ranked by
// hd s2 - s1^2, reweighting of the raw fit), in order within each range.  Scratch: red, pfa, pfb hold SS_NT doubles each; the result is
// valid in thread 0.
template <typename V, int RN>
__device__ __forceinline__ SegStat segstat_regs(const V* __restrict__ v, int L, int S, int a0, int a1,
                                                double craw, double q1,
                                                double crew, double* red, double* pfa,
                                                double* pfb) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  SegStat r{};
  const int n = a1 - a0;
  const int hh = L / 2 + 1;
  const double hd = (double)hh;
  const double c = (double)v[L / 2];
  // window ends j + hh: position hh mod S of a range (the end L aside)
  const int r0 = hh % S;
  // centred sums over the range, and over its first r0 positions
  double pa[2] = {0.0, 0.0}, pr[2] = {0.0, 0.0};
  V xin[RN];
#pragma unroll
  for (int k = 0; k < RN; ++k) xin[k] = v[a0 + k];
#pragma unroll
  for (int k = 0; k < RN; ++k) {
    if (k == r0) {
      pr[0] = pa[0];
      pr[1] = pa[1];
    }
    if (k < n) {
      const double d = (double)xin[k] - c;
      pa[0] += d;
      pa[1] = fma(d, d, pa[1]);
    }
  }
  if (r0 >= RN) {
    pr[0] = pa[0];
    pr[1] = pa[1];
  }
  // exclusive prefix over the block: wave scans, then the wave totals
  // scanned by 16 lanes of every wave (fixed order, so deterministic)
  double ex[2], tot[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const double inc = wave_incl_sum(pa[q]);
    if (lane == 63) red[q * SS_WV + w] = inc;
    ex[q] = dpp_d<0x138, 0xf>(inc, 0.0);   // wave_shr 1: the previous lane's
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    double t = red[q * SS_WV + (lane & 15)];
    t += dpp_d<0x111, 0xf>(t, 0.0);   // row_shr 1, 2, 4, 8: inclusive within each 16 lanes
    t += dpp_d<0x112, 0xf>(t, 0.0);
    t += dpp_d<0x114, 0xf>(t, 0.0);
    t += dpp_d<0x118, 0xf>(t, 0.0);
    const double before = w > 0 ? lane_bcast_d(t, w - 1) : 0.0;
    tot[q] = lane_bcast_d(t, SS_WV - 1);
    ex[q] += before;
  }
  const double P1a = ex[0], P2a = ex[1];
  // publish the prefix at a0 + r0
  pfa[tid] = P1a + pr[0];
  pfb[tid] = P2a + pr[1];
  const int nw = L - hh + 1;                 // number of windows
  const int j0 = a0, j1 = a1 < nw ? a1 : nw;
  __syncthreads();
  double best = INFINITY, b1 = 0.0, b2 = 0.0;
  int64_t bj = -1;
  if (j0 < j1) {
    // prefix at j0 + hh <= L: the owner's published prefix, or the total
    const int pos = j0 + hh;
    double q1h = tot[0], q2h = tot[1];
    if (pos < L) {
      const int ow = pos / S;                // pos = ow S + r0
      q1h = pfa[ow];
      q2h = pfb[ow];
    }
    // (v holds RN readable slots past L: j0 + hh <= L)
    V x[RN], y[RN];
#pragma unroll
    for (int k = 0; k < RN; ++k) {
      x[k] = v[a0 + k];
      y[k] = v[j0 + hh + k];
    }
    // windows are ranked by hd * s2 - s1^2 = hd (hd - 1) var (no division
    // in the loop); the variance itself is formed from the best window's sums
    double q1l = P1a, q2l = P2a;
#pragma unroll
    for (int k = 0; k < RN; ++k) {
      const int j = j0 + k;
      if (j < j1) {
        const double s1 = q1h - q1l, s2 = q2h - q2l;
        const double cr = fma(s2, hd, -(s1 * s1));
        if (cr < best) { best = cr; bj = j; b1 = s1; b2 = s2; }
        const double dl = (double)x[k] - c;
        q1l += dl;
        q2l = fma(dl, dl, q2l);
        if (j + hh < L) {
          const double dh = (double)y[k] - c;
          q1h += dh;
          q2h = fma(dh, dh, q2h);
        }
      }
    }
  }
  // smallest criterion, ties to the lowest start; the lane that owns the
  // winning wave's window publishes its variance and window sum; the 16
  // wave results are reduced by 16 lanes of every wave
  double* __restrict__ rb = red + 64;
  {
    const int64_t own = bj;
    wave_argmin(best, bj);
    if (own >= 0 && own == bj) {
      rb[SS_WV + w] = (b2 - b1 * b1 / hd) / (hd - 1.0);
      rb[2 * SS_WV + w] = b1;
    }
    if (lane == 0) {
      rb[w] = best;
      reinterpret_cast<int64_t*>(rb)[3 * SS_WV + w] = bj;
    }
  }
  __syncthreads();
  double cb = rb[lane & 15];
  int64_t jb = reinterpret_cast<const int64_t*>(rb)[3 * SS_WV + (lane & 15)];
  argmin_step<0x111, 0xf>(cb, jb);   // within each row of 16 lanes
  argmin_step<0x112, 0xf>(cb, jb);
  argmin_step<0x114, 0xf>(cb, jb);
  argmin_step<0x118, 0xf>(cb, jb);
  const int64_t js = lane_bcast_l(jb, 15);
  const int qw = min((int)(js / (64 * S)), SS_WV - 1);   // the wave that holds start js
  const double wmin = rb[SS_WV + qw], s1w = rb[2 * SS_WV + qw];
  const double mu_raw = c + s1w / hd;
  const double var_raw = wmin * craw;
  // reweighting: keep (v - mu_raw)^2 <= q1 var_raw
  const double lim = q1 * var_raw;
  double cs[3] = {0.0, 0.0, 0.0};
  {
    V x[RN];
#pragma unroll
    for (int k = 0; k < RN; ++k) x[k] = v[a0 + k];
#pragma unroll
    for (int k = 0; k < RN; ++k)
      if (k < n) {
        const double xv = (double)x[k];
        const double e = xv - mu_raw;
        if (e * e <= lim) {
          const double d = xv - c;
          cs[0] += 1.0;
          cs[1] += d;
          cs[2] = fma(d, d, cs[2]);
        }
      }
  }
  double* __restrict__ rs = red + 128;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double t = wave_sum(cs[k]);
    if (lane == 0) rs[k * SS_WV + w] = t;
  }
  __syncthreads();
  if (tid == 0) {
    double N = 0.0, S1 = 0.0, S2 = 0.0;
    for (int q = 0; q < SS_WV; ++q) {
      N += rs[q];
      S1 += rs[SS_WV + q];
      S2 += rs[2 * SS_WV + q];
    }
    r.mu_raw = mu_raw;
    r.var_raw = var_raw;
    r.start = js;
    r.n_kept = (int64_t)N;
    r.mu = N > 0 ? c + S1 / N : NAN;
    r.var = N > 1 ? (S2 - S1 * S1 / N) / (N - 1.0) * crew : 0.0;
  }
  return r;
}

template <typename K, int KPT>
__global__ __launch_bounds__(SS_NT) void k_seg_lds(const K* __restrict__ keys,
                                                   const int64_t* __restrict__ seg_off,
                                                   const int64_t* __restrict__ seg_len,
                                                   const double* __restrict__ seg_craw,
                                                   int seg_first, double q1, double crew, int mode,
                                                   SegStat* __restrict__ out) {
  using V = typename std::conditional<sizeof(K) == 8, double, float>::type;
  constexpr int CAP = SS_NT * KPT;             // keys per block
  constexpr int RN = KPT + 1;                  // longest estimator range
  __shared__ K sk[CAP + RN + 1];               // keys, then values (sv); spare
                                               // slots for the range reads
  __shared__ double scratch[3 * SS_NT];        // digit counters / fix-up list / estimator
  int* wc = reinterpret_cast<int*>(scratch);   // [16][256] during the sort
  int* runs = reinterpret_cast<int*>(scratch);   // [FIXUP_LIST][2] after it
  static_assert(2 * FIXUP_LIST <= 6 * SS_NT, "fix-up list exceeds the scratch");
  __shared__ int gs[4 * 256 + 8];              // group sums, wave totals, flags
  int* wt = gs + 4 * 256;
  int* flg = gs + 4 * 256 + 4;                 // [0] descents, [1] redo, [2] runs listed
  V* sv = reinterpret_cast<V*>(sk);
  const int sb = blockIdx.x;                   // index into seg_craw / out
  const int sg = seg_first + sb;               // absolute segment
  const K* __restrict__ src = keys + seg_off[sg];
  const int L = (int)seg_len[sg];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (L <= 0) {   // uniform
    if (tid == 0) out[sb] = SegStat{};
    return;
  }
  K kv[KPT];
  auto load = [&]() {
#pragma unroll
    for (int i = 0; i < KPT; ++i) {
      const int pos = w * KPT * 64 + i * 64 + lane;
      kv[i] = pos < L ? src[pos] : pad_key<K>(pos);
    }
  };
  // this thread's contiguous range of sorted positions: S (odd) from t S
  const int S = ((L + SS_NT - 1) / SS_NT) | 1;   // <= KPT + 1
  const int a0 = min(tid * S, L), a1 = min(a0 + S, L);
  const int n = a1 - a0;
  V x[RN];
  auto load_range = [&]() {
#pragma unroll
    for (int k = 0; k < RN; ++k) {   // a0 + RN <= CAP + RN: no branches
      const V t = sv[a0 + k];
      x[k] = k < n ? t : (V)0;
    }
  };
  load();
  // bounds of the segment's values for the normalised key: the smallest and
  // largest high halves of the order keys (one 32-bit comparison per key);
  // the reduction over the waves happens in the first pass
  DigitNorm dn;
  {
    uint32_t mn = 0xFFFFFFFFu, mx = 0u;
#pragma unroll
    for (int i = 0; i < KPT; ++i) {
      const uint32_t hk = (uint32_t)(kv[i] >> (8 * sizeof(K) - 32));
      mn = min(mn, hk);   // padding is the largest key
      if (w * KPT * 64 + i * 64 + lane < L) mx = max(mx, hk);
    }
    mn = wave_min_u32(mn);
    mx = wave_max_u32(mx);
    uint32_t* rr = reinterpret_cast<uint32_t*>(scratch + 2 * SS_NT);   // clear of the counters
    if (lane == 0) {
      rr[w] = mn;
      rr[SS_WV + w] = mx;
    }
    if (tid < 3) flg[tid] = 0;   // first read after the passes' barriers
  }
  lds_radix_pass<K, RK_ATOM, DigitNorm, KPT, false, true>(
      kv, 0, dn, sk, wc, gs, wt, reinterpret_cast<const uint32_t*>(scratch + 2 * SS_NT));
  lds_radix_pass<K, RK_ATOM, DigitNorm, KPT>(kv, 8, dn, sk, wc, gs, wt);
  lds_radix_pass<K, RK_ATOM, DigitNorm, KPT, true>(kv, 16, dn, sk, wc, gs, wt);
  if (check_fix<V, RN>(sv, L, a0, n, x, KeyNormV{dn}, NORM_MAX_DESC, flg, runs)) {
    // uniform.  Values crowded into few keys (heavy tails, far outliers):
    // left to k_seg_lds_slow, marked by start = SEG_REDO
    if (tid == 0) {
      SegStat r{};
      r.start = SEG_REDO;
      out[sb] = r;
    }
    return;
  }
  if (mode != SEGSTAT_UNIMCD) {
    if (tid == 0) out[sb] = segstat_order<V>(sv, L, mode);
    return;
  }
  const SegStat r = segstat_regs<V, RN>(sv, L, S, a0, a1, seg_craw[sb], q1, crew, scratch,
                                         scratch + SS_NT, scratch + 2 * SS_NT);
  if (tid == 0) out[sb] = r;
}

// The segments k_seg_lds left (start = SEG_REDO), each by one block of a
// small grid: LSD passes on the high 32 bits of the order key (resolution
// relative to each value), checked and fixed up the same way; failing that,
// the full-width sort with ballot ranking only.  Then the same estimator.
template <typename K, int KPT>
__global__ __launch_bounds__(SS_NT) void k_seg_lds_slow(const K* __restrict__ keys,
                                                        const int64_t* __restrict__ seg_off,
                                                        const int64_t* __restrict__ seg_len,
                                                        const double* __restrict__ seg_craw,
                                                        int seg_first, int nseg, double q1,
                                                        double crew, int mode,
                                                        SegStat* __restrict__ out) {
  using V = typename std::conditional<sizeof(K) == 8, double, float>::type;
  constexpr int CAP = SS_NT * KPT;
  constexpr int RN = KPT + 1;
  __shared__ K sk[CAP + RN + 1];
  __shared__ double scratch[3 * SS_NT];
  int* wc = reinterpret_cast<int*>(scratch);
  int* runs = reinterpret_cast<int*>(scratch);
  __shared__ int gs[4 * 256 + 8];
  int* wt = gs + 4 * 256;
  int* flg = gs + 4 * 256 + 4;
  V* sv = reinterpret_cast<V*>(sk);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // this block's segments sb = blockIdx.x + t gridDim.x (t < SS_NT: the
  // grid is sized for that), all marks read at once into a bit set
  __shared__ uint32_t redo_bits[SS_NT / 32];
  if (tid < SS_NT / 32) redo_bits[tid] = 0u;
  __syncthreads();
  if (blockIdx.x + (int64_t)tid * gridDim.x < nseg &&
      out[blockIdx.x + tid * gridDim.x].start == SEG_REDO)
    atomicOr(&redo_bits[tid >> 5], 1u << (tid & 31));
  __syncthreads();
  for (int wd = 0; wd < SS_NT / 32; ++wd)
  for (uint32_t bits = redo_bits[wd]; bits; bits &= bits - 1u) {   // uniform
    const int sb = blockIdx.x + (wd * 32 + __ffs(bits) - 1) * gridDim.x;
    const int sg = seg_first + sb;
    const K* __restrict__ src = keys + seg_off[sg];
    const int L = (int)seg_len[sg];
    K kv[KPT];
    auto load = [&]() {
#pragma unroll
      for (int i = 0; i < KPT; ++i) {
        const int pos = w * KPT * 64 + i * 64 + lane;
        kv[i] = pos < L ? src[pos] : pad_key<K>(pos);
      }
    };
    const int S = ((L + SS_NT - 1) / SS_NT) | 1;
    const int a0 = min(tid * S, L), a1 = min(a0 + S, L), n = a1 - a0;
    __syncthreads();   // the previous segment is done with the shared arrays
    if (tid < 3) flg[tid] = 0;
    load();
    DigitKey32 d32;
    lds_radix_pass<K, RK_ATOM, DigitKey32, KPT>(kv, 0, d32, sk, wc, gs, wt);
    lds_radix_pass<K, RK_ATOM, DigitKey32, KPT>(kv, 8, d32, sk, wc, gs, wt);
    lds_radix_pass<K, RK_ATOM, DigitKey32, KPT>(kv, 16, d32, sk, wc, gs, wt);
    lds_radix_pass<K, RK_PEEL, DigitKey32, KPT, true>(kv, 24, d32, sk, wc, gs, wt);
    V x[RN];
    if (check_fix<V, RN>(sv, L, a0, n, x, Key32{}, CAP, flg, runs)) {
      __syncthreads();
      load();
      DigitFull df;
#pragma unroll 1
      for (int shift = 0; shift < 8 * (int)sizeof(K) - 8; shift += 8)
        lds_radix_pass<K, RK_BALLOT, DigitFull, KPT>(kv, shift, df, sk, wc, gs, wt);
      lds_radix_pass<K, RK_BALLOT, DigitFull, KPT, true>(kv, 8 * (int)sizeof(K) - 8, df, sk, wc,
                                                         gs, wt);
    }
    SegStat r{};
    if (mode != SEGSTAT_UNIMCD) {
      if (tid == 0) r = segstat_order<V>(sv, L, mode);
    } else {
      r = segstat_regs<V, RN>(sv, L, S, a0, a1, seg_craw[sb], q1, crew, scratch, scratch + SS_NT,
                              scratch + 2 * SS_NT);
    }
    if (tid == 0) out[sb] = r;
  }
}

// ---------------------------------------------------------------------------
// Sample sort of long segments.  Splitters are taken from a sorted strided
// sample of each segment; one pass sends every key to its class: the open
// range between two neighbouring splitters, or the value of a splitter.
// Each range (a bucket of at most BK_CAP keys) is then sorted in LDS by one
// block, with the passes and check of k_seg_lds, and written to its final
// place, followed by its upper splitter's value as often as that value
// occurs.  Classes of a segment with nb buckets, in key order:
// range 0, value 0, range 1, ..., value nb-2, range nb-1 (class 2i is range
// i, class 2i + 1 the value of splitter i).
// ---------------------------------------------------------------------------
constexpr int BK_NT = 256;           // threads of the sample kernel
constexpr int BK_SAMPLE = 2048;      // sample of up to 16 buckets (128 keys per bucket)
constexpr int BK_SAMPLE_BIG = 8192;  // sample of up to BK_NBMAX buckets
constexpr int BK_KPT = 16;
constexpr int BK_CAP = SS_NT * BK_KPT;   // keys per bucket (one LDS segment)
constexpr int BK_EXP = 10240;        // expected keys per bucket (capacity / 1.6)
constexpr int BK_NBMAX = 64;         // buckets per segment
static_assert(2 * BK_NBMAX <= RS_NT, "one thread per class in k_bk_scatter");
static_assert(BK_SAMPLE_BIG <= BK_CAP, "a sampled segment holds more keys than the sample");
static_assert(BK_SAMPLE_BIG >= 128 * BK_NBMAX, "128 sampled keys per bucket");

// Order key of a value: the inverse of val_of.
__device__ inline uint64_t key_of_val(double x) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ inline uint32_t key_of_val(float x) {
  const uint32_t b = __float_as_uint(x);
  return (b >> 31) ? ~b : (b | 0x80000000u);
}

// Class of key k among the nsp sorted splitters sp: 2 i + (k == sp[i]),
// i = the number of splitters below k.
template <typename K>
__device__ inline int bk_class(K k, const K* sp, int nsp) {
  int i = 0;
#pragma unroll
  for (int st = BK_NBMAX / 2; st > 0; st >>= 1)
    if (i + st <= nsp && sp[i + st - 1] < k) i += st;
  return 2 * i + ((i < nsp && sp[i] == k) ? 1 : 0);
}

// One block per segment: clears its class counters and, for nb >= 2,
// writes the nb - 1 splitters: order statistics i S / nb of the sample of
// keys (2 s + 1) L / (2 S), s < S, sorted by a bitonic network; S is the
// smallest power of two from 256 to SMAX holding 128 keys per bucket.
template <typename K, int SMAX>
__global__ __launch_bounds__(BK_NT) void k_bk_sample(const K* __restrict__ keys,
                                                     const int64_t* __restrict__ seg_off,
                                                     const int64_t* __restrict__ seg_len,
                                                     const int32_t* __restrict__ bk0,
                                                     int seg_first, int bk_first,
                                                     K* __restrict__ split,
                                                     int32_t* __restrict__ cnt) {
  __shared__ K smp[SMAX];
  const int sg = seg_first + blockIdx.x;
  const int j0 = bk0[sg] - bk_first, nb = bk0[sg + 1] - bk0[sg];
  const int tid = threadIdx.x;
  for (int c = tid; c < 2 * nb; c += BK_NT) cnt[2 * j0 + c] = 0;
  if (nb < 2) return;   // uniform
  const int64_t L = seg_len[sg];   // > BK_CAP >= SMAX: distinct sampled positions
  const K* __restrict__ src = keys + seg_off[sg];
  int S = 256;
  while (S < 128 * nb && S < SMAX) S <<= 1;
  for (int i = tid; i < S; i += BK_NT) smp[i] = src[((2 * (int64_t)i + 1) * L) / (2 * S)];
  __syncthreads();
  for (int k = 2; k <= S; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < S / 2; i += BK_NT) {
        const int lo = 2 * i - (i & (j - 1)), hi = lo + j;   // lo: bit log2(j) clear
        const K a = smp[lo], b = smp[hi];
        if ((a > b) == ((lo & k) == 0)) {
          smp[lo] = b;
          smp[hi] = a;
        }
      }
      __syncthreads();
    }
  }
  for (int i = tid + 1; i < nb; i += BK_NT) split[j0 + i - 1] = smp[(i * S) / nb];
}

// One block per radix tile (RS_TILE keys of one segment): the class of
// every key and its rank within the tile's keys of that class (LDS
// atomics), one global atomic per class for the tile's place in its
// bucket, then each range key written straight to its bucket's staging
// slots (stg[j BK_CAP ...] for bucket j of the plan): a tile's keys of one
// class land in one contiguous run.  Value classes are only counted.  A
// bucket filled beyond BK_CAP sets *flag.
template <typename K>
__global__ __launch_bounds__(RS_NT) void k_bk_scatter(const K* __restrict__ keys,
                                                      K* __restrict__ stg,
                                                      const SegTile* __restrict__ tiles,
                                                      const int64_t* __restrict__ seg_off,
                                                      const int64_t* __restrict__ seg_len,
                                                      const int32_t* __restrict__ bk0,
                                                      int bk_first, const K* __restrict__ split,
                                                      int32_t* __restrict__ cnt,
                                                      int32_t* __restrict__ flag) {
  constexpr int NC = 2 * BK_NBMAX;
  __shared__ K sp[BK_NBMAX];
  __shared__ int lc[NC], gb[NC];
  const SegTile t = tiles[blockIdx.x];
  const int sg = t.seg;
  const int64_t so = seg_off[sg];
  const int64_t base = so + (int64_t)t.tile * RS_TILE;
  const int nvalid = (int)min((int64_t)RS_TILE, so + seg_len[sg] - base);
  const int j0 = bk0[sg] - bk_first, nb = bk0[sg + 1] - bk0[sg], nsp = nb - 1;
  const int tid = threadIdx.x;
  if (tid < nsp) sp[tid] = split[j0 + tid];
  if (tid < NC) lc[tid] = 0;
  __syncthreads();
  K kv[RS_ITEMS];
  int cr[RS_ITEMS];   // class << 16 | rank within the tile's class
#pragma unroll
  for (int i = 0; i < RS_ITEMS; ++i) {
    const int q = i * RS_NT + tid;
    kv[i] = q < nvalid ? keys[base + q] : (K)0;
  }
#pragma unroll
  for (int i = 0; i < RS_ITEMS; ++i) {
    cr[i] = -1;
    if (i * RS_NT + tid < nvalid) {
      const int c = bk_class(kv[i], sp, nsp);
      cr[i] = (c << 16) | atomicAdd(&lc[c], 1);
    }
  }
  __syncthreads();
  if (tid < NC) {
    const int n = lc[tid];
    gb[tid] = n ? atomicAdd(&cnt[2 * j0 + tid], n) : 0;   // n = 0 beyond class 2 nb - 2
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < RS_ITEMS; ++i) {
    const int c = cr[i] >> 16;
    if (cr[i] >= 0 && !(c & 1)) {
      const int pos = gb[c] + (cr[i] & 0xFFFF);
      if (pos < BK_CAP) stg[(int64_t)(j0 + (c >> 1)) * BK_CAP + pos] = kv[i];
      else *flag = 1;
    }
  }
}

// Where bucket jl of the plan goes: its segment's first key, and the keys
// of the classes before it (every wave reads the counts; no barrier).
struct BkPlace {
  int64_t out;   // first output position of the bucket's keys
  int L;         // keys of the bucket (capped at BK_CAP)
  int sg, b, j0, nb;
};
__device__ inline BkPlace bk_place(int jl, const SegTile* __restrict__ bk_tab,
                                   const int64_t* __restrict__ seg_off,
                                   const int32_t* __restrict__ bk0, int bk_first,
                                   const int32_t* __restrict__ cnt) {
  BkPlace r;
  const SegTile e = bk_tab[bk_first + jl];
  r.sg = e.seg;
  r.b = e.tile;
  r.j0 = bk0[r.sg] - bk_first;
  r.nb = bk0[r.sg + 1] - bk0[r.sg];
  const int32_t* __restrict__ c = cnt + 2 * r.j0;
  const int lane = threadIdx.x & 63;
  int s = 0;
  for (int k = lane; k < 2 * r.b; k += 64) s += c[k];
  s = __builtin_amdgcn_readlane(wave_incl_sum(s), 63);
  r.out = seg_off[r.sg] + s;
  r.L = min(c[2 * r.b], BK_CAP);
  return r;
}

// The bucket's upper splitter value, repeated as often as it occurs.
template <typename K>
__device__ inline void bk_fill_value(const BkPlace& pl, K* __restrict__ keys,
                                     const K* __restrict__ split,
                                     const int32_t* __restrict__ cnt) {
  if (pl.b >= pl.nb - 1) return;
  const int ne = cnt[2 * pl.j0 + 2 * pl.b + 1];
  const int64_t o = pl.out + cnt[2 * pl.j0 + 2 * pl.b];   // after every key of the range
  const K v = split[pl.j0 + pl.b];
  for (int i = threadIdx.x; i < ne; i += SS_NT) keys[o + i] = v;
}

template <typename K, typename V>
__device__ inline void bk_write(const BkPlace& pl, const V* __restrict__ sv, K* __restrict__ keys) {
  for (int i = threadIdx.x; i < pl.L; i += SS_NT) keys[pl.out + i] = (K)key_of_val(sv[i]);
}

// The bucket kernels instantiate the shared passes and checks with types of
// their own: sharing the instantiations of k_seg_lds made the compiler
// spill 62 registers in k_seg_lds<uint64_t, 16> (none with separate ones).
struct BkNorm : DigitNorm {};
struct BkKey32Digit : DigitKey32 {};
struct BkFullDigit : DigitFull {};
struct BkKeyNorm {
  BkNorm dn;
  __device__ uint32_t of_val(double x) const { return dn.of_val(x); }
  __device__ uint32_t of_val(float x) const { return dn.of_val((double)x); }
};
struct BkKey32 : Key32 {};

// One block per bucket: the normalised-key passes of k_seg_lds and its
// check; a bucket whose keys crowd into few normalised keys is marked
// (mark[jl] = 1) and left to k_bk_sort_slow.
template <typename K>
__global__ __launch_bounds__(SS_NT) void k_bk_sort(const K* __restrict__ stg, K* __restrict__ keys,
                                                   const SegTile* __restrict__ bk_tab,
                                                   const int64_t* __restrict__ seg_off,
                                                   const int32_t* __restrict__ bk0, int bk_first,
                                                   const K* __restrict__ split,
                                                   const int32_t* __restrict__ cnt,
                                                   int32_t* __restrict__ mark) {
  using V = typename std::conditional<sizeof(K) == 8, double, float>::type;
  constexpr int KPT = BK_KPT;
  constexpr int CAP = BK_CAP;
  constexpr int RN = KPT + 1;
  __shared__ K sk[CAP + RN + 1];
  __shared__ double scratch[3 * SS_NT];
  int* wc = reinterpret_cast<int*>(scratch);
  int* runs = reinterpret_cast<int*>(scratch);
  __shared__ int gs[4 * 256 + 8];
  int* wt = gs + 4 * 256;
  int* flg = gs + 4 * 256 + 4;
  V* sv = reinterpret_cast<V*>(sk);
  const int jl = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const BkPlace pl = bk_place(jl, bk_tab, seg_off, bk0, bk_first, cnt);
  bk_fill_value(pl, keys, split, cnt);
  const int L = pl.L;
  if (L == 0) {   // uniform
    if (tid == 0) mark[jl] = 0;
    return;
  }
  const K* __restrict__ src = stg + (int64_t)jl * BK_CAP;
  K kv[KPT];
#pragma unroll
  for (int i = 0; i < KPT; ++i) {
    const int pos = w * KPT * 64 + i * 64 + lane;
    kv[i] = pos < L ? src[pos] : pad_key<K>(pos);
  }
  const int S = ((L + SS_NT - 1) / SS_NT) | 1;
  const int a0 = min(tid * S, L), a1 = min(a0 + S, L);
  const int n = a1 - a0;
  BkNorm dn;
  {
    uint32_t mn = 0xFFFFFFFFu, mx = 0u;
#pragma unroll
    for (int i = 0; i < KPT; ++i) {
      const uint32_t hk = (uint32_t)(kv[i] >> (8 * sizeof(K) - 32));
      mn = min(mn, hk);
      if (w * KPT * 64 + i * 64 + lane < L) mx = max(mx, hk);
    }
    mn = wave_min_u32(mn);
    mx = wave_max_u32(mx);
    uint32_t* rr = reinterpret_cast<uint32_t*>(scratch + 2 * SS_NT);
    if (lane == 0) {
      rr[w] = mn;
      rr[SS_WV + w] = mx;
    }
    if (tid < 3) flg[tid] = 0;
  }
  lds_radix_pass<K, RK_ATOM, BkNorm, KPT, false, true>(
      kv, 0, dn, sk, wc, gs, wt, reinterpret_cast<const uint32_t*>(scratch + 2 * SS_NT));
  lds_radix_pass<K, RK_ATOM, BkNorm, KPT>(kv, 8, dn, sk, wc, gs, wt);
  lds_radix_pass<K, RK_ATOM, BkNorm, KPT, true>(kv, 16, dn, sk, wc, gs, wt);
  V x[RN];
  if (check_fix<V, RN>(sv, L, a0, n, x, BkKeyNorm{dn}, NORM_MAX_DESC, flg, runs)) {
    if (tid == 0) mark[jl] = 1;
    return;
  }
  if (tid == 0) mark[jl] = 0;
  bk_write(pl, sv, keys);
}

// The buckets k_bk_sort marked, each by one block of a small grid (at most
// SS_NT buckets per block): the order-key passes and the full-width sort
// of k_seg_lds_slow.
template <typename K>
__global__ __launch_bounds__(SS_NT) void k_bk_sort_slow(const K* __restrict__ stg,
                                                        K* __restrict__ keys,
                                                        const SegTile* __restrict__ bk_tab,
                                                        const int64_t* __restrict__ seg_off,
                                                        const int32_t* __restrict__ bk0,
                                                        int bk_first, int nbk,
                                                        const int32_t* __restrict__ cnt,
                                                        const int32_t* __restrict__ mark) {
  using V = typename std::conditional<sizeof(K) == 8, double, float>::type;
  constexpr int KPT = BK_KPT;
  constexpr int CAP = BK_CAP;
  constexpr int RN = KPT + 1;
  __shared__ K sk[CAP + RN + 1];
  __shared__ double scratch[3 * SS_NT];
  int* wc = reinterpret_cast<int*>(scratch);
  int* runs = reinterpret_cast<int*>(scratch);
  __shared__ int gs[4 * 256 + 8];
  int* wt = gs + 4 * 256;
  int* flg = gs + 4 * 256 + 4;
  V* sv = reinterpret_cast<V*>(sk);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  __shared__ uint32_t redo_bits[SS_NT / 32];
  if (tid < SS_NT / 32) redo_bits[tid] = 0u;
  __syncthreads();
  if (blockIdx.x + (int64_t)tid * gridDim.x < nbk && mark[blockIdx.x + tid * gridDim.x])
    atomicOr(&redo_bits[tid >> 5], 1u << (tid & 31));
  __syncthreads();
  for (int wd = 0; wd < SS_NT / 32; ++wd)
  for (uint32_t bits = redo_bits[wd]; bits; bits &= bits - 1u) {   // uniform
    const int jl = blockIdx.x + (wd * 32 + __ffs(bits) - 1) * gridDim.x;
    const BkPlace pl = bk_place(jl, bk_tab, seg_off, bk0, bk_first, cnt);
    const int L = pl.L;
    const K* __restrict__ src = stg + (int64_t)jl * BK_CAP;
    K kv[KPT];
    auto load = [&]() {
#pragma unroll
      for (int i = 0; i < KPT; ++i) {
        const int pos = w * KPT * 64 + i * 64 + lane;
        kv[i] = pos < L ? src[pos] : pad_key<K>(pos);
      }
    };
    const int S = ((L + SS_NT - 1) / SS_NT) | 1;
    const int a0 = min(tid * S, L), a1 = min(a0 + S, L), n = a1 - a0;
    __syncthreads();   // the previous bucket is done with the shared arrays
    if (tid < 3) flg[tid] = 0;
    load();
    BkKey32Digit d32;
    lds_radix_pass<K, RK_ATOM, BkKey32Digit, KPT>(kv, 0, d32, sk, wc, gs, wt);
    lds_radix_pass<K, RK_ATOM, BkKey32Digit, KPT>(kv, 8, d32, sk, wc, gs, wt);
    lds_radix_pass<K, RK_ATOM, BkKey32Digit, KPT>(kv, 16, d32, sk, wc, gs, wt);
    lds_radix_pass<K, RK_PEEL, BkKey32Digit, KPT, true>(kv, 24, d32, sk, wc, gs, wt);
    V x[RN];
    if (check_fix<V, RN>(sv, L, a0, n, x, BkKey32{}, CAP, flg, runs)) {
      __syncthreads();
      load();
      BkFullDigit df;
#pragma unroll 1
      for (int shift = 0; shift < 8 * (int)sizeof(K) - 8; shift += 8)
        lds_radix_pass<K, RK_BALLOT, BkFullDigit, KPT>(kv, shift, df, sk, wc, gs, wt);
      lds_radix_pass<K, RK_BALLOT, BkFullDigit, KPT, true>(kv, 8 * (int)sizeof(K) - 8, df, sk, wc,
                                                         gs, wt);
    }
    bk_write(pl, sv, keys);
  }
}

// ---------------------------------------------------------------------------
// Univariate MCD over long sorted segments, spread over many blocks (the
// radix tiles, RS_TILE keys each): block sums -> per-segment prefix -> window
// minima per block -> per-segment choice of the window -> kept-row sums ->
// per-segment result.  Same estimator as segstat_body, every reduction in a
// fixed order.
// ---------------------------------------------------------------------------
constexpr int MB_NT = RS_NT;                  // 256 threads, RS_ITEMS keys each

constexpr int MB_WV = MB_NT / 64;

// Centred partial sums of v[a, b), b - a <= RS_TILE, by the whole block:
// lane-strided (coalesced) loads, all issued before the first sum, a fixed
// order per thread, then block sums.
template <typename K>
__device__ inline void blk_range_sums(const K* __restrict__ v, int64_t a, int64_t b, double c,
                                      double* red, double& s1, double& s2) {
  double l[2] = {0.0, 0.0};
  K kv[RS_ITEMS];
#pragma unroll
  for (int i = 0; i < RS_ITEMS; ++i) {
    const int64_t k = a + i * MB_NT + threadIdx.x;
    kv[i] = k < b ? v[k] : (K)0;
  }
#pragma unroll
  for (int i = 0; i < RS_ITEMS; ++i) {
    if (a + i * MB_NT + threadIdx.x < b) {
      const double d = val_of<K>(kv[i]) - c;
      l[0] += d;
      l[1] = fma(d, d, l[1]);
    }
  }
  block_sums<2, MB_WV>(l, red);
  s1 = l[0];
  s2 = l[1];
}

template <typename K>
__global__ __launch_bounds__(MB_NT) void k_mb_sums(const K* __restrict__ keys,
                                                   const SegTile* __restrict__ tiles,
                                                   const int64_t* __restrict__ seg_off,
                                                   const int64_t* __restrict__ seg_len,
                                                   double* __restrict__ bs1,
                                                   double* __restrict__ bs2) {
  __shared__ double red[MB_NT];
  const SegTile t = tiles[blockIdx.x];
  const K* __restrict__ v = keys + seg_off[t.seg];
  const int64_t L = seg_len[t.seg];
  const double c = val_of<K>(v[L / 2]);
  const int64_t a = (int64_t)t.tile * RS_TILE, b = min(a + (int64_t)RS_TILE, L);
  double s1, s2;
  blk_range_sums<K>(v, a, b, c, red, s1, s2);
  if (threadIdx.x == 0) {
    bs1[blockIdx.x] = s1;
    bs2[blockIdx.x] = s2;
  }
}

// Per segment: block sums -> exclusive prefixes; totals kept aside.  Each
// thread takes a contiguous run of the segment's tiles, in order.
__global__ __launch_bounds__(MB_NT) void k_mb_scan(const int32_t* __restrict__ seg_tile0,
                                                   int tile_first, double* __restrict__ bs1,
                                                   double* __restrict__ bs2,
                                                   double* __restrict__ tot) {
  __shared__ double red[2 * MB_WV];
  const int s = blockIdx.x, tid = threadIdx.x;
  const int t0 = seg_tile0[s] - tile_first, t1 = seg_tile0[s + 1] - tile_first;
  const int nt = t1 - t0;
  const int a = t0 + (int)(((int64_t)nt * tid) / MB_NT);
  const int b = t0 + (int)(((int64_t)nt * (tid + 1)) / MB_NT);
  double r[2] = {0.0, 0.0};
  for (int t = a; t < b; ++t) {
    r[0] += bs1[t];
    r[1] += bs2[t];
  }
  const double own1 = r[0], own2 = r[1];
  block_excl_prefix<2, true, MB_WV>(r, red);
  double r1 = r[0], r2 = r[1];
  for (int t = a; t < b; ++t) {
    const double x = bs1[t], y = bs2[t];
    bs1[t] = r1;
    bs2[t] = r2;
    r1 += x;
    r2 += y;
  }
  if (tid == MB_NT - 1) {
    tot[2 * s] = r[0] + own1;
    tot[2 * s + 1] = r[1] + own2;
  }
}

// Prefix sums P(x) of the centred values at any position x of a segment.
template <typename K>
__device__ inline void prefix_at(const K* __restrict__ v, int64_t L, double c, int64_t x,
                                 const double* bs1, const double* bs2, const double* tot,
                                 int t0rel, int s_rel, double* red, double& p1, double& p2) {
  const int64_t bx = x / RS_TILE;
  const int64_t nb = (L + RS_TILE - 1) / RS_TILE;
  if (bx >= nb) {
    p1 = tot[2 * s_rel];
    p2 = tot[2 * s_rel + 1];
    return;
  }
  double q1, q2;
  blk_range_sums<K>(v, bx * RS_TILE, x, c, red, q1, q2);
  p1 = bs1[t0rel + bx] + q1;
  p2 = bs2[t0rel + bx] + q2;
}

template <typename K>
__global__ __launch_bounds__(MB_NT) void k_mb_window(const K* __restrict__ keys,
                                                     const SegTile* __restrict__ tiles,
                                                     const int64_t* __restrict__ seg_off,
                                                     const int64_t* __restrict__ seg_len,
                                                     const int32_t* __restrict__ seg_tile0,
                                                     int tile_first, int seg_first,
                                                     const double* __restrict__ bs1,
                                                     const double* __restrict__ bs2,
                                                     const double* __restrict__ tot,
                                                     double* __restrict__ wbest,
                                                     int64_t* __restrict__ wj) {
  // the tile's window starts v[a, a + RS_TILE) and ends v[a + hh, ...) are
  // staged once, coalesced, in LDS; each thread then walks RS_ITEMS
  // consecutive starts, at a padded stride that keeps lanes off one bank
  constexpr int PADN = RS_TILE + RS_TILE / RS_ITEMS;
  __shared__ K sl[PADN], sh[PADN];
  __shared__ double red[4 * MB_WV];
  __shared__ double sb[MB_WV];
  __shared__ int64_t sj[MB_WV];
  const SegTile t = tiles[blockIdx.x];
  const K* __restrict__ v = keys + seg_off[t.seg];
  const int64_t L = seg_len[t.seg];
  const int s_rel = t.seg - seg_first;
  const int t0rel = seg_tile0[s_rel] - tile_first;
  const double c = val_of<K>(v[L / 2]);
  const int64_t hh = L / 2 + 1, nw = L - hh + 1;
  const int64_t a = (int64_t)t.tile * RS_TILE;
  const int64_t e = min(a + (int64_t)RS_TILE, nw);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double best = INFINITY;
  int64_t bj = -1;
  if (a < nw) {   // uniform over the block
    {
      K lo[RS_ITEMS], hi[RS_ITEMS];   // every load issued before the first store
#pragma unroll
      for (int i = 0; i < RS_ITEMS; ++i) {
        const int64_t pl = a + i * MB_NT + tid, ph = pl + hh;
        lo[i] = v[pl < L ? pl : L - 1];
        hi[i] = v[ph < L ? ph : L - 1];
      }
#pragma unroll
      for (int i = 0; i < RS_ITEMS; ++i) {
        const int q = i * MB_NT + tid;
        sl[q + q / RS_ITEMS] = lo[i];
        sh[q + q / RS_ITEMS] = hi[i];
      }
    }
    __syncthreads();
    double x1, x2;   // P at a + hh (block-wide, ends with a barrier)
    prefix_at<K>(v, L, c, a + hh, bs1, bs2, tot, t0rel, s_rel, red, x1, x2);
    // this thread's starts a + ja .. + RS_ITEMS; P there and at start + hh
    const int ja = tid * RS_ITEMS;
    const K* __restrict__ ml = sl + tid * (RS_ITEMS + 1);
    const K* __restrict__ mh = sh + tid * (RS_ITEMS + 1);
    double pp[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
      if (a + ja + i < L) {
        const double d = val_of<K>(ml[i]) - c;
        pp[0] += d;
        pp[1] = fma(d, d, pp[1]);
      }
      if (a + hh + ja + i < L) {
        const double d = val_of<K>(mh[i]) - c;
        pp[2] += d;
        pp[3] = fma(d, d, pp[3]);
      }
    }
    block_excl_prefix<4, true, MB_WV>(pp, red);
    double q1l = bs1[t0rel + t.tile] + pp[0], q2l = bs2[t0rel + t.tile] + pp[1];
    double q1h = x1 + pp[2], q2h = x2 + pp[3];
    // windows ranked by hd * s2 - s1^2 = hd (hd - 1) var, as in segstat_body
    const double hd = (double)hh;
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
      const int64_t j = a + ja + i;
      if (j < e) {
        const double s1 = q1h - q1l, s2 = q2h - q2l;
        const double cr = fma(s2, hd, -(s1 * s1));
        if (cr < best) { best = cr; bj = j; }
        const double dl = val_of<K>(ml[i]) - c;
        q1l += dl;
        q2l = fma(dl, dl, q2l);
        if (j + hh < L) {
          const double dh = val_of<K>(mh[i]) - c;
          q1h += dh;
          q2h = fma(dh, dh, q2h);
        }
      }
    }
  }
  // smallest criterion, ties to the lowest start (an exact min)
  wave_argmin(best, bj);
  if (lane == 0) {
    sb[w] = best;
    sj[w] = bj;
  }
  __syncthreads();
  if (tid == 0) {
    for (int q = 1; q < MB_WV; ++q) {
      const double b2 = sb[q];
      const int64_t j2 = sj[q];
      if (j2 >= 0 && (bj < 0 || b2 < best || (b2 == best && j2 < bj))) {
        best = b2;
        bj = j2;
      }
    }
    wbest[blockIdx.x] = best;
    wj[blockIdx.x] = bj;
  }
}

// Per segment: the window of smallest variance (lowest start on ties; the
// blocks rank windows by hd s2 - s1^2), the raw location and variance from
// its prefix sums, the reweighting bound.  prm[s] = {c, mu_raw, var_raw,
// lim, start}.
template <typename K>
__global__ __launch_bounds__(MB_NT) void k_mb_mid(const K* __restrict__ keys,
                                                  const int64_t* __restrict__ seg_off,
                                                  const int64_t* __restrict__ seg_len,
                                                  const int32_t* __restrict__ seg_tile0,
                                                  int tile_first, int seg_first,
                                                  const double* __restrict__ bs1,
                                                  const double* __restrict__ bs2,
                                                  const double* __restrict__ tot,
                                                  const double* __restrict__ wbest,
                                                  const int64_t* __restrict__ wj,
                                                  const double* __restrict__ seg_craw, double q1,
                                                  double* __restrict__ prm) {
  __shared__ double red[MB_NT];
  __shared__ int64_t s_j;
  const int s_rel = blockIdx.x;
  const int sg = seg_first + s_rel;
  const K* __restrict__ v = keys + seg_off[sg];
  const int64_t L = seg_len[sg];
  const int t0rel = seg_tile0[s_rel] - tile_first, t1rel = seg_tile0[s_rel + 1] - tile_first;
  {
    // smallest criterion over the segment's blocks, ties to the lowest start
    // (an exact min: the order of the comparisons does not matter)
    double b = INFINITY;
    int64_t j = -1;
    for (int t = t0rel + (int)threadIdx.x; t < t1rel; t += MB_NT) {
      const int64_t j2 = wj[t];
      const double b2 = wbest[t];
      if (j2 >= 0 && (j < 0 || b2 < b || (b2 == b && j2 < j))) { b = b2; j = j2; }
    }
    wave_argmin(b, j);
    if ((threadIdx.x & 63) == 0) {
      red[threadIdx.x >> 6] = b;
      reinterpret_cast<int64_t*>(red)[MB_WV + (threadIdx.x >> 6)] = j;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int q = 0; q < MB_WV; ++q) {
        const double b2 = red[q];
        const int64_t j2 = reinterpret_cast<const int64_t*>(red)[MB_WV + q];
        if (j2 >= 0 && (j < 0 || b2 < b || (b2 == b && j2 < j))) { b = b2; j = j2; }
      }
      s_j = j;
    }
    __syncthreads();
  }
  const double c = val_of<K>(v[L / 2]);
  const int64_t hh = L / 2 + 1, js = s_j;
  double pa1, pa2, pb1, pb2;
  prefix_at<K>(v, L, c, js, bs1, bs2, tot, t0rel, s_rel, red, pa1, pa2);
  prefix_at<K>(v, L, c, js + hh, bs1, bs2, tot, t0rel, s_rel, red, pb1, pb2);
  if (threadIdx.x == 0) {
    const double hd = (double)hh, s1 = pb1 - pa1, s2 = pb2 - pa2;
    const double mu_raw = c + s1 / hd;
    const double var_raw = (s2 - s1 * s1 / hd) / (hd - 1.0) * seg_craw[s_rel];
    double* P = prm + 5 * s_rel;
    P[0] = c;
    P[1] = mu_raw;
    P[2] = var_raw;
    P[3] = q1 * var_raw;
    P[4] = (double)js;
  }
}

template <typename K>
__global__ __launch_bounds__(MB_NT) void k_mb_kept(const K* __restrict__ keys,
                                                   const SegTile* __restrict__ tiles,
                                                   const int64_t* __restrict__ seg_off,
                                                   const int64_t* __restrict__ seg_len,
                                                   int seg_first, const double* __restrict__ prm,
                                                   double* __restrict__ k0, double* __restrict__ k1,
                                                   double* __restrict__ k2) {
  __shared__ double red[MB_NT];
  const SegTile t = tiles[blockIdx.x];
  const K* __restrict__ v = keys + seg_off[t.seg];
  const int64_t L = seg_len[t.seg];
  const double* P = prm + 5 * (t.seg - seg_first);
  const double c = P[0], mu = P[1], lim = P[3];
  const int64_t a = (int64_t)t.tile * RS_TILE, b = min(a + (int64_t)RS_TILE, L);
  double cs[3] = {0.0, 0.0, 0.0};
  K kv[RS_ITEMS];   // every load issued before the first sum
#pragma unroll
  for (int i = 0; i < RS_ITEMS; ++i) {
    const int64_t k = a + i * MB_NT + threadIdx.x;
    kv[i] = k < b ? v[k] : (K)0;
  }
#pragma unroll
  for (int i = 0; i < RS_ITEMS; ++i) {
    if (a + i * MB_NT + threadIdx.x >= b) continue;
    const double x = val_of<K>(kv[i]);
    const double e = x - mu;
    if (e * e <= lim) {
      const double d = x - c;
      cs[0] += 1.0;
      cs[1] += d;
      cs[2] = fma(d, d, cs[2]);
    }
  }
  block_sums<3, MB_WV>(cs, red);
  if (threadIdx.x == 0) {
    k0[blockIdx.x] = cs[0];
    k1[blockIdx.x] = cs[1];
    k2[blockIdx.x] = cs[2];
  }
}

__global__ __launch_bounds__(MB_NT) void k_mb_final(const int32_t* __restrict__ seg_tile0,
                                                    int tile_first, const double* __restrict__ prm,
                                                    const double* __restrict__ k0,
                                                    const double* __restrict__ k1,
                                                    const double* __restrict__ k2, double crew,
                                                    SegStat* __restrict__ out) {
  __shared__ double red[3 * MB_WV];
  const int s = blockIdx.x;
  const int t0 = seg_tile0[s] - tile_first, t1 = seg_tile0[s + 1] - tile_first;
  double cs[3] = {0.0, 0.0, 0.0};
  for (int t = t0 + (int)threadIdx.x; t < t1; t += MB_NT) {
    cs[0] += k0[t];
    cs[1] += k1[t];
    cs[2] += k2[t];
  }
  block_sums<3, MB_WV>(cs, red);
  if (threadIdx.x != 0) return;
  const double N = cs[0], S1 = cs[1], S2 = cs[2];
  const double* P = prm + 5 * s;
  SegStat r{};
  r.mu_raw = P[1];
  r.var_raw = P[2];
  r.start = (int64_t)P[4];
  r.n_kept = (int64_t)N;
  r.mu = N > 0 ? P[0] + S1 / N : NAN;
  r.var = N > 1 ? (S2 - S1 * S1 / N) / (N - 1.0) * crew : 0.0;
  out[s] = r;
}

}  // namespace

template <typename K>
hipError_t sort_segments_t(SortPlan& P, hipStream_t s) {
  K* a = static_cast<K*>(P.keys);
  K* b = static_cast<K*>(P.tmp);
  // 64-bit keys (of doubles): the passes order the high 48 bits (sign,
  // exponent and 36 mantissa bits: values that agree there are equal in
  // practice), and the runs of equal high bits that are out of order on the
  // full key are then put in order in place; the full-width sort (eight
  // passes) only with ballot ranking
  const bool hi_only = sizeof(K) == 8 && !P.safe;
  const int ps0 = hi_only ? 2 : 0;
  // the run list of the fix-up lives in the tile counts, free after the
  // last scan: its count (list[0]) is cleared by the last scatter
  // (32 runs per tile of 4096 keys: continuous data hold a few; more fall
  // back to the full-width sort)
  uint64_t* list = reinterpret_cast<uint64_t*>(P.counts);
  const int cap = (int)std::min<int64_t>((int64_t)P.ntiles * 32, INT32_MAX / 2);
  for (int ps = ps0; ps < (int)sizeof(K); ++ps) {
    const int shift = 8 * ps;
    const bool last = ps == (int)sizeof(K) - 1;
    // the top byte of a double's key (sign and the high 7 of 11 exponent
    // bits) takes one or two values in practice: peel it; a float's (high 7
    // of 8 exponent bits) spreads enough for atomics
    const bool top = sizeof(K) == 8 && last;
    if (top)
      hipLaunchKernelGGL((k_rs_count<K, true>), dim3(P.ntiles), dim3(RS_NT), 0, s, a, P.tiles,
                         P.seg_off, P.seg_len, shift, P.counts);
    else
      hipLaunchKernelGGL((k_rs_count<K, false>), dim3(P.ntiles), dim3(RS_NT), 0, s, a, P.tiles,
                         P.seg_off, P.seg_len, shift, P.counts);
    hipLaunchKernelGGL(k_rs_scan, dim3(P.nseg), dim3(SCAN_NT), 0, s, P.counts, P.seg_tile0,
                       P.tile_first, P.offs);
    int32_t* zero = (hi_only && last) ? P.counts : nullptr;
    if (P.safe)
      hipLaunchKernelGGL((k_rs_scatter<K, true, false>), dim3(P.ntiles), dim3(RS_NT), 0, s, a,
                         b, P.tiles, P.seg_off, P.seg_len, shift, P.offs, zero);
    else if (top)
      hipLaunchKernelGGL((k_rs_scatter<K, false, true>), dim3(P.ntiles), dim3(RS_NT), 0, s, a,
                         b, P.tiles, P.seg_off, P.seg_len, shift, P.offs, zero);
    else
      hipLaunchKernelGGL((k_rs_scatter<K, false, false>), dim3(P.ntiles), dim3(RS_NT), 0, s, a,
                         b, P.tiles, P.seg_off, P.seg_len, shift, P.offs, zero);
    K* t = a;
    a = b;
    b = t;
  }
  // an even number of passes leaves the result in P.keys
  if (hi_only) {
    hipLaunchKernelGGL((k_rs_runs<K>), dim3(P.ntiles), dim3(RS_NT), 0, s, a, P.tiles, P.seg_off,
                       P.seg_len, list, cap, P.flag);
    // one thread per listed run: a grid for the capacity, threads beyond
    // the count return at once
    hipLaunchKernelGGL((k_rs_fixup<K>), dim3((cap + 255) / 256), dim3(256), 0, s, a, list, cap);
  }
  // the atomic ranks and the fix-up are checked through the order of the result
  if (!P.safe)
    hipLaunchKernelGGL((k_rs_check<K>), dim3(P.ntiles), dim3(RS_NT), 0, s, a, P.tiles, P.seg_off,
                       P.seg_len, P.flag);
  return hipGetLastError();
}

hipError_t sort_segments(SortPlan& P, hipStream_t s) {
  if (P.ntiles <= 0) return hipSuccess;
  return P.key_bytes == 4 ? sort_segments_t<uint32_t>(P, s) : sort_segments_t<uint64_t>(P, s);
}

hipError_t launch_seg_lds(const SortPlan& P, const double* seg_craw, double q1, double crew,
                          int mode, SegStat* out, int64_t max_len, hipStream_t s) {
  if (P.nseg <= 0) return hipSuccess;
  // k_seg_lds sorts and estimates every segment but those whose values
  // crowd into few normalised keys, which k_seg_lds_slow then takes up
  // (a small grid that skips the rest)
  constexpr int SLOW_GRID = 256;
  // at most SS_NT segments per block of the slow kernel
  const int slow_grid = std::min(P.nseg, std::max(SLOW_GRID, (P.nseg + SS_NT - 1) / SS_NT));
  // keys per thread: the smallest of 4, 6, ..., 16 that holds the longest
  // segment (the passes work on every slot, padding included: 9,765-row
  // blocks take 10,240 slots, not 12,288)
  int kpt = 16;
  for (const int k : {4, 6, 8, 10, 12, 14})
    if (max_len <= (int64_t)k * SS_NT) { kpt = k; break; }
#define SEG_LDS(K, KPT)                                                                        \
  hipLaunchKernelGGL((k_seg_lds<K, KPT>), dim3(P.nseg), dim3(SS_NT), 0, s,                     \
                     static_cast<const K*>(P.keys), P.seg_off, P.seg_len, seg_craw, P.seg_first, \
                     q1, crew, mode, out);                                                     \
  hipLaunchKernelGGL((k_seg_lds_slow<K, KPT>), dim3(slow_grid), dim3(SS_NT),                  \
                     0, s, static_cast<const K*>(P.keys), P.seg_off, P.seg_len, seg_craw,       \
                     P.seg_first, P.nseg, q1, crew, mode, out)
#define BY_KPT(K)                        \
  switch (kpt) {                         \
    case 4: SEG_LDS(K, 4); break;        \
    case 6: SEG_LDS(K, 6); break;        \
    case 8: SEG_LDS(K, 8); break;        \
    case 10: SEG_LDS(K, 10); break;      \
    case 12: SEG_LDS(K, 12); break;      \
    case 14: SEG_LDS(K, 14); break;      \
    default: SEG_LDS(K, 16); break;      \
  }
  if (P.key_bytes == 4) {
    BY_KPT(uint32_t)
  } else {
    BY_KPT(uint64_t)
  }
#undef BY_KPT
#undef SEG_LDS
  return hipGetLastError();
}

int lds_sort_capacity() { return LDS_KEYS; }

int64_t bucket_count(int64_t L) { return L <= BK_CAP ? 1 : (L + BK_EXP - 1) / BK_EXP; }
int bucket_capacity() { return BK_CAP; }
int64_t bucket_max_len() { return (int64_t)BK_NBMAX * BK_EXP; }

template <typename K>
hipError_t sort_buckets_t(SortPlan& P, hipStream_t s) {
  K* keys = static_cast<K*>(P.keys);
  K* stg = static_cast<K*>(P.tmp);
  // class counters [2 nbk], splitters [nbk], marks [nbk] in the tile counts
  int32_t* cnt = P.counts;
  K* split = reinterpret_cast<K*>(P.counts + 2 * (size_t)P.nbk);
  int32_t* mark = P.counts + 2 * (size_t)P.nbk + (size_t)P.nbk * sizeof(K) / 4;
  // (a block's LDS holds the largest sample any of its segments takes)
  if (P.bk_max * 128 > BK_SAMPLE)
    hipLaunchKernelGGL((k_bk_sample<K, BK_SAMPLE_BIG>), dim3(P.nseg), dim3(BK_NT), 0, s, keys,
                       P.seg_off, P.seg_len, P.bk0, P.seg_first, P.bk_first, split, cnt);
  else
    hipLaunchKernelGGL((k_bk_sample<K, BK_SAMPLE>), dim3(P.nseg), dim3(BK_NT), 0, s, keys,
                       P.seg_off, P.seg_len, P.bk0, P.seg_first, P.bk_first, split, cnt);
  hipLaunchKernelGGL((k_bk_scatter<K>), dim3(P.ntiles), dim3(RS_NT), 0, s, keys, stg, P.tiles,
                     P.seg_off, P.seg_len, P.bk0, P.bk_first, split, cnt, P.flag);
  hipLaunchKernelGGL((k_bk_sort<K>), dim3(P.nbk), dim3(SS_NT), 0, s, stg, keys, P.bk_tab,
                     P.seg_off, P.bk0, P.bk_first, split, cnt, mark);
  // at most SS_NT buckets per block of the slow kernel
  const int slow_grid = std::min(P.nbk, std::max(256, (P.nbk + SS_NT - 1) / SS_NT));
  hipLaunchKernelGGL((k_bk_sort_slow<K>), dim3(slow_grid), dim3(SS_NT), 0, s, stg, keys,
                     P.bk_tab, P.seg_off, P.bk0, P.bk_first, P.nbk, cnt, mark);
  return hipGetLastError();
}

hipError_t sort_buckets(SortPlan& P, hipStream_t s) {
  if (P.nseg <= 0 || P.nbk <= 0) return hipSuccess;
  return P.key_bytes == 4 ? sort_buckets_t<uint32_t>(P, s) : sort_buckets_t<uint64_t>(P, s);
}

template <typename K>
hipError_t unimcd_multiblock_t(const SortPlan& P, const double* seg_craw, double q1, double crew,
                               SegStat* out, hipStream_t s) {
  const MbScratch& M = *P.mb;
  const K* keys = static_cast<const K*>(P.keys);
  hipLaunchKernelGGL((k_mb_sums<K>), dim3(P.ntiles), dim3(MB_NT), 0, s, keys, P.tiles, P.seg_off,
                     P.seg_len, M.bs1, M.bs2);
  hipLaunchKernelGGL(k_mb_scan, dim3(P.nseg), dim3(MB_NT), 0, s, P.seg_tile0, P.tile_first, M.bs1,
                     M.bs2, M.tot);
  hipLaunchKernelGGL((k_mb_window<K>), dim3(P.ntiles), dim3(MB_NT), 0, s, keys, P.tiles,
                     P.seg_off, P.seg_len, P.seg_tile0, P.tile_first, P.seg_first, M.bs1, M.bs2,
                     M.tot, M.wbest, M.wj);
  hipLaunchKernelGGL((k_mb_mid<K>), dim3(P.nseg), dim3(MB_NT), 0, s, keys, P.seg_off, P.seg_len,
                     P.seg_tile0, P.tile_first, P.seg_first, M.bs1, M.bs2, M.tot, M.wbest, M.wj,
                     seg_craw, q1, M.prm);
  hipLaunchKernelGGL((k_mb_kept<K>), dim3(P.ntiles), dim3(MB_NT), 0, s, keys, P.tiles, P.seg_off,
                     P.seg_len, P.seg_first, M.prm, M.k0, M.k1, M.k2);
  hipLaunchKernelGGL(k_mb_final, dim3(P.nseg), dim3(MB_NT), 0, s, P.seg_tile0, P.tile_first, M.prm,
                     M.k0, M.k1, M.k2, crew, out);
  return hipGetLastError();
}

hipError_t launch_unimcd_multiblock(const SortPlan& P, const double* seg_craw, double q1,
                                    double crew, SegStat* out, hipStream_t s) {
  if (P.nseg <= 0) return hipSuccess;
  return P.key_bytes == 4 ? unimcd_multiblock_t<uint32_t>(P, seg_craw, q1, crew, out, s)
                          : unimcd_multiblock_t<uint64_t>(P, seg_craw, q1, crew, out, s);
}

hipError_t launch_segstats(const SortPlan& P, const double* seg_craw, double q1, double crew,
                           int mode, SegStat* out, hipStream_t s) {
  if (P.nseg <= 0) return hipSuccess;
  if (P.key_bytes == 4)
    hipLaunchKernelGGL((k_segstats<uint32_t>), dim3(P.nseg), dim3(SS_NT), 0, s,
                       static_cast<const uint32_t*>(P.keys), P.seg_off + P.seg_first, P.seg_len + P.seg_first, seg_craw, q1,
                       crew, mode, out);
  else
    hipLaunchKernelGGL((k_segstats<uint64_t>), dim3(P.nseg), dim3(SS_NT), 0, s,
                       static_cast<const uint64_t*>(P.keys), P.seg_off + P.seg_first, P.seg_len + P.seg_first, seg_craw, q1,
                       crew, mode, out);
  return hipGetLastError();
}

int sort_tile_keys() { return RS_TILE; }

}  // namespace rtd
