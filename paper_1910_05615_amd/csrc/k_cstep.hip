// Per-item kernels of the C-step loop: exact h-subset selection, and the
// float64 statistics / Cholesky / condition-monitor step.
#include "common.h"
#include "wave.h"

namespace rtd {

namespace {

// d2 >= 0, so the IEEE bit pattern orders like the value.  NaN sorts last.
__device__ inline uint64_t key_of(double v) {
  if (!(v == v)) return ~0ull;
  if (v <= 0.0) return 0ull;     // also maps -0.0 to +0.0
  return (uint64_t)__double_as_longlong(v);
}

// Block-wide exclusive scan of one int per thread (blockDim = NT, NT/64 waves).
template <int NT>
__device__ inline int block_excl_scan(int v, int* wtot, int& total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int x = v;
  // inclusive wave scan
  x = wave_incl_sum(x);
  if (lane == 63) wtot[wv] = x;
  __syncthreads();
  int off = 0;
  total = 0;
#pragma unroll
  for (int k = 0; k < NT / 64; ++k) {
    const int t = wtot[k];
    if (k < wv) off += t;
    total += t;
  }
  __syncthreads();
  return off + x - v;
}

// ---------------------------------------------------------------------------
// h-subset selection (Sec. 2.1 C-step steps 2-3): the h-th smallest key (the
// float64 bit pattern of d2) from one histogram over the item's key range
// and an exact ranking of the keys in the bin that holds rank h (radix select
// when that bin is crowded), then one pass in row order that resolves ties
// by index and records the swapped rows for the update-based step (Sec. 3.5).
// ---------------------------------------------------------------------------
constexpr int SEL_NT = 1024;


// Same selection for items of at most SEL_NT * SEL_KR rows, with the keys
// held in registers (row i * SEL_NT + tid in slot i): the digit passes do not
// re-read d2, and the row-order pass ranks rows with wave ballots and one
// scan over the (slot, wave) counts instead of block scans per 1024 rows.
// Row order is slot-major, then wave, then lane, i.e. plain index order.
constexpr int SEL_KR = 16;
constexpr int SEL_WV = SEL_NT / 64;
constexpr int SEL_NBB = 13;               // bins of the one-pass histogram: 2^13
constexpr int SEL_NB = 1 << SEL_NBB;
constexpr int SEL_CMAX = 512;             // keys ranked exactly in the threshold bin

// unsigned 64-bit minimum / maximum over the wave, in every lane
__device__ inline uint64_t wave_min_u64(uint64_t x) {
#define RTD_MIN_STEP(C, R) { const uint64_t y = (uint64_t)dpp_l<C, R>((int64_t)x, -1); x = y < x ? y : x; }
  RTD_MIN_STEP(0x111, 0xf) RTD_MIN_STEP(0x112, 0xf) RTD_MIN_STEP(0x114, 0xf)
  RTD_MIN_STEP(0x118, 0xf) RTD_MIN_STEP(0x142, 0xa) RTD_MIN_STEP(0x143, 0xc)
#undef RTD_MIN_STEP
  return (uint64_t)lane_bcast_l((int64_t)x, 63);
}
__device__ inline uint64_t wave_max_u64(uint64_t x) {
#define RTD_MAX_STEP(C, R) { const uint64_t y = (uint64_t)dpp_l<C, R>((int64_t)x, 0); x = y > x ? y : x; }
  RTD_MAX_STEP(0x111, 0xf) RTD_MAX_STEP(0x112, 0xf) RTD_MAX_STEP(0x114, 0xf)
  RTD_MAX_STEP(0x118, 0xf) RTD_MAX_STEP(0x142, 0xa) RTD_MAX_STEP(0x143, 0xc)
#undef RTD_MAX_STEP
  return (uint64_t)lane_bcast_l((int64_t)x, 63);
}

// Exclusive scan, in place, of n <= 256 ints laid out in order, by the first
// four waves; returns the total to every thread.  wsum: 4 ints.
__device__ inline int scan256_excl(int* __restrict__ v, int n, int* __restrict__ wsum) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int x = 0, own = 0;
  if (tid < 256) {
    own = tid < n ? v[tid] : 0;
    x = own;
    x = wave_incl_sum(x);
    if (lane == 63) wsum[w] = x;
  }
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int t = wsum[k];
    if (k < w) off += t;
    tot += t;
  }
  if (tid < n) v[tid] = off + x - own;
  __syncthreads();
  return tot;
}

// Two such scans at once: waves 0-3 scan v1, waves 4-7 scan v2; returns
// both totals.  wsum: 8 ints.
__device__ inline int2 scan256_excl2(int* __restrict__ v1, int* __restrict__ v2, int n,
                                     int* __restrict__ wsum) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int* __restrict__ v = tid < 256 ? v1 : v2;
  const int t = tid & 255;
  int x = 0, own = 0;
  if (tid < 512) {
    own = t < n ? v[t] : 0;
    x = wave_incl_sum(own);
    if (lane == 63) wsum[w] = x;
  }
  __syncthreads();
  const int wb = w & 4;
  int off = 0, tot1 = 0, tot2 = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    tot1 += wsum[k];
    tot2 += wsum[4 + k];
    if (wb + k < w) off += wsum[wb + k];
  }
  if (tid < 512 && t < n) v[t] = off + x - own;
  __syncthreads();
  return make_int2(tot1, tot2);
}

__global__ __launch_bounds__(SEL_NT) void k_select_reg(const ItemDesc* __restrict__ items,
                                                       ItemArrays A, int first_item,
                                                       int cstep_mode, int reset_nactive) {
  if (reset_nactive && blockIdx.x == 0 && threadIdx.x == 0) *A.nactive = 0;
  __shared__ __align__(16) unsigned hist[8192];
  __shared__ int wtot[SEL_WV];
  __shared__ int tab[3][SEL_KR * SEL_WV];   // eq, entering, leaving per (slot, wave)
  __shared__ int wsum[8];
  __shared__ int s_bin, s_cnt, s_nc, s_all;
  __shared__ long long s_below, s_rank;
  __shared__ uint64_t s_prefix;
  __shared__ uint64_t s_bound[2 * SEL_WV];
  const int it = first_item + blockIdx.x;
  if (A.status[it] != ACTIVE) return;
  const ItemDesc D = items[it];
  const int m = (int)D.m;
  const int64_t h = D.h;
  const double* __restrict__ d2 = A.d2 + D.roff;
  uint8_t* __restrict__ mask = A.mask + D.roff;
  int32_t* __restrict__ swp = A.swap + D.roff;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint64_t below = (1ull << lane) - 1ull;

  uint64_t key[SEL_KR];
  uint32_t oldb = 0;   // the previous subset's membership of this thread's rows
#pragma unroll
  for (int i = 0; i < SEL_KR; ++i) {
    const int r = i * SEL_NT + tid;
    key[i] = r < m ? key_of(d2[r]) : 0ull;
    if (r < m && mask[r] != 0) oldb |= 1u << i;
  }
  const int it0 = A.iter[it];
  uint64_t prefix = 0, pmask = ~0ull;
  int64_t rank = h;
  bool take_all = false;
  // One histogram of the keys over 8192 bins of the segment's key range
  // (bin = (key - kmin) >> sh: monotone, and logarithmic in the value, so
  // far outliers do not crowd the bulk into a few bins), then the keys of the
  // bin that holds rank h, ranked among themselves exactly.
  {
    uint64_t kmn = ~0ull, kmx = 0ull;
#pragma unroll
    for (int i = 0; i < SEL_KR; ++i) {
      if (i * SEL_NT + tid < m) {
        kmn = key[i] < kmn ? key[i] : kmn;
        if (key[i] != ~0ull && key[i] > kmx) kmx = key[i];   // NaN keys: the last bin
      }
    }
    kmn = wave_min_u64(kmn);
    kmx = wave_max_u64(kmx);
    if (lane == 0) {
      s_bound[w] = kmn;
      s_bound[SEL_WV + w] = kmx;
    }
    for (int b = tid; b < SEL_NB; b += SEL_NT) hist[b] = 0u;
    if (tid == 0) s_nc = 0;
    __syncthreads();
    kmn = ~0ull;
    kmx = 0ull;
#pragma unroll
    for (int q = 0; q < SEL_WV; ++q) {
      kmn = s_bound[q] < kmn ? s_bound[q] : kmn;
      kmx = s_bound[SEL_WV + q] > kmx ? s_bound[SEL_WV + q] : kmx;
    }
    const uint64_t span = kmx > kmn ? kmx - kmn : 0ull;
    const int bl = span ? 64 - __clzll((long long)span) : 0;
    const int sh = bl > SEL_NBB ? bl - SEL_NBB : 0;
    auto bin_of = [&](uint64_t k) -> int {
      if (k == ~0ull) return SEL_NB - 1;
      const uint64_t b = (k - kmn) >> sh;
      return b < (uint64_t)SEL_NB ? (int)b : SEL_NB - 1;
    };
#pragma unroll
    for (int i = 0; i < SEL_KR; ++i)
      if (i * SEL_NT + tid < m) atomicAdd(&hist[bin_of(key[i])], 1u);
    __syncthreads();
    constexpr int per = SEL_NB / SEL_NT;
    int loc = 0;
#pragma unroll
    for (int b = 0; b < per; ++b) loc += (int)hist[tid * per + b];
    int tot;
    const int before = block_excl_scan<SEL_NT>(loc, wtot, tot);
    if ((int64_t)before < rank && rank <= (int64_t)(before + loc)) {
      int64_t run = before;
      for (int b = 0; b < per; ++b) {
        const int c = (int)hist[tid * per + b];
        if (rank <= run + c) { s_bin = tid * per + b; s_cnt = c; s_below = run; break; }
        run += c;
      }
    }
    __syncthreads();
    const int bstar = s_bin, cnt = s_cnt;
    const int64_t k1 = rank - s_below;   // 1-based rank within the bin
    if (cnt <= SEL_CMAX) {   // uniform
      uint64_t* ck = reinterpret_cast<uint64_t*>(hist);   // the counts are read
#pragma unroll
      for (int i = 0; i < SEL_KR; ++i)
        if (i * SEL_NT + tid < m && bin_of(key[i]) == bstar) ck[atomicAdd(&s_nc, 1)] = key[i];
      __syncthreads();
      if (tid < cnt) {
        const uint64_t x = ck[tid];
        int nless = 0, nleq = 0;
        for (int j = 0; j < cnt; ++j) {
          const uint64_t y = ck[j];
          nless += y < x ? 1 : 0;
          nleq += y <= x ? 1 : 0;
        }
        if (nless < k1 && k1 <= nleq) {   // x is the h-th smallest key (equal keys agree)
          s_prefix = x;
          s_rank = k1 - nless;
          s_all = k1 == nleq ? 1 : 0;
        }
      }
      __syncthreads();
      prefix = s_prefix;
      rank = s_rank;
      take_all = s_all != 0;
    } else {
      // a bin crowded with equal or nearly equal keys: radix select on the
      // float64 bit patterns, digits 12/13/13/13/13 bits from the top
      __syncthreads();   // every thread has read s_bin / s_cnt
      pmask = 0;
      const int shifts[5] = {52, 39, 26, 13, 0};
      const int bitsv[5] = {12, 13, 13, 13, 13};
#pragma unroll
      for (int ps = 0; ps < 5; ++ps) {
        const int shift = shifts[ps], bits = bitsv[ps];
        const int nbins = 1 << bits;
        for (int b = tid; b < nbins; b += SEL_NT) hist[b] = 0u;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < SEL_KR; ++i) {
          const int r = i * SEL_NT + tid;
          if (r < m && (key[i] & pmask) == prefix)
            atomicAdd(&hist[(key[i] >> shift) & (uint64_t)(nbins - 1)], 1u);
        }
        __syncthreads();
        const int per = nbins / SEL_NT;
        int loc = 0;
        for (int b = 0; b < per; ++b) loc += (int)hist[tid * per + b];
        int tot;
        const int before = block_excl_scan<SEL_NT>(loc, wtot, tot);
        if ((int64_t)before < rank && rank <= (int64_t)(before + loc)) {
          int64_t run = before;
          for (int b = 0; b < per; ++b) {
            const int c = (int)hist[tid * per + b];
            if (rank <= run + c) { s_bin = tid * per + b; s_cnt = c; s_below = run; break; }
            run += c;
          }
        }
        __syncthreads();
        prefix |= (uint64_t)s_bin << shift;
        pmask |= (uint64_t)(nbins - 1) << shift;
        rank -= s_below;
        const int cnt = s_cnt;
        __syncthreads();
        if ((int64_t)cnt == rank) { take_all = true; break; }
      }
    }
  }

  // membership; ties at the threshold key go to the lowest row indices
  uint32_t selb = 0;
#pragma unroll
  for (int i = 0; i < SEL_KR; ++i) {
    const int r = i * SEL_NT + tid;
    const bool valid = r < m;
    const bool sel = take_all ? (valid && (key[i] & pmask) <= prefix) : (valid && key[i] < prefix);
    if (sel) selb |= 1u << i;
  }
  if (!take_all) {   // uniform over the block
    uint32_t eqb = 0;
#pragma unroll
    for (int i = 0; i < SEL_KR; ++i) {
      const bool eq = (i * SEL_NT + tid) < m && key[i] == prefix;
      const uint64_t b = __ballot(eq);
      if (eq) eqb |= 1u << i;
      if (lane == 0) tab[0][i * SEL_WV + w] = __popcll(b);
    }
    __syncthreads();
    scan256_excl(tab[0], SEL_KR * SEL_WV, wsum);
#pragma unroll
    for (int i = 0; i < SEL_KR; ++i) {
      const bool eq = (eqb >> i) & 1u;
      const uint64_t b = __ballot(eq);
      const int64_t er = tab[0][i * SEL_WV + w] + __popcll(b & below);
      if (eq && er < rank) selb |= 1u << i;
    }
  }
  const bool first = (it0 == 0);
  uint32_t entb = 0, lftb = 0;
#pragma unroll
  for (int i = 0; i < SEL_KR; ++i) {
    const int r = i * SEL_NT + tid;
    const bool valid = r < m;
    const bool sel = (selb >> i) & 1u;
    const bool old = (oldb >> i) & 1u;
    const bool ent = sel && !old, lft = valid && !sel && old;
    if (ent) entb |= 1u << i;
    if (lft) lftb |= 1u << i;
    const uint64_t be = __ballot(ent), bl = __ballot(lft);
    if (lane == 0) {
      tab[1][i * SEL_WV + w] = __popcll(be);
      tab[2][i * SEL_WV + w] = __popcll(bl);
    }
    if (valid) mask[r] = sel ? 1 : 0;
  }
  __syncthreads();
  const int2 nio = scan256_excl2(tab[1], tab[2], SEL_KR * SEL_WV, wsum);
  const int nin = nio.x;
  if (!first) {
    const int half = m / 2;
#pragma unroll
    for (int i = 0; i < SEL_KR; ++i) {
      const int r = i * SEL_NT + tid;
      const bool ent = (entb >> i) & 1u, lft = (lftb >> i) & 1u;
      const uint64_t be = __ballot(ent), bl = __ballot(lft);
      if (ent) swp[tab[1][i * SEL_WV + w] + __popcll(be & below)] = r;
      if (lft) swp[half + tab[2][i * SEL_WV + w] + __popcll(bl & below)] = r;
    }
  }
  if (tid == 0) {
    A.iter[it] = it0 + 1;
    A.kswap[it] = first ? 0 : nin;
    int full;
    if (first || cstep_mode == 0) full = 1;
    else if (cstep_mode == 1) full = 0;
    else full = (8 * (int64_t)nin > h) ? 1 : 0;
    A.full[it] = full;
    if (!first && nin == 0) A.status[it] = ST_CONVERGED;
  }
}

// h-subset selection of an item longer than SEL_NT * SEL_KR rows: the
// threshold search and the membership of k_select_reg over chunks of
// SEL_NT * SEL_KR rows (the keys read again for each of: bounds, histogram,
// the threshold bin's keys, membership), swap lists in row order across the
// chunks.
__global__ __launch_bounds__(SEL_NT) void k_select(const ItemDesc* __restrict__ items,
                                                   ItemArrays A, int first_item,
                                                   int cstep_mode, int reset_nactive) {
  if (reset_nactive && blockIdx.x == 0 && threadIdx.x == 0) *A.nactive = 0;
  __shared__ __align__(16) unsigned hist[8192];
  __shared__ int wtot[SEL_WV];
  __shared__ int tab[3][SEL_KR * SEL_WV];
  __shared__ int wsum[8];
  __shared__ int s_bin, s_cnt, s_nc, s_all;
  __shared__ long long s_below, s_rank;
  __shared__ uint64_t s_prefix;
  __shared__ uint64_t s_bound[2 * SEL_WV];
  const int it = first_item + blockIdx.x;
  if (A.status[it] != ACTIVE) return;
  const ItemDesc D = items[it];
  const int64_t m = D.m, h = D.h;
  const double* __restrict__ d2 = A.d2 + D.roff;
  uint8_t* __restrict__ mask = A.mask + D.roff;
  int32_t* __restrict__ swp = A.swap + D.roff;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint64_t below = (1ull << lane) - 1ull;
  constexpr int CH = SEL_NT * SEL_KR;
  // the bounds and histogram passes walk the chunks with the next chunk's
  // loads in flight while the current one is worked on: prime(), then
  // next(c0) at the top of the chunk at c0; the candidate and membership
  // passes (more live state: prefetching there spills) load each chunk when
  // they reach it, load(c0).  Keys of rows beyond m are 0.
  uint64_t key[SEL_KR];
  double nraw[SEL_KR];
  auto fetch = [&](int64_t c0) {
#pragma unroll
    for (int i = 0; i < SEL_KR; ++i) {
      const int64_t r = c0 + i * SEL_NT + tid;
      nraw[i] = r < m ? d2[r] : 0.0;
    }
  };
  auto prime = [&]() { fetch(0); };
  auto next = [&](int64_t c0) {
#pragma unroll
    for (int i = 0; i < SEL_KR; ++i)
      key[i] = c0 + i * SEL_NT + tid < m ? key_of(nraw[i]) : 0ull;
    if (c0 + CH < m) fetch(c0 + CH);
  };
  auto load = [&](int64_t c0) {
#pragma unroll
    for (int i = 0; i < SEL_KR; ++i) {
      const int64_t r = c0 + i * SEL_NT + tid;
      key[i] = r < m ? key_of(d2[r]) : 0ull;
    }
  };
  const int it0 = A.iter[it];
  uint64_t prefix = 0, pmask = ~0ull;
  int64_t rank = h;
  bool take_all = false;
  {
    uint64_t kmn = ~0ull, kmx = 0ull;
    prime();
    for (int64_t c0 = 0; c0 < m; c0 += CH) {
      next(c0);
#pragma unroll
      for (int i = 0; i < SEL_KR; ++i)
        if (c0 + i * SEL_NT + tid < m) {
          kmn = key[i] < kmn ? key[i] : kmn;
          if (key[i] != ~0ull && key[i] > kmx) kmx = key[i];
        }
    }
    kmn = wave_min_u64(kmn);
    kmx = wave_max_u64(kmx);
    if (lane == 0) {
      s_bound[w] = kmn;
      s_bound[SEL_WV + w] = kmx;
    }
    for (int b = tid; b < SEL_NB; b += SEL_NT) hist[b] = 0u;
    if (tid == 0) s_nc = 0;
    __syncthreads();
    kmn = ~0ull;
    kmx = 0ull;
#pragma unroll
    for (int q = 0; q < SEL_WV; ++q) {
      kmn = s_bound[q] < kmn ? s_bound[q] : kmn;
      kmx = s_bound[SEL_WV + q] > kmx ? s_bound[SEL_WV + q] : kmx;
    }
    const uint64_t span = kmx > kmn ? kmx - kmn : 0ull;
    const int bl = span ? 64 - __clzll((long long)span) : 0;
    const int sh = bl > SEL_NBB ? bl - SEL_NBB : 0;
    auto bin_of = [&](uint64_t k) -> int {
      if (k == ~0ull) return SEL_NB - 1;
      const uint64_t b = (k - kmn) >> sh;
      return b < (uint64_t)SEL_NB ? (int)b : SEL_NB - 1;
    };
    prime();
    for (int64_t c0 = 0; c0 < m; c0 += CH) {
      next(c0);
#pragma unroll
      for (int i = 0; i < SEL_KR; ++i)
        if (c0 + i * SEL_NT + tid < m) atomicAdd(&hist[bin_of(key[i])], 1u);
    }
    __syncthreads();
    constexpr int per = SEL_NB / SEL_NT;
    int loc = 0;
#pragma unroll
    for (int b = 0; b < per; ++b) loc += (int)hist[tid * per + b];
    int tot;
    const int before = block_excl_scan<SEL_NT>(loc, wtot, tot);
    if ((int64_t)before < rank && rank <= (int64_t)(before + loc)) {
      int64_t run = before;
      for (int b = 0; b < per; ++b) {
        const int c = (int)hist[tid * per + b];
        if (rank <= run + c) { s_bin = tid * per + b; s_cnt = c; s_below = run; break; }
        run += c;
      }
    }
    __syncthreads();
    const int bstar = s_bin, cnt = s_cnt;
    const int64_t k1 = rank - s_below;
    if (cnt <= SEL_CMAX) {   // uniform
      uint64_t* ck = reinterpret_cast<uint64_t*>(hist);
      for (int64_t c0 = 0; c0 < m; c0 += CH) {
        load(c0);
#pragma unroll
        for (int i = 0; i < SEL_KR; ++i)
          if (c0 + i * SEL_NT + tid < m && bin_of(key[i]) == bstar)
            ck[atomicAdd(&s_nc, 1)] = key[i];
      }
      __syncthreads();
      if (tid < cnt) {
        const uint64_t x = ck[tid];
        int nless = 0, nleq = 0;
        for (int j = 0; j < cnt; ++j) {
          const uint64_t y = ck[j];
          nless += y < x ? 1 : 0;
          nleq += y <= x ? 1 : 0;
        }
        if (nless < k1 && k1 <= nleq) {
          s_prefix = x;
          s_rank = k1 - nless;
          s_all = k1 == nleq ? 1 : 0;
        }
      }
      __syncthreads();
      prefix = s_prefix;
      rank = s_rank;
      take_all = s_all != 0;
    } else {
      // a crowded bin: radix select on the float64 bit patterns, digits
      // 12/13/13/13/13 bits from the top
      __syncthreads();
      pmask = 0;
      const int shifts[5] = {52, 39, 26, 13, 0};
      const int bitsv[5] = {12, 13, 13, 13, 13};
      for (int ps = 0; ps < 5; ++ps) {
        const int shift = shifts[ps], bits = bitsv[ps];
        const int nbins = 1 << bits;
        for (int b = tid; b < nbins; b += SEL_NT) hist[b] = 0u;
        __syncthreads();
        for (int64_t i = tid; i < m; i += SEL_NT) {
          const uint64_t k = key_of(d2[i]);
          if ((k & pmask) == prefix) atomicAdd(&hist[(k >> shift) & (uint64_t)(nbins - 1)], 1u);
        }
        __syncthreads();
        const int pb = nbins / SEL_NT;
        int lc = 0;
        for (int b = 0; b < pb; ++b) lc += (int)hist[tid * pb + b];
        int tt;
        const int bf = block_excl_scan<SEL_NT>(lc, wtot, tt);
        if ((int64_t)bf < rank && rank <= (int64_t)(bf + lc)) {
          int64_t run = bf;
          for (int b = 0; b < pb; ++b) {
            const int c = (int)hist[tid * pb + b];
            if (rank <= run + c) { s_bin = tid * pb + b; s_cnt = c; s_below = run; break; }
            run += c;
          }
        }
        __syncthreads();
        prefix |= (uint64_t)s_bin << shift;
        pmask |= (uint64_t)(nbins - 1) << shift;
        rank -= s_below;
        const int c2 = s_cnt;
        __syncthreads();
        if ((int64_t)c2 == rank) { take_all = true; break; }
      }
    }
  }
  // membership chunk by chunk; ties at the threshold key go to the lowest
  // row indices; swap lists in row order
  const bool first = (it0 == 0);
  const int64_t half = m / 2;
  int64_t tie_seen = 0, nin = 0;
  int64_t nout = 0;
  for (int64_t c0 = 0; c0 < m; c0 += CH) {
    load(c0);
    uint32_t selb = 0, oldb = 0;
#pragma unroll
    for (int i = 0; i < SEL_KR; ++i) {
      const int64_t r = c0 + i * SEL_NT + tid;
      const bool valid = r < m;
      if (valid && mask[r] != 0) oldb |= 1u << i;
      const bool sel = take_all ? (valid && (key[i] & pmask) <= prefix) : (valid && key[i] < prefix);
      if (sel) selb |= 1u << i;
    }
    if (!take_all) {   // uniform
      uint32_t eqb = 0;
#pragma unroll
      for (int i = 0; i < SEL_KR; ++i) {
        const bool eq = (c0 + i * SEL_NT + tid) < m && key[i] == prefix;
        const uint64_t b = __ballot(eq);
        if (eq) eqb |= 1u << i;
        if (lane == 0) tab[0][i * SEL_WV + w] = __popcll(b);
      }
      __syncthreads();
      const int neq = scan256_excl(tab[0], SEL_KR * SEL_WV, wsum);
#pragma unroll
      for (int i = 0; i < SEL_KR; ++i) {
        const bool eq = (eqb >> i) & 1u;
        const uint64_t b = __ballot(eq);
        const int64_t er = tie_seen + tab[0][i * SEL_WV + w] + __popcll(b & below);
        if (eq && er < rank) selb |= 1u << i;
      }
      tie_seen += neq;
    }
    uint32_t entb = 0, lftb = 0;
#pragma unroll
    for (int i = 0; i < SEL_KR; ++i) {
      const int64_t r = c0 + i * SEL_NT + tid;
      const bool valid = r < m;
      const bool sel = (selb >> i) & 1u;
      const bool old = (oldb >> i) & 1u;
      const bool ent = sel && !old, lft = valid && !sel && old;
      if (ent) entb |= 1u << i;
      if (lft) lftb |= 1u << i;
      const uint64_t be = __ballot(ent), bl = __ballot(lft);
      if (lane == 0) {
        tab[1][i * SEL_WV + w] = __popcll(be);
        tab[2][i * SEL_WV + w] = __popcll(bl);
      }
      if (valid) mask[r] = sel ? 1 : 0;
    }
    __syncthreads();
    const int2 nio = scan256_excl2(tab[1], tab[2], SEL_KR * SEL_WV, wsum);
    if (!first) {
#pragma unroll
      for (int i = 0; i < SEL_KR; ++i) {
        const int64_t r = c0 + i * SEL_NT + tid;
        const bool ent = (entb >> i) & 1u, lft = (lftb >> i) & 1u;
        const uint64_t be = __ballot(ent), bl = __ballot(lft);
        if (ent) swp[nin + tab[1][i * SEL_WV + w] + __popcll(be & below)] = (int32_t)r;
        if (lft) swp[half + nout + tab[2][i * SEL_WV + w] + __popcll(bl & below)] = (int32_t)r;
      }
    }
    nin += nio.x;
    nout += nio.y;
    __syncthreads();   // tab is read by every thread before the next chunk writes it
  }
  if (tid == 0) {
    A.iter[it] = it0 + 1;
    A.kswap[it] = first ? 0 : (int32_t)nin;
    int full;
    if (first || cstep_mode == 0) full = 1;
    else if (cstep_mode == 1) full = 0;
    else full = (8 * nin > h) ? 1 : 0;
    A.full[it] = full;
    if (!first && nin == 0) A.status[it] = ST_CONVERGED;
  }
}

// ---------------------------------------------------------------------------
// Statistics and Cholesky step of one item (Sec. 2.1 eq. cstep4a/cstep4b,
// Sec. 3.4, Sec. 3.5), all in float64:
//   * from the sscp tile partials, mean and sscp about the new mean, either
//     recomputed (full) or updated from the swapped rows:
//       mu_new = c + s/h,  Lambda_new = Lambda_old + S - s s^T / h
//     with c = mu_old the pivot of the partial sums (Lambda_old = 0 when full);
//   * Sigma = D^{-1} Lambda D^{-1} / (h-1) in standardised units, its Cholesky
//     factor, log det, inverse factor and exact 1-norm condition number;
//   * M = L^{-1} D^{-1} packed for the distance kernel.
// from_start: (muz, sigz) already hold the start; nothing is reduced.
//
// One wave per item, P >= p a compile-time bound: lane i holds row i of
// Sigma, then of L, in registers (rows and columns p..P-1 are the identity,
// so the factor and its inverse carry an identity block that is never
// written); the inverse is formed one column per lane.  Every loop is
// unrolled over P.  Each finished row of L, and each column of the inverse,
// is published to LDS and read back by all lanes with broadcast loads
// (single values of other lanes with readlane); the dot products of the
// Cholesky and of the forward substitution run as two interleaved partial
// sums, and the divisions are multiplications by the reciprocal diagonal.
// ---------------------------------------------------------------------------
__device__ inline double lane_bcast(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Single-swap step of an item (Sec. 3.5): the leaving row, then the entering
// row, update the mean and the sscp matrix case by case (eq. propcstep1,
// muUpdate, propcstep2), and the inverse of the sscp matrix by the
// Sherman-Morrison-Woodbury identity (eq. woodbury), with the determinant
// ratio Delta_i of eq. (scaleddetUpdate).  Lane i holds row i of the sscp
// matrix (lr) and of its inverse (li), in data units.  Returns false when a
// Delta_i is not positive (the new sscp matrix would be singular).
template <int P>
__device__ inline bool smw_swaps(const ItemDesc& D, const int32_t* __restrict__ swp, double h,
                                 double& mu, double (&lr)[P], double (&li)[P], double& ldsum) {
  const int lane = threadIdx.x;
  const bool in = lane < D.p;
  const int64_t rows[2] = {swp[D.m / 2], swp[0]};   // leaving, entering
  const double dl[2] = {-1.0, 1.0};
  double hc = h;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int64_t r = D.row0 + rows[c];
    double x = 0.0;
    if (in) {
      x = D.dtype == 0 ? (double)static_cast<const float*>(D.X)[r * D.ld + lane]
                       : static_cast<const double*>(D.X)[r * D.ld + lane];
    }
    const double dlt = dl[c];
    hc += dlt;
    const double u = in ? x - mu : 0.0;
    mu = mu + (dlt / hc) * u;
    const double v = in ? x - mu : 0.0;
    double av = 0.0, bv = 0.0;   // (Lam^{-1} u)_i, (Lam^{-1} v)_i
#pragma unroll
    for (int j = 0; j < P; ++j) {
      av = fma(li[j], lane_bcast(u, j), av);
      bv = fma(li[j], lane_bcast(v, j), bv);
    }
    const double dot = wave_sum(in ? v * av : 0.0);
    const double Delta = 1.0 + dlt * dot;
    if (!(Delta > 0.0)) return false;
    const double f = dlt / Delta;
#pragma unroll
    for (int j = 0; j < P; ++j) {
      li[j] = fma(-f * av, lane_bcast(bv, j), li[j]);
      lr[j] = fma(dlt * u, lane_bcast(v, j), lr[j]);
    }
    ldsum += log(Delta);
  }
  return true;
}

template <int P>
__global__ __launch_bounds__(64) void k_finalize(const ItemDesc* __restrict__ items,
                                                 ItemArrays A, int first_item, int from_start,
                                                 int max_csteps, double kappa_max,
                                                 int cstep_mode, int dist_form) {
  const int it = first_item + blockIdx.x;
  if (A.status[it] != ACTIVE) return;
  const ItemDesc D = items[it];
  const int p = D.p;                       // p <= P
  const int lane = threadIdx.x;            // row i (Sigma, L), column j (L^{-1})
  const bool in = lane < p;
  const double h = (double)D.h;
  double* __restrict__ mux = A.mux + (size_t)it * PMAX;
  double* __restrict__ lam = A.lamx + (size_t)it * MSTRIDE;
  double* __restrict__ muz = A.muz + (size_t)it * PMAX;
  double* __restrict__ sigz = A.sigz + (size_t)it * MSTRIDE;
  double* __restrict__ sinv = A.sinv + (size_t)it * MSTRIDE;
  double* __restrict__ mt = A.mtri + (size_t)it * MSTRIDE;
  const double sc = in ? D.scale[lane] : 1.0;
  const bool smw_mode = cstep_mode == 3;   // RTDETMCD_CSTEP_SMW
  // a step whose subset changed by one row out and one in, in the single-swap
  // mode: the inverse and the determinant are carried, no Cholesky
  if (!from_start && smw_mode && !A.full[it] && A.kswap[it] == 1) {
    double lr[P], li[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const bool ok = in && j < p;
      lr[j] = ok ? lam[lane * PMAX + j] : 0.0;
      li[j] = ok ? sinv[lane * PMAX + j] : 0.0;
    }
    double mu = in ? mux[lane] : 0.0;
    double ldsum = 0.0;
    if (!smw_swaps<P>(D, A.swap + D.roff, h, mu, lr, li, ldsum)) {
      if (lane == 0) A.status[it] = ST_SINGULAR;
      return;
    }
    // Sigma_z = D^{-1} Lam D^{-1} / (h-1), Sigma_z^{-1} = (h-1) D Lam^{-1} D;
    // the distance factor is the packed inverse in data units
    double n1 = 0.0, n2 = 0.0;
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const double scj = lane_bcast(sc, j);
      if (in && j < p) {
        lam[lane * PMAX + j] = lr[j];
        sinv[lane * PMAX + j] = li[j];
        const double sz = lr[j] / (sc * scj) / (h - 1.0);
        sigz[lane * PMAX + j] = sz;
        n1 += fabs(sz);
        n2 += fabs((h - 1.0) * li[j] * (sc * scj));
        if (j <= lane) mt[lane * PMAX + j] = (j < lane ? 2.0 : 1.0) * (h - 1.0) * li[j];
      }
    }
    if (in) {
      mux[lane] = mu;
      muz[lane] = (mu - D.loc[lane]) / sc;
    }
    n1 = wave_max(n1);
    n2 = wave_max(n2);
    if (lane == 0) {
      A.form[it] = 1;
      A.logdet[it] += ldsum;
      const double kap = n1 * n2;
      int st = ACTIVE;
      if (A.iter[it] >= max_csteps) st = ST_NOTCONV;
      else if (!(kap < kappa_max)) st = ST_ILLCOND;
      A.status[it] = st;
      if (st == ACTIVE && A.nactive) atomicAdd(A.nactive, 1);
      if (st == ACTIVE && A.ldtr && A.iter[it] < A.ldtr_n)   // the step will be evaluated
        A.ldtr[(size_t)it * A.ldtr_n + A.iter[it]] = A.logdet[it];
    }
    return;
  }
  // rows of L, then rows of X^T = (L^{-1})^T (lane j's column of L^{-1}),
  // read by every lane with broadcast loads; 1 / L_kk
  constexpr int LD = (P + 1) & ~1;   // even: 16-byte aligned rows
  __shared__ __align__(16) double Ls[P * LD];
  __shared__ __align__(16) double XT[P * LD];
  __shared__ double rdg[P];
  const double isc = 1.0 / sc;
  const double ih1 = 1.0 / (h - 1.0);
  double a[P];
  if (!from_start) {
    const int full = A.full[it];
    // tile partials already collapsed into the first tile's
    const double* __restrict__ P0 = A.part + (size_t)D.tile0 * PSTRIDE;
    const double dm = in ? P0[1 + lane] / h : 0.0;   // mu_new - c (pivot-centred sum / h)
    // every load first (a loop without stores, so they all go out at once),
    // then the update and the stores
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const int hi = lane >= j ? lane : j, lo = lane >= j ? j : lane;
      const bool ok = in && j < p;
      const double old = (ok && !full) ? lam[lane * PMAX + j] : 0.0;
      a[j] = ok ? old + P0[1 + PMAX + hi * (hi + 1) / 2 + lo] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const double dmj = lane_bcast(dm, j), iscj = lane_bcast(isc, j);
      if (in && j < p) {
        const double v = a[j] - h * (dm * dmj);
        lam[lane * PMAX + j] = v;
        a[j] = v * (isc * iscj) * ih1;
      } else {
        a[j] = j == lane ? 1.0 : 0.0;
      }
    }
    if (in) {
      const double mnew = mux[lane] + dm;
      mux[lane] = mnew;
      muz[lane] = (mnew - D.loc[lane]) * isc;
    }
  } else {
#pragma unroll
    for (int j = 0; j < P; ++j)
      a[j] = (in && j < p) ? 0.5 * (sigz[lane * PMAX + j] + sigz[j * PMAX + lane])
                           : (j == lane ? 1.0 : 0.0);
    if (in) mux[lane] = D.loc[lane] + sc * muz[lane];
    __syncthreads();   // every lane has read sigz before any lane writes it
  }
  double n1 = 0.0;     // 1-norm of Sigma: largest absolute row sum (symmetric)
  if (in) {
#pragma unroll
    for (int j = 0; j < P; ++j)
      if (j < p) {
        sigz[lane * PMAX + j] = a[j];
        n1 += fabs(a[j]);
      }
  }
  n1 = wave_max(n1);
  // Cholesky, column by column: L_ik = (S_ik - sum_{j<k} L_ij L_kj) / L_kk,
  // lane i holding row i; row k of L comes from LDS (its entries j < k were
  // stored at the steps j); two partial sums shorten the chain
  double diag = 1.0, rdiag = 1.0;   // L[lane][lane], its reciprocal
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const double* __restrict__ Lk = Ls + k * LD;
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int j = 0; j + 1 < k; j += 2) {
      const double2 l2 = *reinterpret_cast<const double2*>(Lk + j);
      s0 = fma(a[j], l2.x, s0);
      s1 = fma(a[j + 1], l2.y, s1);
    }
    if (k & 1) s0 = fma(a[k - 1], Lk[k - 1], s0);
    const double sk = a[k] - (s0 + s1);
    const double d = lane_bcast(sk, k);
    if (!(d > 0.0) || !(d < 1e300)) {    // uniform
      if (lane == 0) A.status[it] = from_start ? ST_DROP_FIRST : ST_SINGULAR;
      return;
    }
    const double lkk = sqrt(d);
    const double r = 1.0 / lkk;
    if (lane == k) {
      diag = lkk;
      rdiag = r;
      rdg[k] = r;
    }
    a[k] = lane == k ? lkk : (lane > k ? sk * r : 0.0);
    if (lane >= k && lane < P) Ls[lane * LD + k] = a[k];
    __syncthreads();   // one wave: orders the row stores before the next reads
  }
  // inverse factor X = L^{-1}: column `lane`, rows in order, x_i =
  // (delta_i - sum_{k<i} L_ik x_k) / L_ii with row i of L from LDS
  double x[P];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const double* __restrict__ Li = Ls + i * LD;
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int k = 0; k + 1 < i; k += 2) {
      const double2 l2 = *reinterpret_cast<const double2*>(Li + k);
      s0 = fma(l2.x, x[k], s0);
      s1 = fma(l2.y, x[k + 1], s1);
    }
    if (i & 1) s0 = fma(Li[i - 1], x[i - 1], s0);
    x[i] = ((lane == i ? 1.0 : 0.0) - (s0 + s1)) * rdg[i];
  }
  if (lane < P) {
#pragma unroll
    for (int k = 0; k < P; ++k) XT[lane * LD + k] = x[k];
  }
  __syncthreads();
  // 1-norm of Sigma^{-1} = X^T X: column `lane`, entry b = sum_k x_k X_kb
  // with row b of X^T from LDS.  The single-swap mode keeps Lam^{-1} =
  // D^{-1} Sigma^{-1} D^{-1} / (h-1); the distance switch takes the packed
  // inverse P~ (data units) as the factor.
  const bool keep_inv = smw_mode || dist_form;
  double n2 = 0.0;
#pragma unroll
  for (int b = 0; b < P; ++b) {
    if (b < p) {
      const double* __restrict__ Xb = XT + b * LD;
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int k = 0; k + 1 < P; k += 2) {
        const double2 x2 = *reinterpret_cast<const double2*>(Xb + k);
        s0 = fma(x[k], x2.x, s0);
        s1 = fma(x[k + 1], x2.y, s1);
      }
      if (P & 1) s0 = fma(x[P - 1], Xb[P - 1], s0);
      const double v = s0 + s1;
      n2 += fabs(v);
      if (keep_inv) {
        const double vx = v * (isc * lane_bcast(isc, b));   // (Sigma^{-1} in data units)_{lane, b}
        if (in && smw_mode) sinv[lane * PMAX + b] = vx * ih1;
        if (in && dist_form && b <= lane) mt[lane * PMAX + b] = (b < lane ? 2.0 : 1.0) * vx;
      }
    }
  }
  if (!in) n2 = 0.0;
  n2 = wave_max(n2);
  double* __restrict__ linv = A.linv + (size_t)it * MSTRIDE;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    if (i < p) {
      if (!dist_form) mt[i * PMAX + lane] = lane <= i ? x[i] * isc : 0.0;
      if (in) linv[i * PMAX + lane] = x[i];
    }
  }
  (void)rdiag;
  const double ld = wave_sum(in ? log(diag) : 0.0);
  if (lane == 0) {
    A.form[it] = dist_form ? 1 : 0;
    A.logdet[it] = 2.0 * ld;
    const double kap = n1 * n2;
    int st = ACTIVE;
    if (from_start) {
      if (!(kap < kappa_max)) st = ST_DROP_FIRST;
    } else if (A.iter[it] >= max_csteps) {
      st = ST_NOTCONV;
    } else if (!(kap < kappa_max)) {
      st = ST_ILLCOND;
    }
    A.status[it] = st;
    if (st == ACTIVE && A.nactive) atomicAdd(A.nactive, 1);
    if (st == ACTIVE && A.ldtr && A.iter[it] < A.ldtr_n)   // the step will be evaluated
      A.ldtr[(size_t)it * A.ldtr_n + A.iter[it]] = 2.0 * ld;
  }
}

__global__ __launch_bounds__(256) void k_upload_scatter(const char* __restrict__ stage) {
  const uint64_t* __restrict__ h = reinterpret_cast<const uint64_t*>(stage) + 3 * blockIdx.x;
  char* __restrict__ dst = reinterpret_cast<char*>((uintptr_t)h[0]);
  const char* __restrict__ src = stage + h[1];
  const uint64_t bytes = h[2];
  uint64_t k0 = 0;
  if ((((uintptr_t)dst | h[1]) & 15) == 0) {   // 16-byte words, then the tail
    typedef unsigned V __attribute__((ext_vector_type(4)));
    const V* __restrict__ s4 = reinterpret_cast<const V*>(src);
    V* __restrict__ d4 = reinterpret_cast<V*>(dst);
    for (uint64_t k = threadIdx.x; k < bytes / 16; k += 256) d4[k] = s4[k];
    k0 = bytes & ~(uint64_t)15;
  }
  for (uint64_t k = k0 + threadIdx.x; k < bytes; k += 256) dst[k] = src[k];
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_u8(uint8_t* p, uint8_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Inverse of a given lower Cholesky factor, row stride PMAX (low-level distance call).
__global__ void k_chol_factor(const double* __restrict__ L, int p, double* __restrict__ mt) {
  __shared__ double Li[PMAX * PMAX];
  const int tid = threadIdx.x;
  for (int j = tid; j < p; j += blockDim.x) {
    for (int i = 0; i < j; ++i) Li[i * PMAX + j] = 0.0;
    Li[j * PMAX + j] = 1.0 / L[j * p + j];
    for (int i = j + 1; i < p; ++i) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s = fma(L[i * p + k], Li[k * PMAX + j], s);
      Li[i * PMAX + j] = -s / L[i * p + i];
    }
  }
  __syncthreads();
  for (int e = tid; e < p * PMAX; e += blockDim.x) {
    const int i = e / PMAX, k = e % PMAX;
    mt[e] = (k <= i) ? Li[i * PMAX + k] : 0.0;
  }
}

// Ascending row indices of each item's subset (offset by row0 when global_rows).
__global__ __launch_bounds__(1024) void k_extract_subset(const ItemDesc* __restrict__ items,
                                                         ItemArrays A, int first_item,
                                                         int32_t* __restrict__ out,
                                                         int64_t out_stride, int global_rows) {
  __shared__ int wtot[16];
  const int it = first_item + blockIdx.x;
  const ItemDesc D = items[it];
  const uint8_t* __restrict__ mask = A.mask + D.roff;
  int32_t* __restrict__ o = out + (size_t)blockIdx.x * out_stride;
  int64_t n = 0;
  for (int64_t base = 0; base < D.m; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const int f = (i < D.m && mask[i]) ? 1 : 0;
    int tot;
    const int pos = block_excl_scan<1024>(f, wtot, tot);
    if (f && n + pos < D.h) o[n + pos] = (int32_t)(global_rows ? D.row0 + i : i);
    n += tot;
  }
}

}  // namespace

hipError_t launch_select(const ItemDesc* items, ItemArrays A, int first_item, int nitems,
                         int64_t max_m, int cstep_mode, hipStream_t s, int reset_nactive) {
  if (nitems <= 0) return hipSuccess;
  if (max_m <= (int64_t)SEL_NT * SEL_KR)
    hipLaunchKernelGGL(k_select_reg, dim3(nitems), dim3(SEL_NT), 0, s, items, A, first_item,
                       cstep_mode, reset_nactive);
  else
    hipLaunchKernelGGL(k_select, dim3(nitems), dim3(SEL_NT), 0, s, items, A, first_item,
                       cstep_mode, reset_nactive);
  return hipGetLastError();
}

hipError_t launch_finalize(int bucket, const ItemDesc* items, ItemArrays A, int first_item,
                           int nitems, int from_start, int max_csteps, double kappa_max,
                           int cstep_mode, int dist_form, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
#define CASE(PB)                                                                              \
  case PB:                                                                                    \
    hipLaunchKernelGGL((k_finalize<PB>), dim3(nitems), dim3(64), 0, s, items, A, first_item, \
                       from_start, max_csteps, kappa_max, cstep_mode, dist_form);             \
    break;
  switch (bucket) {
    CASE(4) CASE(5) CASE(8) CASE(10) CASE(16) CASE(20) CASE(24) CASE(32) CASE(40) CASE(48)
    CASE(64)
    default: return hipErrorInvalidValue;
  }
#undef CASE
  return hipGetLastError();
}

hipError_t launch_upload_scatter(const void* stage, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_upload_scatter, dim3(n), dim3(256), 0, s,
                     static_cast<const char*>(stage));
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)nb), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_fill_u8, dim3((unsigned)nb), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_chol_factor(const double* L, int p, double* mtri, hipStream_t s) {
  hipLaunchKernelGGL(k_chol_factor, dim3(1), dim3(64), 0, s, L, p, mtri);
  return hipGetLastError();
}

hipError_t launch_extract_subset(const ItemDesc* items, ItemArrays A, int first_item, int nitems,
                                 int32_t* out, int64_t out_stride, int global_rows,
                                 hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_extract_subset, dim3(nitems), dim3(1024), 0, s, items, A, first_item,
                     out, out_stride, global_rows);
  return hipGetLastError();
}

}  // namespace rtd
