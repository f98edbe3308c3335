// Row-streaming kernel: weighted sscp partial sums.
//
// Reads the rows of X once per launch and computes in float64; float32 inputs
// are widened exactly.  Instantiated per p-bucket P (p <= P, the padding
// contributes exact zeros).
#include "common.h"
#include "fitk.h"
#include "wave.h"

namespace rtd {

namespace {

template <typename T>
__device__ inline double ld_elem(const T* __restrict__ p, int64_t i) {
  return static_cast<double>(p[i]);
}

// Wrapping transform g of Sec. 3.2 (eq. wrapping) with the paper's defaults:
// z for |z| <= b, sign(z) q1 tanh(q2 (c - |z|)) for b < |z| <= c, else 0.
constexpr double WRAP_B = 1.5, WRAP_C = 4.0, WRAP_Q1 = 1.541, WRAP_Q2 = 0.862;

// ---------------------------------------------------------------------------
// Weighted sscp partial sums over one tile of candidate rows:
//   count = sum w,  s = sum w v,  S = sum w v v^T (lower triangle)
// where v is the row value of the mode (see SscpMode) and w its weight.
//
// This is a contraction over rows, so it runs on the float64 matrix cores
// (16x16x4 MFMA: 16x16 output block, 4 rows per instruction).  The row is
// extended by a constant 1 in column p, so that the block products also
// deliver the weighted sums (row p of the result) and the count (entry
// (p, p)).  Each wave stages chunks of CR rows in its own LDS region
// (contiguous rows with 16-byte loads, the next chunk's loads in flight
// while the current one is multiplied; gathered rows element by element);
// then lane l takes, for column group g, column 16 g + (l mod 16) of row
// (l div 16) of each four-row step.  That one value is the A operand (times
// the weight) of the group's block row and the B operand of its block
// column; only lower blocks (gi >= gj) are formed.  Rows of weight 0
// contribute exact zeros (their values never enter a product).  Each wave
// sums its own rows and the four waves are added in a fixed order, so
// results do not depend on scheduling.
// ---------------------------------------------------------------------------
typedef double dbl4 __attribute__((ext_vector_type(4)));

// Candidates per tile in an update step: the swap list (at most 2 (m - h)
// rows) is spread over all of the item's tiles, at least 256 per tile, so
// that short lists still keep many waves busy.
__device__ inline int64_t list_tile_rows(const ItemDesc& D) {
  const int64_t most = 2 * (D.m - D.h);
  const int64_t t = (most + D.ntiles - 1) / D.ntiles;
  return t > 256 ? t : 256;
}

template <typename T, int P>
struct SscpShape {
  static constexpr int NG = (P + 1 + 15) / 16;        // 16-column groups (with the 1 column)
  static constexpr int NBL = NG * (NG + 1) / 2;       // lower blocks
  // rows per staged chunk: at most 8 KB of row data per wave, multiple of 4
  static constexpr int CR0 = 8192 / (P * (int)sizeof(T));
  static constexpr int CR = CR0 >= 64 ? 64 : (CR0 / 4) * 4;
  static constexpr int XS = CR * P;                   // staged elements per wave
  static constexpr int NV = (XS * (int)sizeof(T) / 16 + 63) / 64;   // 16-byte loads per lane
};

template <typename T, int P, int MODE>
__global__ __launch_bounds__(256) void k_sscp(const ItemDesc* __restrict__ items, ItemArrays A,
                                              const Tile* __restrict__ tiles, int tile_rows,
                                              const double* __restrict__ wsrc,
                                              const double* __restrict__ cut) {
  using S = SscpShape<T, P>;
  constexpr int NG = S::NG, NBL = S::NBL, CR = S::CR;
  __shared__ T xs_all[4][S::XS];          // per-wave row staging
  // the wrap mode takes U four-row steps at a time (one tanh pass for all)
  constexpr int U = MODE == SSCP_WRAP ? 2 : 1;
  // block accumulators, summed wave by wave after the rows; during the rows
  // the same LDS holds each wave's tanh arguments (wrap mode)
  constexpr int TW = MODE == SSCP_WRAP ? 64 * NG * U : 0;
  constexpr int NRED = NBL * 4 * 64 > 4 * TW ? NBL * 4 * 64 : 4 * TW;
  __shared__ double red_tw[NRED];
  double(*red)[4][64] = reinterpret_cast<double(*)[4][64]>(red_tw);
  __shared__ int64_t rows_all[4][CR];     // gathered row indices (update steps)

  const Tile tl = tiles[blockIdx.x];
  const int it = tl.item;
  const ItemDesc D = items[it];
  const int p = D.p;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  T* __restrict__ xs = xs_all[wv];
  int64_t* __restrict__ rws = rows_all[wv];

  bool list_mode = false;
  int64_t nsrc = D.m;
  int kin = 0;
  if (MODE == SSCP_CSTEP) {
    if (A.status[it] != ACTIVE) return;
    if (!A.full[it]) {
      list_mode = true;
      kin = A.kswap[it];
      nsrc = 2 * (int64_t)kin;
    }
  }
  const int64_t trows = list_mode ? list_tile_rows(D) : tile_rows;
  const int64_t s0 = (int64_t)tl.t * trows;
  if (s0 >= nsrc && !(s0 == 0)) return;   // tile beyond the update list: no partial
  const int64_t s1 = min(s0 + trows, nsrc);

  double gA = 0.0, gB = 0.0, dcut = 0.0;
  if (MODE == SSCP_GSSCM) { gA = cut[2 * it]; gB = cut[2 * it + 1]; }
  if (MODE == SSCP_D2CUT) dcut = cut[D.ds];
  const T* __restrict__ X = static_cast<const T*>(D.X) + D.row0 * D.ld;

  // per-lane column constants: centre (or standardisation) of each group column
  const int kr = lane >> 4, cc = lane & 15;
  double cen[NG], isc[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const int col = 16 * g + cc;
    cen[g] = 0.0;
    isc[g] = 1.0;
    if (col < p) {
      if (MODE == SSCP_CSTEP || MODE == SSCP_D2CUT || MODE == SSCP_ADJ)
        cen[g] = A.mux[(size_t)it * PMAX + col];
      else { cen[g] = D.loc[col]; isc[g] = D.scale[col]; }
    }
  }

  dbl4 acc[NBL];
#pragma unroll
  for (int q = 0; q < NBL; ++q) acc[q] = dbl4{0.0, 0.0, 0.0, 0.0};

  // this wave's candidates: a contiguous quarter of the tile
  const int64_t wrows = (trows + 3) / 4;
  const int64_t q0 = s0 + (int64_t)wv * wrows;
  const int64_t q1 = min(q0 + wrows, s1);
  const int64_t half = D.m / 2;
  // contiguous rows of exactly P elements, 16-byte aligned: vector staging
  const bool vec = !list_mode && p == P && D.ld == P &&
                   ((reinterpret_cast<uintptr_t>(X) & 15) == 0);
  typedef unsigned V __attribute__((ext_vector_type(4)));   // 16 bytes
  V nx[S::NV];
  // selection of row b + lane in the dense modes (loaded a chunk ahead too)
  auto dense_sel = [&](int64_t b, int nn) -> bool {
    if (lane >= nn) return false;
    if (MODE == SSCP_CSTEP) return A.mask[D.roff + b + lane] != 0;
    if (MODE == SSCP_D2CUT) return A.d2[D.roff + b + lane] <= dcut;
    return true;
  };
  // real weight of row b + lane in SSCP_ADJ: cotangent / distance
  auto adj_w = [&](int64_t b, int nn) -> double {
    if (MODE != SSCP_ADJ || lane >= nn) return 0.0;
    const double dd = A.d2[D.roff + b + lane];
    return dd > 0.0 ? wsrc[D.roff + b + lane] / dd : 0.0;
  };
  int64_t base = q0;
  int n = (int)max((int64_t)0, min((int64_t)CR, q1 - base));
  bool sel_next = list_mode ? false : dense_sel(base, n);
  double w_next = adj_w(base, n);
  if (vec && base < q1) {   // vector loads of the first chunk's rows
    const V* __restrict__ src = reinterpret_cast<const V*>(X + base * P);
    const int nv = (n * P * (int)sizeof(T)) / 16;
#pragma unroll
    for (int k = 0; k < S::NV; ++k)
      if (lane + 64 * k < nv) nx[k] = src[lane + 64 * k];
  }
  for (; base < q1; base += CR) {
    // weight of row base + lane (lanes < n), and the chunk's rows into LDS
    bool sel = sel_next, neg = false;
    const double wcur = w_next;
    if (list_mode && lane < n) {
      const int64_t cand = base + lane;
      if (cand < kin) rws[lane] = A.swap[D.roff + cand];
      else { rws[lane] = A.swap[D.roff + half + (cand - kin)]; neg = true; }
      sel = true;
    }
    const uint64_t selm = __ballot(sel), negm = __ballot(neg);
    __syncwarp();   // previous chunk's reads of xs are done
    if (vec) {   // the staged loads (and a tail of single elements) into LDS
      const int nv = (n * P * (int)sizeof(T)) / 16;
      V* __restrict__ dst = reinterpret_cast<V*>(xs);
#pragma unroll
      for (int k = 0; k < S::NV; ++k)
        if (lane + 64 * k < nv) dst[lane + 64 * k] = nx[k];
      for (int e = nv * (16 / (int)sizeof(T)) + lane; e < n * P; e += 64) xs[e] = X[base * P + e];
    } else if (list_mode) {
      __syncwarp();
      for (int e = lane; e < n * P; e += 64) {
        const int r = e / P, j = e - r * P;
        xs[e] = j < p ? X[rws[r] * D.ld + j] : (T)0;
      }
    } else {
      for (int e = lane; e < n * P; e += 64) {
        const int r = e / P, j = e - r * P;
        xs[e] = j < p ? X[(base + r) * D.ld + j] : (T)0;
      }
    }
    const int64_t bn = base + CR;
    const int nn = bn < q1 ? (int)min((int64_t)CR, q1 - bn) : 0;
    if (!list_mode) sel_next = dense_sel(bn, nn);
    w_next = adj_w(bn, nn);
    if (vec && nn > 0) {   // next chunk's loads in flight
      const V* __restrict__ src = reinterpret_cast<const V*>(X + bn * P);
      const int nv = (nn * P * (int)sizeof(T)) / 16;
#pragma unroll
      for (int k = 0; k < S::NV; ++k)
        if (lane + 64 * k < nv) nx[k] = src[lane + 64 * k];
    }
    __syncwarp();   // staged rows visible to the whole wave
    for (int st = 0; st < n; st += 4 * U) {
      double v[U][NG], wu[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int r = st + 4 * u + kr;
        const bool on = r < n && ((selm >> r) & 1ull);
        double w = on ? (((negm >> r) & 1ull) ? -1.0 : 1.0) : 0.0;
        double r2 = 0.0;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
          const int col = 16 * g + cc;
          double z = 0.0;
          if (col < p) {
            const double x = r < n ? (double)xs[r * P + col] : 0.0;
            if (MODE == SSCP_CSTEP || MODE == SSCP_D2CUT || MODE == SSCP_ADJ) z = x - cen[g];
            else z = (x - cen[g]) / isc[g];
            if (MODE == SSCP_GSSCM) r2 = fma(z, z, r2);
          } else if (col == p) {
            z = 1.0;
          }
          v[u][g] = z;
        }
        if (MODE == SSCP_ADJ) {
          const double wr = __shfl(wcur, r < n ? r : 0, 64);
          w = on ? wr : 0.0;
        }
        if (MODE == SSCP_GSSCM) {
          // weight xi^2(||z||) of eq. (LR); the 16 lanes of a row add their parts
          r2 = row16_sum(r2);
          const double rr = sqrt(r2);
          double xi;
          if (gB <= gA) xi = (rr <= gA) ? 1.0 : 0.0;
          else xi = (rr <= gA) ? 1.0 : ((rr <= gB) ? (gB - rr) / (gB - gA) : 0.0);
          w = on ? xi * xi : 0.0;
        }
        wu[u] = w;
      }
      if (MODE == SSCP_WRAP) {
        // g of every value of the U steps; the tanh branch (a minority of
        // the values) is evaluated once for all of the wave's values that
        // take it, gathered in LDS, instead of once per column group and step
        double* __restrict__ tw = red_tw + wv * TW;
        const uint64_t below = (1ull << lane) - 1ull;
        int cnt = 0, slot[U][NG];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int g = 0; g < NG; ++g) {
            const double a = fabs(v[u][g]);
            const bool mid = !(a <= WRAP_B) && a <= WRAP_C;
            const uint64_t m = __ballot(mid);
            slot[u][g] = mid ? cnt + __popcll(m & below) : -1;
            if (mid) tw[slot[u][g]] = WRAP_Q2 * (WRAP_C - a);
            cnt += __popcll(m);
          }
        __syncwarp();
        for (int b0 = 0; b0 < cnt; b0 += 64)
          if (b0 + lane < cnt) tw[b0 + lane] = tanh(tw[b0 + lane]);
        __syncwarp();
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int g = 0; g < NG; ++g) {
            const double a = fabs(v[u][g]);
            if (slot[u][g] >= 0) v[u][g] = copysign(WRAP_Q1 * tw[slot[u][g]], v[u][g]);
            else if (!(a <= WRAP_C)) v[u][g] = 0.0;
          }
        __syncwarp();   // tw is free for the next steps
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (st + 4 * u >= n) break;   // uniform: no rows left in the chunk
        const double w = wu[u];
        double av[NG], bv[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) {
          bv[g] = w == 0.0 ? 0.0 : v[u][g];
          av[g] = w * bv[g];
        }
        int q = 0;
#pragma unroll
        for (int gi = 0; gi < NG; ++gi)
#pragma unroll
          for (int gj = 0; gj <= gi; ++gj, ++q)
            acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[gi], bv[gj], acc[q], 0, 0, 0);
      }
    }
    n = nn;
  }

  // fixed-order sum over the four waves (wave 0 first) and the tile partial
  if (MODE == SSCP_WRAP) __syncthreads();   // every wave is done with its tanh arguments
  for (int k = 0; k < 4; ++k) {
    if (wv == k) {
#pragma unroll
      for (int q = 0; q < NBL; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) red[q][e][lane] = k == 0 ? acc[q][e] : red[q][e][lane] + acc[q][e];
    }
    __syncthreads();
  }
  double* __restrict__ part = A.part + (size_t)(D.tile0 + tl.t) * PSTRIDE;
  for (int o = tid; o < NBL * 4 * 64; o += 256) {
    const int q = o / 256, e = (o / 64) % 4, l = o % 64;
    const double sum = red[q][e][l];
    // block q = (gi, gj); lane l, register e hold entry (16 gi + l/16 + 4 e, 16 gj + l%16)
    int gi = 0, k = q;
    while (k > gi) { k -= gi + 1; ++gi; }
    const int gj = k;
    const int I = 16 * gi + (l >> 4) + 4 * e, J = 16 * gj + (l & 15);
    if (I < p && J <= I) part[1 + PMAX + I * (I + 1) / 2 + J] = sum;
    else if (I == p && J < p) part[1 + J] = sum;
    else if (I == p && J == p) part[0] = sum;
  }
}

template <typename T, int P>
hipError_t sscp_t(int mode, const ItemDesc* items, ItemArrays A, const Tile* tiles, int ntiles,
                  int tile_rows, const double* wsrc, const double* cut,
                  hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  switch (mode) {
    case SSCP_CSTEP:
      hipLaunchKernelGGL((k_sscp<T, P, SSCP_CSTEP>), dim3(ntiles), dim3(256), 0, s, items, A,
                         tiles, tile_rows, wsrc, cut);
      break;
    case SSCP_D2CUT:
      hipLaunchKernelGGL((k_sscp<T, P, SSCP_D2CUT>), dim3(ntiles), dim3(256), 0, s, items, A,
                         tiles, tile_rows, wsrc, cut);
      break;
    case SSCP_WRAP:
      hipLaunchKernelGGL((k_sscp<T, P, SSCP_WRAP>), dim3(ntiles), dim3(256), 0, s, items, A,
                         tiles, tile_rows, wsrc, cut);
      break;
    case SSCP_GSSCM:
      hipLaunchKernelGGL((k_sscp<T, P, SSCP_GSSCM>), dim3(ntiles), dim3(256), 0, s, items, A,
                         tiles, tile_rows, wsrc, cut);
      break;
    case SSCP_ADJ:
      hipLaunchKernelGGL((k_sscp<T, P, SSCP_ADJ>), dim3(ntiles), dim3(256), 0, s, items, A,
                         tiles, tile_rows, wsrc, cut);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Collapse of an item's tile partials into the partial of its first tile, in
// a fixed order: level 0 sums runs of COL_CT consecutive tiles into the first
// tile of each run, level 1 sums the run heads.  cstep = 1: only the tiles
// the C-step sscp wrote (all in full mode, those covering the swap list in
// update mode) take part, and inactive items are skipped.
// ---------------------------------------------------------------------------
constexpr int COL_CT = 32;
constexpr int COL_U = 8;

__global__ __launch_bounds__(256) void k_collapse(const ItemDesc* __restrict__ items, ItemArrays A,
                                                  int first, int cstep, int tile_rows, int level) {
  const int it = first + blockIdx.x;
  if (cstep && A.status[it] != ACTIVE) return;
  const ItemDesc D = items[it];
  int nv = D.ntiles;
  if (cstep) {
    const bool full = A.full[it] != 0;
    const int64_t nsrc = full ? D.m : 2 * (int64_t)A.kswap[it];
    const int64_t trows = full ? tile_rows : list_tile_rows(D);
    nv = (int)((nsrc + trows - 1) / trows);
    if (nv < 1) nv = 1;
  }
  int t0, t1, stride;
  if (level == 0) {
    t0 = (int)blockIdx.y * COL_CT;
    t1 = min(t0 + COL_CT, nv);
    stride = 1;
  } else {
    t0 = 0;
    t1 = (nv + COL_CT - 1) / COL_CT;
    stride = COL_CT;
  }
  if (t1 - t0 <= 1) return;
  const int p = D.p;
  const int E = 1 + p + p * (p + 1) / 2;
  double* __restrict__ base = A.part + (size_t)D.tile0 * PSTRIDE;
  for (int e = threadIdx.x; e < E; e += blockDim.x) {
    const int idx = e <= p ? e : 1 + PMAX + (e - 1 - p);
    double s = 0.0;
    for (int k = t0; k < t1; k += COL_U) {
      double v[COL_U];
#pragma unroll
      for (int u = 0; u < COL_U; ++u)
        v[u] = (k + u < t1) ? base[(size_t)(k + u) * stride * PSTRIDE + idx] : 0.0;
#pragma unroll
      for (int u = 0; u < COL_U; ++u) s += v[u];
    }
    base[(size_t)t0 * stride * PSTRIDE + idx] = s;
  }
}

}  // namespace

hipError_t launch_collapse(const ItemDesc* items, ItemArrays A, int first, int nitems,
                           int max_ntiles, int cstep, int tile_rows, hipStream_t s) {
  if (nitems <= 0 || max_ntiles <= 1) return hipSuccess;
  const int nch = (max_ntiles + COL_CT - 1) / COL_CT;
  hipLaunchKernelGGL(k_collapse, dim3(nitems, nch), dim3(256), 0, s, items, A, first, cstep,
                     tile_rows, 0);
  if (nch > 1)
    hipLaunchKernelGGL(k_collapse, dim3(nitems), dim3(256), 0, s, items, A, first, cstep,
                       tile_rows, 1);
  return hipGetLastError();
}

#define RTD_BUCKETS(X) X(4) X(5) X(8) X(10) X(16) X(20) X(24) X(32) X(40) X(48) X(64)

hipError_t launch_sscp(int bucket, int dtype, int mode, const ItemDesc* items, ItemArrays A,
                       const Tile* tiles, int ntiles, int tile_rows, const double* wsrc,
                       const double* cut, hipStream_t s) {
#define CASE(PB)                                                                         \
  case PB:                                                                               \
    return dtype == 0 ? sscp_t<float, PB>(mode, items, A, tiles, ntiles, tile_rows, wsrc, \
                                          cut, s)                                      \
                      : sscp_t<double, PB>(mode, items, A, tiles, ntiles, tile_rows, wsrc, \
                                           cut, s);
  switch (bucket) {
    RTD_BUCKETS(CASE)
    default: return hipErrorInvalidValue;
  }
#undef CASE
}

}  // namespace rtd
