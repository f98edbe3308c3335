// Row-streaming kernel: weighted sscp partial sums.
//
// Reads the rows of X once per launch and computes in float64; float32 inputs
// are widened exactly.  Instantiated per p-bucket P (p <= P, the padding
// contributes exact zeros).
#include "common.h"
#include "fitk.h"

namespace rtd {

namespace {

template <typename T>
__device__ inline double ld_elem(const T* __restrict__ p, int64_t i) {
  return static_cast<double>(p[i]);
}

// Wrapping transform g of Sec. 3.2 (eq. wrapping) with the paper's defaults.
__device__ inline double wrap_g(double z) {
  const double b = 1.5, c = 4.0, q1 = 1.541, q2 = 0.862;
  const double a = fabs(z);
  if (a <= b) return z;
  if (a <= c) return copysign(q1 * tanh(q2 * (c - a)), z);
  return 0.0;
}

// ---------------------------------------------------------------------------
// Weighted sscp partial sums over one tile of candidate rows:
//   count = sum w,  s = sum w v,  S = sum w v v^T (lower triangle)
// where v is the row value of the mode (see SscpMode) and w its weight.
// Selected rows are compacted into LDS in batches and the lower triangle is
// accumulated in 4x4 register blocks; every reduction has a fixed order, so
// results do not depend on scheduling.
// ---------------------------------------------------------------------------
template <int P>
struct SscpShape {
  static constexpr int NB = (P + 3) / 4;              // 4-wide column blocks
  static constexpr int NBLK = NB * (NB + 1) / 2;      // lower blocks
  static constexpr int NRL = 256 / NBLK;              // row lanes
  static constexpr int BR = P <= 40 ? 128 : 64;      // rows per batch
  static constexpr int PP = NB * 4 + 1;               // padded LDS row pitch (doubles)
  static constexpr int XS = BR * PP;
  static constexpr int RED = NRL * NBLK * 16;
  static constexpr int LDSD = XS > RED ? XS : RED;
  static constexpr int NRR = 256 / P;                 // row lanes of the sum vector
};

template <typename T, int P, int MODE>
__global__ __launch_bounds__(256) void k_sscp(const ItemDesc* __restrict__ items, ItemArrays A,
                                              const Tile* __restrict__ tiles, int tile_rows,
                                              const double* __restrict__ pivot, int pivot_stride,
                                              const double* __restrict__ cut) {
  using S = SscpShape<P>;
  __shared__ double lds[S::LDSD];
  __shared__ double wsh[S::BR];
  __shared__ int64_t rsh[S::BR];
  __shared__ int wcount[4];
  __shared__ double sred[256];

  const Tile tl = tiles[blockIdx.x];
  const int it = tl.item;
  const ItemDesc D = items[it];
  const int p = D.p;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;

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
  const int64_t s0 = (int64_t)tl.t * tile_rows;
  if (s0 >= nsrc && !(s0 == 0)) return;   // tile beyond the update list: no partial
  const int64_t s1 = min(s0 + (int64_t)tile_rows, nsrc);

  __shared__ double c[P];   // centre of the rows (the item's current mean)
  for (int j = tid; j < P; j += 256)
    c[j] = ((MODE == SSCP_CSTEP || MODE == SSCP_D2CUT) && j < p) ? A.mux[(size_t)it * PMAX + j]
                                                                 : 0.0;
  double gA = 0.0, gB = 0.0, dcut = 0.0;
  if (MODE == SSCP_GSSCM) { gA = cut[2 * it]; gB = cut[2 * it + 1]; }
  if (MODE == SSCP_D2CUT) dcut = cut[D.ds];

  const T* __restrict__ X = static_cast<const T*>(D.X) + D.row0 * D.ld;

  // block accumulators
  const int blk = tid % S::NBLK;
  const int rl = tid / S::NBLK;
  int bi = 0, bj = 0;
  {
    int k = blk;
    while (k > bi) { k -= bi + 1; ++bi; }
    bj = k;
  }
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  const int sj = tid % P, srr = tid / P;
  double sacc = 0.0, wacc = 0.0;

  for (int64_t base = s0; base < s1; base += S::BR) {
    // 1. evaluate candidates and compact the selected rows (order preserving)
    int64_t row = -1;
    double w = 0.0;
    const int64_t cand = base + tid;
    if (tid < S::BR && cand < s1) {
      if (MODE == SSCP_CSTEP) {
        if (list_mode) {
          const int64_t half = D.m / 2;
          if (cand < kin) { row = A.swap[D.roff + cand]; w = 1.0; }
          else { row = A.swap[D.roff + half + (cand - kin)]; w = -1.0; }
        } else if (A.mask[D.roff + cand]) {
          row = cand; w = 1.0;
        }
      } else if (MODE == SSCP_D2CUT) {
        if (A.d2[D.roff + cand] <= dcut) { row = cand; w = 1.0; }
      } else if (MODE == SSCP_WRAP) {
        row = cand; w = 1.0;
      } else {  // GSSCM: weight xi^2(||z||) of eq. (LR)
        const T* xr = X + cand * D.ld;
        double r2 = 0.0;
#pragma unroll
        for (int j = 0; j < P; ++j)
          if (j < p) {
            const double z = (ld_elem(xr, j) - D.loc[j]) / D.scale[j];
            r2 = fma(z, z, r2);
          }
        const double r = sqrt(r2);
        double xi;
        if (gB <= gA) xi = (r <= gA) ? 1.0 : 0.0;
        else xi = (r <= gA) ? 1.0 : ((r <= gB) ? (gB - r) / (gB - gA) : 0.0);
        row = cand; w = xi * xi;
      }
    }
    const bool sel = row >= 0 && w != 0.0;
    const uint64_t bal = __ballot(sel);
    const int pos_w = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wcount[wv] = __popcll(bal);
    __syncthreads();
    int off = 0, nb = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (k < wv) off += wcount[k];
      nb += wcount[k];
    }
    if (sel) { rsh[off + pos_w] = row; wsh[off + pos_w] = w; }
    __syncthreads();
    // 2. load the selected rows, transformed, into LDS (a fixed trip count so
    // that every load of the batch is issued before the first one is used)
    {
      constexpr int NE = (S::BR * P + 255) / 256;
      double xv[NE];
#pragma unroll
      for (int k = 0; k < NE; ++k) {
        const int e = tid + k * 256;
        const int r = e / P, j = e - r * P;
        xv[k] = (e < nb * P && j < p) ? ld_elem(X + rsh[r] * D.ld, j) : 0.0;
      }
#pragma unroll
      for (int k = 0; k < NE; ++k) {
        const int e = tid + k * 256;
        if (e < nb * P) {
          const int r = e / P, j = e - r * P;
          double v = 0.0;
          if (j < p) v = (MODE == SSCP_CSTEP || MODE == SSCP_D2CUT) ? xv[k] - c[j] : xv[k];
          lds[r * S::PP + j] = v;
        }
      }
      if (MODE == SSCP_WRAP || MODE == SSCP_GSSCM) {
        // standardise (and wrap) in place: the same thread wrote these entries
        for (int e = tid; e < nb * P; e += 256) {
          const int r = e / P, j = e - r * P;
          if (j < p) {
            const double z = (lds[r * S::PP + j] - D.loc[j]) / D.scale[j];
            lds[r * S::PP + j] = MODE == SSCP_WRAP ? wrap_g(z) : z;
          }
        }
      }
    }
    for (int e = tid; e < nb * (S::PP - P); e += 256) {
      const int r = e / (S::PP - P), j = P + e % (S::PP - P);
      lds[r * S::PP + j] = 0.0;
    }
    __syncthreads();
    // 3. accumulate the lower-triangular 4x4 blocks
    if (rl < S::NRL) {
      for (int r = rl; r < nb; r += S::NRL) {
        const double* xr = lds + r * S::PP;
        const double wr = wsh[r];
        double a[4], b[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) { a[k] = wr * xr[4 * bi + k]; b[k] = xr[4 * bj + k]; }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
      }
    }
    if (srr < S::NRR) {
      for (int r = srr; r < nb; r += S::NRR) {
        sacc = fma(wsh[r], lds[r * S::PP + sj], sacc);
        if (sj == 0) wacc += wsh[r];
      }
    }
    __syncthreads();
  }

  // 4. fixed-order reductions and the tile partial
  double* __restrict__ part = A.part + (size_t)(D.tile0 + tl.t) * PSTRIDE;
  if (rl < S::NRL) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) lds[(rl * S::NBLK + blk) * 16 + u * 4 + v] = acc[u][v];
  }
  sred[tid] = (srr < S::NRR) ? sacc : 0.0;
  __syncthreads();
  for (int o = tid; o < S::NBLK * 16; o += 256) {
    const int b = o / 16, e = o % 16;
    double s = 0.0;
    for (int k = 0; k < S::NRL; ++k) s += lds[(k * S::NBLK + b) * 16 + e];
    int bi2 = 0, k2 = b;
    while (k2 > bi2) { k2 -= bi2 + 1; ++bi2; }
    const int i = 4 * bi2 + e / 4, j = 4 * k2 + e % 4;
    if (i < p && j <= i) part[1 + PMAX + i * (i + 1) / 2 + j] = s;
  }
  if (tid < P && tid < p) {
    double s = 0.0;
    for (int k = 0; k < S::NRR; ++k) s += sred[k * P + tid];
    part[1 + tid] = s;
  }
  __syncthreads();
  sred[tid] = (sj == 0 && srr < S::NRR) ? wacc : 0.0;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int k = 0; k < S::NRR; ++k) s += sred[k * P];
    part[0] = s;
  }
}

template <typename T, int P>
hipError_t sscp_t(int mode, const ItemDesc* items, ItemArrays A, const Tile* tiles, int ntiles,
                  int tile_rows, const double* pivot, int pivot_stride, const double* cut,
                  hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  switch (mode) {
    case SSCP_CSTEP:
      hipLaunchKernelGGL((k_sscp<T, P, SSCP_CSTEP>), dim3(ntiles), dim3(256), 0, s, items, A,
                         tiles, tile_rows, pivot, pivot_stride, cut);
      break;
    case SSCP_D2CUT:
      hipLaunchKernelGGL((k_sscp<T, P, SSCP_D2CUT>), dim3(ntiles), dim3(256), 0, s, items, A,
                         tiles, tile_rows, pivot, pivot_stride, cut);
      break;
    case SSCP_WRAP:
      hipLaunchKernelGGL((k_sscp<T, P, SSCP_WRAP>), dim3(ntiles), dim3(256), 0, s, items, A,
                         tiles, tile_rows, pivot, pivot_stride, cut);
      break;
    default:
      hipLaunchKernelGGL((k_sscp<T, P, SSCP_GSSCM>), dim3(ntiles), dim3(256), 0, s, items, A,
                         tiles, tile_rows, pivot, pivot_stride, cut);
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
    const int64_t nsrc = A.full[it] ? D.m : 2 * (int64_t)A.kswap[it];
    nv = (int)((nsrc + tile_rows - 1) / tile_rows);
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
                       const Tile* tiles, int ntiles, int tile_rows, const double* pivot,
                       int pivot_stride, const double* cut, hipStream_t s) {
#define CASE(PB)                                                                         \
  case PB:                                                                               \
    return dtype == 0 ? sscp_t<float, PB>(mode, items, A, tiles, ntiles, tile_rows, pivot, \
                                          pivot_stride, cut, s)                          \
                      : sscp_t<double, PB>(mode, items, A, tiles, ntiles, tile_rows, pivot, \
                                           pivot_stride, cut, s);
  switch (bucket) {
    RTD_BUCKETS(CASE)
    default: return hipErrorInvalidValue;
  }
#undef CASE
}

}  // namespace rtd
