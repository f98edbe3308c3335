// Statistical distances (Sec. 2.1 eq. statdist computed as in Sec. 3.4):
// d2 = ||M (x - mu)||^2 with M the inverse Cholesky factor (folded with the
// standardisation scales inside the fit).  An item whose form word is 1
// holds instead the explicit inverse P of its scatter, packed like M as a
// lower triangle with doubled off-diagonal entries (P~), and
// d2 = sum_i r_i (P~ r)_i = r^T P r: the distance computation that Sec. 3.4
// replaces (Table 1, version I), and the form the single-swap update of
// Sec. 3.5 produces.  Both forms cost p(p+1)/2 multiply-adds per row.
//
// Every thread reads its own row straight into registers (16- or 8-byte
// loads when the row size and base allow, else one load per element), and
// each block takes one 256-row slice, so no LDS, no barrier and a full chip
// of short blocks.  The factor and the centre are read at uniform offsets:
// the loads go through the scalar unit and every FMA takes its M entry from
// scalar registers.  The factor is evaluated column by column (y_i += M_ij
// z_j over j, the p partial sums independent of one another, each still
// summed in order of j); above p = 40 the outputs are formed 16 at a time,
// the same operations in the same order, so that the partial sums fit the
// registers.  The C-step runs it over both starts' items of a block (each
// row read twice: faster than one read feeding two factors).
#include <stdint.h>

#include "common.h"
#include "fitk.h"
#include "rowload.h"

namespace rtd {

namespace {

// ---------------------------------------------------------------------------
// Direct row evaluation.

constexpr int DROWS = 256;     // rows per block of the direct kernels
constexpr int DIRECT_MAX = 64; // widest bucket evaluated directly

template <typename T, int P>
struct RowVec {
  static constexpr int BYTES = P * (int)sizeof(T);
  static constexpr int VB = BYTES % 16 == 0 ? 16 : BYTES % 8 == 0 ? 8 : (int)sizeof(T);
  static constexpr int E = VB / (int)sizeof(T);   // elements per load
};

// Row r of a dense, VB-aligned row-major matrix of P columns.
template <typename T, int P>
__device__ inline void load_row_vec(const T* xr_, T (&v)[P]) {
  constexpr int E = RowVec<T, P>::E;
  const gptr_t<T> xr = as_global(xr_);
  if constexpr (E == 1) {
#pragma unroll
    for (int j = 0; j < P; ++j) v[j] = xr[j];
  } else {
    typedef T V __attribute__((ext_vector_type(E)));
    const V __attribute__((address_space(1)))* s =
        (const V __attribute__((address_space(1)))*)xr;
#pragma unroll
    for (int u = 0; u < P / E; ++u) {
      const V t = s[u];
#pragma unroll
      for (int c = 0; c < E; ++c) v[u * E + c] = t[c];
    }
  }
}

// ||M (v - mu)||^2 column by column: y_i accumulates M_ij z_j in order of j
// (the same operations, in the same order per y_i, as the row-wise form).
// INV: z^T (M z) with M = P~ (explicit inverse).
template <typename T, int P, bool INV>
__device__ inline double col_norm2_g(const double* __restrict__ Mg, int ldm, int p,
                                     const double* __restrict__ mu, const T (&v)[P]) {
  if constexpr (P > 40) {
    // wide rows: the outputs 16 at a time (each y_i still sums over j in
    // order, and acc over i in order: the same operations as below)
    constexpr int B = 16;
    double acc = 0.0;
#pragma unroll
    for (int b0 = 0; b0 < P; b0 += B) {
      double y[B];
#pragma unroll
      for (int ii = 0; ii < B; ++ii) y[ii] = 0.0;
#pragma unroll
      for (int j = 0; j < b0 + B && j < P; ++j) {
        if (j < p) {
          const double zj = (double)v[j] - mu[j];
#pragma unroll
          for (int ii = 0; ii < B; ++ii) {
            const int i = b0 + ii;
            if (i >= j && i < p) y[ii] = fma(Mg[i * ldm + j], zj, y[ii]);
          }
        }
      }
#pragma unroll
      for (int ii = 0; ii < B; ++ii) {
        const int i = b0 + ii;
        if (i < p) acc = fma(y[ii], INV ? (double)v[i] - mu[i] : y[ii], acc);
      }
    }
    return acc;
  } else {
    double y[P];
#pragma unroll
    for (int i = 0; i < P; ++i) y[i] = 0.0;
#pragma unroll
    for (int j = 0; j < P; ++j) {
      if (j < p) {
        const double zj = (double)v[j] - mu[j];
#pragma unroll
        for (int i = j; i < P; ++i)
          if (i < p) y[i] = fma(Mg[i * ldm + j], zj, y[i]);
      }
    }
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < P; ++i)
      if (i < p) acc = fma(y[i], INV ? (double)v[i] - mu[i] : y[i], acc);
    return acc;
  }
}

template <typename T, int P, int NI, bool INV, typename Emit>
__device__ inline void eval_row(T (&v)[P], int p, int ldm, const double* const (&Mg)[NI],
                                const double* const (&mug)[NI], const bool (&act)[NI],
                                Emit emit) {
  // the factors one after the other on the same row, each column by column;
  // between them the row goes through all_loaded again, so that its float64
  // conversions are not kept live from the first factor to the second (the
  // launches use one factor per pass)
#pragma unroll
  for (int q = 0; q < NI; ++q) {
    if (q > 0) all_loaded(v);
    if (act[q]) emit(q, col_norm2_g<T, P, INV>(Mg[q], ldm, p, mug[q], v));
  }
}

// Row r of X; emit(q, d2) for each active factor.  LDM_IS_P: the factor's row
// stride is p (a p x p factor), which the fast path then knows to be P.
// GEN: rows may be narrower than P, strided or unaligned (checked per item);
// without it the launch guarantees dense, aligned rows of P columns.
// INV: the factors are P~ (explicit inverse).
template <typename T, int P, int NI, bool LDM_IS_P, bool GEN, bool INV, typename Emit>
__device__ inline void dist_row_direct(const T* __restrict__ X, int64_t ld, int p, int ldm,
                                       int64_t r, const double* const (&Mg)[NI],
                                       const double* const (&mug)[NI], const bool (&act)[NI],
                                       Emit emit) {
  constexpr int VB = RowVec<T, P>::VB;
  const bool fast = !GEN || (p == P && ld == P && ((reinterpret_cast<uintptr_t>(X) % VB) == 0));
  T v[P];
  if (fast) {
    load_row_vec<T, P>(X + r * P, v);
    all_loaded(v);
    eval_row<T, P, NI, INV>(v, P, LDM_IS_P ? P : ldm, Mg, mug, act, emit);   // guards fold
  } else if constexpr (GEN) {
    const gptr_t<T> xr = as_global(X + r * ld);
#pragma unroll
    for (int j = 0; j < P; ++j) v[j] = j < p ? xr[j] : (T)0;
    all_loaded(v);
    eval_row<T, P, NI, INV>(v, p, ldm, Mg, mug, act, emit);
  }
}

// PER_ITEM: read each tile's distance form (form may then be null: all
// Cholesky); without it every factor of the launch is L^{-1} D^{-1} (the
// default path carries no second evaluation).
template <typename T, int P, int NI, bool GEN, bool PER_ITEM>
__global__ __launch_bounds__(DROWS) void k_dist_direct(const ItemDesc* __restrict__ items,
                                                       const Tile* __restrict__ tiles,
                                                       int tile_rows,
                                                       const double* __restrict__ mtri,
                                                       const double* __restrict__ mux,
                                                       const int32_t* __restrict__ status,
                                                       const int32_t* __restrict__ form,
                                                       double* __restrict__ d2) {
  const int nsub = tile_rows / DROWS;
  const Tile tl = tiles[blockIdx.x / nsub];
  bool act[NI];
  bool any = false;
#pragma unroll
  for (int q = 0; q < NI; ++q) {
    act[q] = status == nullptr || status[tl.item + q] == ACTIVE;
    any = any || act[q];
  }
  if (!any) return;
  const ItemDesc D = items[tl.item];
  const int64_t t0 = (int64_t)tl.t * tile_rows;
  const int64_t r = t0 + (int64_t)(blockIdx.x % nsub) * DROWS + threadIdx.x;
  if (r >= min(t0 + (int64_t)tile_rows, D.m)) return;
  int64_t roff[NI];
  const double* Mg[NI];
  const double* mug[NI];
#pragma unroll
  for (int q = 0; q < NI; ++q) {
    const int it = tl.item + q;
    roff[q] = items[it].roff;
    Mg[q] = mtri + (size_t)it * MSTRIDE;
    mug[q] = mux + (size_t)it * PMAX;
  }
  const T* __restrict__ X = static_cast<const T*>(D.X) + D.row0 * D.ld;
  auto emit = [&](int q, double v) { d2[roff[q] + r] = v; };
  // the form of the tile's factor (uniform over the block; one factor per
  // tile in the direct launches)
  if (PER_ITEM && form != nullptr && form[tl.item] != 0)
    dist_row_direct<T, P, NI, false, GEN, true>(X, D.ld, D.p, PMAX, r, Mg, mug, act, emit);
  else
    dist_row_direct<T, P, NI, false, GEN, false>(X, D.ld, D.p, PMAX, r, Mg, mug, act, emit);
}

template <typename T, int P, bool GEN, bool PER_ITEM>
__global__ __launch_bounds__(DROWS) void k_final_dist_direct(
    const ItemDesc* __restrict__ items, const Tile* __restrict__ tiles, int tile_rows,
    const double* __restrict__ mtri, const double* __restrict__ mux,
    const int32_t* __restrict__ form, const double* __restrict__ d2,
    const DsInfo* __restrict__ ds, const rtdetmcd_out* __restrict__ outs) {
  const int nsub = tile_rows / DROWS;
  const Tile tl = tiles[blockIdx.x / nsub];
  const int it = tl.item;
  const ItemDesc D = items[it];
  const int64_t t0 = (int64_t)tl.t * tile_rows;
  const int64_t r = t0 + (int64_t)(blockIdx.x % nsub) * DROWS + threadIdx.x;
  if (r >= min(t0 + (int64_t)tile_rows, D.m)) return;
  const DsInfo dd = ds[D.ds];
  if (dd.err) return;
  const double cut = dd.chi2p;
  double* __restrict__ od = outs[D.ds].dist;
  uint8_t* __restrict__ of = outs[D.ds].outlier;
  uint8_t* __restrict__ ow = outs[D.ds].rew_mask;
  // reweighting set: as in k_final_dist
  const ItemDesc R = items[dd.glob0];
  const double* __restrict__ d2r = d2 + R.roff;
  const T* __restrict__ X = static_cast<const T*>(D.X) + D.row0 * D.ld;
  const double* Mg[1] = {mtri + (size_t)it * MSTRIDE};
  const double* mug[1] = {mux + (size_t)it * PMAX};
  const bool act[1] = {true};
  auto emit = [&](int, double v) {
    if (od) od[D.row0 + r] = sqrt(v);
    if (of) of[D.row0 + r] = v > cut ? 1 : 0;
    if (ow) {
      // position of the row among the fitted rows (through the inverse
      // permutation for a random partition)
      const int64_t rr = dd.inv ? (int64_t)dd.inv[D.row0 + r] : D.row0 + r - R.row0;
      ow[D.row0 + r] = (rr >= 0 && rr < R.m && d2r[rr] <= cut) ? 1 : 0;
    }
  };
  if (PER_ITEM && form != nullptr && form[it] != 0)
    dist_row_direct<T, P, 1, false, GEN, true>(X, D.ld, D.p, PMAX, r, Mg, mug, act, emit);
  else
    dist_row_direct<T, P, 1, false, GEN, false>(X, D.ld, D.p, PMAX, r, Mg, mug, act, emit);
}

template <typename T, int P, bool GEN>
__global__ __launch_bounds__(DROWS) void k_score_direct(const T* __restrict__ X, int64_t n,
                                                        int64_t ld, int p,
                                                        const double* __restrict__ mu,
                                                        const double* __restrict__ M,
                                                        double cut, double* __restrict__ dist,
                                                        uint8_t* __restrict__ flag) {
  const int64_t r = (int64_t)blockIdx.x * DROWS + threadIdx.x;
  if (r >= n) return;
  const double* Mg[1] = {M};
  const double* mug[1] = {mu};
  const bool act[1] = {true};
  dist_row_direct<T, P, 1, true, GEN, false>(X, ld, p, p, r, Mg, mug, act, [&](int, double v) {
    if (dist) dist[r] = sqrt(v);
    if (flag) flag[r] = v > cut ? 1 : 0;
  });
}

}  // namespace

#define RTD_DIRECT_BUCKETS(X) X(4) X(5) X(8) X(10) X(16) X(20) X(24) X(32) X(40) X(48) X(64)
static_assert(DIRECT_MAX == 64, "bucket lists");

hipError_t launch_dist(int bucket, int dtype, int dense, const ItemDesc* items,
                       const Tile* tiles,
                       int ntiles, int tile_rows, const double* mtri, const double* mux,
                       const int32_t* status, const int32_t* form, double* d2, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (tile_rows <= 0 || tile_rows % DROWS != 0) return hipErrorInvalidValue;
  const unsigned nbd = (unsigned)ntiles * (unsigned)(tile_rows / DROWS);
#define LAUNCH(K)                                                                               \
  hipLaunchKernelGGL(K, dim3(nbd), dim3(DROWS), 0, s, items, tiles, tile_rows, mtri, mux,      \
                     status, form, d2)
#define DIRECT(T, PB)                                                                           \
  do {                                                                                          \
    if (dense && !form) LAUNCH((k_dist_direct<T, PB, 1, false, false>));                        \
    else if (dense) LAUNCH((k_dist_direct<T, PB, 1, false, true>));                             \
    else LAUNCH((k_dist_direct<T, PB, 1, true, true>));                                         \
  } while (0)
#define CASE(PB)                                                                                \
  case PB:                                                                                      \
    if (dtype == 0) DIRECT(float, PB);                                                          \
    else DIRECT(double, PB);                                                                    \
    return hipGetLastError();
  switch (bucket) {
    RTD_DIRECT_BUCKETS(CASE)
    default: return hipErrorInvalidValue;
  }
#undef CASE
#undef DIRECT
#undef LAUNCH
}

hipError_t launch_final_dist(int bucket, int dtype, int dense, const ItemDesc* items,
                             const Tile* tiles,
                             int ntiles, int tile_rows, const double* mtri, const double* mux,
                             const int32_t* form, const double* d2, const DsInfo* ds,
                             const rtdetmcd_out* outs, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (tile_rows <= 0 || tile_rows % DROWS != 0) return hipErrorInvalidValue;
  const unsigned nbd = (unsigned)ntiles * (unsigned)(tile_rows / DROWS);
#define LAUNCH(K)                                                                               \
  hipLaunchKernelGGL(K, dim3(nbd), dim3(DROWS), 0, s, items, tiles, tile_rows, mtri, mux,      \
                     form, d2, ds, outs)
#define DIRECT(T, PB)                                                                           \
  do {                                                                                          \
    if (dense && !form) LAUNCH((k_final_dist_direct<T, PB, false, false>));                     \
    else if (dense) LAUNCH((k_final_dist_direct<T, PB, false, true>));                          \
    else LAUNCH((k_final_dist_direct<T, PB, true, true>));                                      \
  } while (0)
#define CASE(PB)                                                                                \
  case PB:                                                                                      \
    if (dtype == 0) DIRECT(float, PB);                                                          \
    else DIRECT(double, PB);                                                                    \
    return hipGetLastError();
  switch (bucket) {
    RTD_DIRECT_BUCKETS(CASE)
    default: return hipErrorInvalidValue;
  }
#undef CASE
#undef DIRECT
#undef LAUNCH
}

hipError_t launch_score(int bucket, int dtype, const void* X, int64_t n, int64_t ld, int p,
                        const double* mu, const double* M, int ldm, double cut, double* dist,
                        uint8_t* flag, hipStream_t s) {
  if (ldm != p) return hipErrorInvalidValue;   // the factor is p x p, row stride p
  if (n <= 0) return hipSuccess;
  // one row per thread, 256 rows per block
  const int64_t nbd = (n + DROWS - 1) / DROWS;
  const bool dense = rows_dense_at(X, ld, p, dtype, bucket);
#define LAUNCH(T, PB, GEN)                                                                      \
  hipLaunchKernelGGL((k_score_direct<T, PB, GEN>), dim3((unsigned)nbd), dim3(DROWS), 0, s,      \
                     static_cast<const T*>(X), n, ld, p, mu, M, cut, dist, flag)
#define CASE(PB)                                                                                \
  case PB:                                                                                      \
    if (dtype == 0) {                                                                           \
      if (dense) LAUNCH(float, PB, false);                                                      \
      else LAUNCH(float, PB, true);                                                             \
    } else {                                                                                    \
      if (dense) LAUNCH(double, PB, false);                                                     \
      else LAUNCH(double, PB, true);                                                            \
    }                                                                                           \
    return hipGetLastError();
  switch (bucket) {
    RTD_DIRECT_BUCKETS(CASE)
    default: return hipErrorInvalidValue;
  }
#undef CASE
#undef LAUNCH
}

}  // namespace rtd
