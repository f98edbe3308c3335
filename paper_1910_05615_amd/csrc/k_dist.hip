// Statistical distances (Sec. 2.1 eq. statdist computed as in Sec. 3.4):
// d2 = ||M (x - mu)||^2 with M the inverse Cholesky factor (folded with the
// standardisation scales inside the fit).  An item whose form word is 1
// holds instead the explicit inverse P of its scatter, packed like M as a
// lower triangle with doubled off-diagonal entries (P~), and
// d2 = sum_i r_i (P~ r)_i = r^T P r: the distance computation that Sec. 3.4
// replaces (Table 1, version I), and the form the single-swap update of
// Sec. 3.5 produces.  Both forms cost p(p+1)/2 multiply-adds per row.
//
// Up to p = 40 every thread reads its own row straight into registers (16-
// or 8-byte loads when the row size and base allow, else one load per
// element), and each block takes one 256-row slice, so no LDS, no barrier
// and a full chip of short blocks.  The factor and the centre are read at
// uniform offsets: the loads go through the scalar unit and every FMA takes
// its M entry from scalar registers.  The factor is evaluated column by
// column (y_i += M_ij z_j over j, the p partial sums independent of one
// another, each still summed in order of j).  The C-step runs it over both
// starts' items of a block (each row read twice: still faster than one read
// feeding two factors).  Rows of p = 48, 64 stream through LDS in chunks
// loaded with 16-byte coalesced loads, the factors staged in LDS and read as
// broadcasts, both starts of a block from one read of each row.
#include <stdint.h>

#include "common.h"
#include "fitk.h"
#include "rowload.h"

namespace rtd {

namespace {

constexpr int CH = 256;   // threads per block

template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  using type = float4;
};
template <>
struct Vec16<double> {
  using type = double2;
};

template <typename T, int P>
struct Shape {
  static constexpr int PP = P + 1;                    // LDS pitch (odd)
  // Two rows per thread would halve the broadcast reads of M, but hipcc then
  // spills at p = 20 (measured): one row per thread.
  static constexpr int R = 1;
  static constexpr int CHR = R * CH;                  // rows per chunk
  static constexpr bool ON = (size_t)PP * sizeof(T) * CHR <= 65536;
  static constexpr int XS = ON ? PP * CHR : 1;
  static constexpr bool PIPE = R == 1;                // next chunk's loads overlap compute
};

// Generic staging of n rows (pp used columns, stride ld) into xs.
template <typename T, int P>
__device__ inline void stage_chunk(const T* __restrict__ X, int64_t ld, int pp, int64_t rc,
                                   int n, T* __restrict__ xs) {
  constexpr int PP = Shape<T, P>::PP;
  const T* __restrict__ src = X + rc * ld;
  for (int e = threadIdx.x; e < n * pp; e += CH) {
    const int r = e / pp;
    const int j = e - r * pp;
    xs[r * PP + j] = src[(int64_t)r * ld + j];
  }
}

// M (row stride ldm, p x p used) packed and zero-padded into LDS, and mu.
template <int P>
__device__ inline void stage_factor(const double* __restrict__ M, int ldm,
                                    const double* __restrict__ mu, int p,
                                    double* __restrict__ Ml, double* __restrict__ mul) {
  for (int e = threadIdx.x; e < P * (P + 1) / 2; e += CH) {
    int i = 0, k = e;
    while (k > i) { k -= i + 1; ++i; }
    Ml[e] = (i < p && k < p) ? M[i * ldm + k] : 0.0;
  }
  for (int j = threadIdx.x; j < P; j += CH) mul[j] = j < p ? mu[j] : 0.0;
}

// ||M z||^2 (INV: z^T (M z), M = P~) for R rows at once, M packed lower
// triangular in LDS (one LDS read of an entry feeds R FMAs).
template <int P, int R, bool INV>
__device__ inline void tri_norm2_r(const double* __restrict__ Ml, const double (&z)[R][P],
                                   double (&acc)[R]) {
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.0;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    double y[R];
#pragma unroll
    for (int r = 0; r < R; ++r) y[r] = 0.0;
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      const double mij = Ml[i * (i + 1) / 2 + j];
#pragma unroll
      for (int r = 0; r < R; ++r) y[r] = fma(mij, z[r][j], y[r]);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = fma(y[r], INV ? z[r][i] : y[r], acc[r]);
  }
}

// ||M z||^2 (INV: z^T (M z)) with M read from global memory at uniform,
// compile-time offsets (row stride LDM): the loads go through the scalar unit
// and every FMA takes its M entry from SGPRs.
template <int P, bool INV>
__device__ inline double tri_norm2_g(const double* __restrict__ Mg, int ldm, int p,
                                     const double (&z)[P]) {
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    if (i < p) {
      const double* __restrict__ mr = Mg + i * ldm;
      double y = 0.0;
#pragma unroll
      for (int j = 0; j <= i; ++j) y = fma(mr[j], z[j], y);
      acc = fma(y, INV ? z[i] : y, acc);
    }
  }
  return acc;
}

template <int P, bool INV>
__device__ inline double tri_norm2_l(const double* __restrict__ Ml, const double (&z)[P]) {
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    double y = 0.0;
#pragma unroll
    for (int j = 0; j <= i; ++j) y = fma(Ml[i * (i + 1) / 2 + j], z[j], y);
    acc = fma(y, INV ? z[i] : y, acc);
  }
  return acc;
}

// Evaluate rows [r0, r1) of X against NI factors; emit(q, row, d2).
// Mg[q], mug[q]: factor (row stride ldm) and centre in global memory;
// inv[q]: the factor is P~ (explicit inverse) rather than L^{-1}.
template <typename T, int P, int NI, typename Emit>
__device__ inline void dist_rows(const T* __restrict__ X, int64_t ld, int p, int ldm, int64_t r0,
                                 int64_t r1, const double* const (&Mg)[NI],
                                 const double* const (&mug)[NI], const bool (&inv)[NI],
                                 double* Ml, double* mul, T* xs, Emit emit) {
  using S = Shape<T, P>;
  const int tid = threadIdx.x;
  const bool fast = p == P && ld == P && ((reinterpret_cast<uintptr_t>(X) & 15) == 0);
#pragma unroll
  for (int q = 0; q < NI; ++q)
    stage_factor<P>(Mg[q], ldm, mug[q], p, Ml + q * (P * (P + 1) / 2), mul + q * P);
  if constexpr (S::ON) {
    if (fast) {
      using V = typename Vec16<T>::type;
      constexpr int VN = 16 / sizeof(T);
      constexpr int NV = (S::R * P + VN - 1) / VN;   // vectors per thread per full chunk
      V buf[NV];
      auto issue = [&](int64_t rc, int n) {
        const V* __restrict__ s4 = reinterpret_cast<const V*>(X + rc * P);
        const int nv = (n * P) / VN;
#pragma unroll
        for (int u = 0; u < NV; ++u) {
          const int k = tid + u * CH;
          if (k < nv) buf[u] = s4[k];
        }
      };
      auto commit = [&](int64_t rc, int n) {
        const int nv = (n * P) / VN;
#pragma unroll
        for (int u = 0; u < NV; ++u) {
          const int k = tid + u * CH;
          if (k < nv) {
            const T* vv = reinterpret_cast<const T*>(&buf[u]);
#pragma unroll
            for (int c = 0; c < VN; ++c) {
              const int e = k * VN + c;
              const int r = e / P;
              xs[r * S::PP + (e - r * P)] = vv[c];
            }
          }
        }
        for (int e = nv * VN + tid; e < n * P; e += CH) {
          const int r = e / P;
          xs[r * S::PP + (e - r * P)] = X[rc * P + e];
        }
      };
      int n = (int)min((int64_t)S::CHR, r1 - r0);
      if (S::PIPE && r0 < r1) issue(r0, n);
      for (int64_t rc = r0; rc < r1; rc += S::CHR) {
        if (!S::PIPE) issue(rc, n);
        commit(rc, n);
        const int64_t rn = rc + S::CHR;
        const int nn = rn < r1 ? (int)min((int64_t)S::CHR, r1 - rn) : 0;
        if (S::PIPE && nn > 0) issue(rn, nn);
        __syncthreads();
        if (tid < n) {
#pragma unroll
          for (int q = 0; q < NI; ++q) {
            double z[S::R][P];
#pragma unroll
            for (int r = 0; r < S::R; ++r)
#pragma unroll
              for (int j = 0; j < P; ++j)
                z[r][j] = (double)xs[(tid + r * CH) * S::PP + j] - mul[q * P + j];
            double acc[S::R];
            if constexpr (NI == 1 && S::R == 1) {
              acc[0] = inv[q] ? tri_norm2_g<P, true>(Mg[q], ldm, p, z[0])
                              : tri_norm2_g<P, false>(Mg[q], ldm, p, z[0]);
            } else if (inv[q]) {
              tri_norm2_r<P, S::R, true>(Ml + q * (P * (P + 1) / 2), z, acc);
            } else {
              tri_norm2_r<P, S::R, false>(Ml + q * (P * (P + 1) / 2), z, acc);
            }
#pragma unroll
            for (int r = 0; r < S::R; ++r)
              if (tid + r * CH < n) emit(q, rc + tid + r * CH, acc[r]);
          }
        }
        __syncthreads();
        n = nn;
      }
      return;
    }
  }
  // generic path (rows of another width or stride)
  if constexpr (S::ON) {
    for (int e = tid; e < S::XS; e += CH) xs[e] = (T)0;   // padding columns stay zero
    __syncthreads();
    for (int64_t rc = r0; rc < r1; rc += CH) {
      const int n = (int)min((int64_t)CH, r1 - rc);
      stage_chunk<T, P>(X, ld, p, rc, n, xs);
      __syncthreads();
      if (tid < n) {
#pragma unroll
        for (int q = 0; q < NI; ++q) {
          double z[P];
#pragma unroll
          for (int j = 0; j < P; ++j) z[j] = (double)xs[tid * S::PP + j] - mul[q * P + j];
          const double* Mq = Ml + q * (P * (P + 1) / 2);
          emit(q, rc + tid, inv[q] ? tri_norm2_l<P, true>(Mq, z) : tri_norm2_l<P, false>(Mq, z));
        }
      }
      __syncthreads();
    }
  } else {
    __syncthreads();
    for (int64_t r = r0 + tid; r < r1; r += CH) {
      const T* __restrict__ xr = X + r * ld;
#pragma unroll
      for (int q = 0; q < NI; ++q) {
        double z[P];
#pragma unroll
        for (int j = 0; j < P; ++j) z[j] = (j < p ? (double)xr[j] : 0.0) - mul[q * P + j];
        const double* Mq = Ml + q * (P * (P + 1) / 2);
        emit(q, r, inv[q] ? tri_norm2_l<P, true>(Mq, z) : tri_norm2_l<P, false>(Mq, z));
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Direct row evaluation (p <= 40).

constexpr int DROWS = 256;     // rows per block of the direct kernels
constexpr int DIRECT_MAX = 40; // widest bucket evaluated directly

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

template <typename T, int P, int NI, bool INV, typename Emit>
__device__ inline void eval_row(T (&v)[P], int p, int ldm, const double* const (&Mg)[NI],
                                const double* const (&mug)[NI], const bool (&act)[NI],
                                Emit emit) {
  // the factors one after the other on the same row, each column by column;
  // between them the row goes through all_loaded again, so that its float64
  // conversions are not kept live from the first factor to the second (the
  // launches use one factor: see dist_pairs_pay)
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

// ---------------------------------------------------------------------------
// Staged evaluation (p = 48, 64).

// C-step distances.  NI = 2: tile.item and tile.item + 1 are the two starts of
// one block (same rows); an inactive start is skipped.
template <typename T, int P, int NI>
__global__ __launch_bounds__(CH) void k_dist(const ItemDesc* __restrict__ items,
                                             const Tile* __restrict__ tiles, int tile_rows,
                                             const double* __restrict__ mtri,
                                             const double* __restrict__ mux,
                                             const int32_t* __restrict__ status,
                                             const int32_t* __restrict__ form,
                                             double* __restrict__ d2) {
  __shared__ double Ml[NI * P * (P + 1) / 2];
  __shared__ double mul[NI * P];
  __shared__ T xs[Shape<T, P>::XS];
  const Tile tl = tiles[blockIdx.x];
  bool act[NI];
  bool any = false;
#pragma unroll
  for (int q = 0; q < NI; ++q) {
    act[q] = status == nullptr || status[tl.item + q] == ACTIVE;
    any = any || act[q];
  }
  if (!any) return;
  const ItemDesc D = items[tl.item];
  int64_t roff[NI];
  const double* Mg[NI];
  const double* mug[NI];
  bool inv[NI];
#pragma unroll
  for (int q = 0; q < NI; ++q) {
    const int it = tl.item + q;
    roff[q] = items[it].roff;
    Mg[q] = mtri + (size_t)it * MSTRIDE;
    mug[q] = mux + (size_t)it * PMAX;
    inv[q] = form != nullptr && form[it] != 0;
  }
  const int64_t r0 = (int64_t)tl.t * tile_rows;
  const int64_t r1 = min(r0 + (int64_t)tile_rows, D.m);
  const T* __restrict__ X = static_cast<const T*>(D.X) + D.row0 * D.ld;
  dist_rows<T, P, NI>(X, D.ld, D.p, PMAX, r0, r1, Mg, mug, inv, Ml, mul, xs,
                            [&](int q, int64_t r, double v) {
                              if (act[q]) d2[roff[q] + r] = v;
                            });
}

// Final robust distances and flags of the fit (Sec. 4 step 10).
template <typename T, int P>
__global__ __launch_bounds__(CH) void k_final_dist(const ItemDesc* __restrict__ items,
                                                   const Tile* __restrict__ tiles, int tile_rows,
                                                   const double* __restrict__ mtri,
                                                   const double* __restrict__ mux,
                                                   const int32_t* __restrict__ form,
                                                   const double* __restrict__ d2,
                                                   const DsInfo* __restrict__ ds,
                                                   const rtdetmcd_out* __restrict__ outs) {
  __shared__ double Ml[P * (P + 1) / 2];
  __shared__ double mul[P];
  __shared__ T xs[Shape<T, P>::XS];
  const Tile tl = tiles[blockIdx.x];
  const int it = tl.item;
  const ItemDesc D = items[it];
  const DsInfo dd = ds[D.ds];
  if (dd.err) return;
  const double cut = dd.chi2p;
  double* __restrict__ od = outs[D.ds].dist;
  uint8_t* __restrict__ of = outs[D.ds].outlier;
  uint8_t* __restrict__ ow = outs[D.ds].rew_mask;
  // reweighting set: fitted rows whose distance under the raw fit (the
  // dataset's first global item) is within the cutoff
  const ItemDesc R = items[dd.glob0];
  const double* __restrict__ d2r = d2 + R.roff;
  const int64_t r0 = (int64_t)tl.t * tile_rows;
  const int64_t r1 = min(r0 + (int64_t)tile_rows, D.m);
  const T* __restrict__ X = static_cast<const T*>(D.X) + D.row0 * D.ld;
  const double* Mg[1] = {mtri + (size_t)it * MSTRIDE};
  const double* mug[1] = {mux + (size_t)it * PMAX};
  const bool inv[1] = {form != nullptr && form[it] != 0};
  dist_rows<T, P, 1>(X, D.ld, D.p, PMAX, r0, r1, Mg, mug, inv, Ml, mul, xs,
                           [&](int, int64_t r, double v) {
                             if (od) od[D.row0 + r] = sqrt(v);
                             if (of) of[D.row0 + r] = v > cut ? 1 : 0;
                             if (ow) {
                               // position of the row among the fitted rows (through the inverse
      // permutation for a random partition)
      const int64_t rr = dd.inv ? (int64_t)dd.inv[D.row0 + r] : D.row0 + r - R.row0;
                               ow[D.row0 + r] = (rr >= 0 && rr < R.m && d2r[rr] <= cut) ? 1 : 0;
                             }
                           });
}

// Scoring against a stored fit: M row-major p x p (inverse Cholesky factor).
template <typename T, int P>
__global__ __launch_bounds__(CH) void k_score(const T* __restrict__ X, int64_t n, int64_t ld,
                                              int p, const double* __restrict__ mu,
                                              const double* __restrict__ M, double cut,
                                              int tile_rows, double* __restrict__ dist,
                                              uint8_t* __restrict__ flag) {
  __shared__ double Ml[P * (P + 1) / 2];
  __shared__ double mul[P];
  __shared__ T xs[Shape<T, P>::XS];
  const int64_t r0 = (int64_t)blockIdx.x * tile_rows;
  const int64_t r1 = min(r0 + (int64_t)tile_rows, n);
  const double* Mg[1] = {M};
  const double* mug[1] = {mu};
  const bool inv[1] = {false};
  dist_rows<T, P, 1>(X, ld, p, p, r0, r1, Mg, mug, inv, Ml, mul, xs,
                        [&](int, int64_t r, double v) {
                          if (dist) dist[r] = sqrt(v);
                          if (flag) flag[r] = v > cut ? 1 : 0;
                        });
}

}  // namespace

#define RTD_DIRECT_BUCKETS(X) X(4) X(5) X(8) X(10) X(16) X(20) X(24) X(32) X(40)
#define RTD_STAGED_BUCKETS(X) X(48) X(64)
static_assert(DIRECT_MAX == 40, "bucket lists");

hipError_t launch_dist(int bucket, int dtype, int dense, int ipt, const ItemDesc* items,
                       const Tile* tiles,
                       int ntiles, int tile_rows, const double* mtri, const double* mux,
                       const int32_t* status, const int32_t* form, double* d2, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (tile_rows <= 0 || tile_rows % DROWS != 0) return hipErrorInvalidValue;
  const unsigned nbd = (unsigned)ntiles * (unsigned)(tile_rows / DROWS);
#define LAUNCH(K, NB, NT)                                                                       \
  hipLaunchKernelGGL(K, dim3(NB), dim3(NT), 0, s, items, tiles, tile_rows, mtri, mux, status, \
                     form, d2)
#define DIRECT(T, PB, NI)                                                                       \
  do {                                                                                          \
    if (dense && !form) LAUNCH((k_dist_direct<T, PB, NI, false, false>), nbd, DROWS);           \
    else if (dense) LAUNCH((k_dist_direct<T, PB, NI, false, true>), nbd, DROWS);                \
    else LAUNCH((k_dist_direct<T, PB, NI, true, true>), nbd, DROWS);                            \
  } while (0)
#define STAGED(T, PB, NI) LAUNCH((k_dist<T, PB, NI>), ntiles, CH)
#define CASE(K1, K2, PB)                                                                        \
  case PB:                                                                                      \
    if (dtype == 0) {                                                                           \
      if (ipt == 2) K2(float, PB, 2);                                                           \
      else K1(float, PB, 1);                                                                    \
    } else {                                                                                    \
      if (ipt == 2) K2(double, PB, 2);                                                          \
      else K1(double, PB, 1);                                                                   \
    }                                                                                           \
    return hipGetLastError();
  // pairs (ipt = 2) exist for the staged buckets only (dist_pairs_pay): the
  // direct buckets run one factor per launch, and a pair launch of one of
  // them is an invalid request
#define NOPAIR(T, PB, NI) return hipErrorInvalidValue
#define DCASE(PB) CASE(DIRECT, NOPAIR, PB)
#define SCASE(PB) CASE(STAGED, STAGED, PB)
  switch (bucket) {
    RTD_DIRECT_BUCKETS(DCASE)
    RTD_STAGED_BUCKETS(SCASE)
    default: return hipErrorInvalidValue;
  }
#undef SCASE
#undef DCASE
#undef NOPAIR
#undef CASE
#undef STAGED
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
#define LAUNCH(K, NB, NT)                                                                       \
  hipLaunchKernelGGL(K, dim3(NB), dim3(NT), 0, s, items, tiles, tile_rows, mtri, mux, form, d2, \
                     ds, outs)
#define DIRECT(T, PB)                                                                           \
  do {                                                                                          \
    if (dense && !form) LAUNCH((k_final_dist_direct<T, PB, false, false>), nbd, DROWS);         \
    else if (dense) LAUNCH((k_final_dist_direct<T, PB, false, true>), nbd, DROWS);              \
    else LAUNCH((k_final_dist_direct<T, PB, true, true>), nbd, DROWS);                          \
  } while (0)
#define STAGED(T, PB) LAUNCH((k_final_dist<T, PB>), ntiles, CH)
#define CASE(K, PB)                                                                             \
  case PB:                                                                                      \
    if (dtype == 0) K(float, PB);                                                               \
    else K(double, PB);                                                                         \
    return hipGetLastError();
#define DCASE(PB) CASE(DIRECT, PB)
#define SCASE(PB) CASE(STAGED, PB)
  switch (bucket) {
    RTD_DIRECT_BUCKETS(DCASE)
    RTD_STAGED_BUCKETS(SCASE)
    default: return hipErrorInvalidValue;
  }
#undef SCASE
#undef DCASE
#undef CASE
#undef STAGED
#undef DIRECT
#undef LAUNCH
}

hipError_t launch_score(int bucket, int dtype, const void* X, int64_t n, int64_t ld, int p,
                        const double* mu, const double* M, int ldm, double cut, double* dist,
                        uint8_t* flag, hipStream_t s) {
  if (ldm != p) return hipErrorInvalidValue;   // the factor is p x p, row stride p
  if (n <= 0) return hipSuccess;
  // direct buckets: one row per thread, 256 rows per block; the staged
  // buckets take 2,048-row tiles (fewer stagings of the wide factor)
  const int64_t nbd = (n + DROWS - 1) / DROWS;
  const int64_t nbs = (n + 2047) / 2048;
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
#define SCASE(PB)                                                                               \
  case PB:                                                                                      \
    if (dtype == 0)                                                                             \
      hipLaunchKernelGGL((k_score<float, PB>), dim3((unsigned)nbs), dim3(CH), 0, s,             \
                         static_cast<const float*>(X), n, ld, p, mu, M, cut, 2048, dist, flag); \
    else                                                                                        \
      hipLaunchKernelGGL((k_score<double, PB>), dim3((unsigned)nbs), dim3(CH), 0, s,            \
                         static_cast<const double*>(X), n, ld, p, mu, M, cut, 2048, dist,       \
                         flag);                                                                 \
    return hipGetLastError();
  switch (bucket) {
    RTD_DIRECT_BUCKETS(CASE)
    RTD_STAGED_BUCKETS(SCASE)
    default: return hipErrorInvalidValue;
  }
#undef SCASE
#undef CASE
#undef LAUNCH
}

}  // namespace rtd
