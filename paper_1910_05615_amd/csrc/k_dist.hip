// Statistical distances (Sec. 2.1 eq. statdist computed as in Sec. 3.4):
// d2 = ||M (x - mu)||^2 with M the inverse Cholesky factor (folded with the
// standardisation scales inside the fit).
//
// Rows stream through LDS in chunks loaded with 16-byte coalesced loads, the
// next chunk's loads in flight while the current one is evaluated in
// float64.  With one factor per launch (scoring, final distances) M is read
// from global memory at uniform offsets, so the loads go through the scalar
// unit and each FMA takes its entry from SGPRs; the C-step variant, which
// evaluates the two starts of a block from one read of each row, stages both
// factors (packed, zero-padded to the p-bucket) in LDS and reads them as
// broadcasts (two factors in SGPRs measured slower).  mu is staged in LDS.
#include <stdint.h>

#include "common.h"
#include "fitk.h"

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

// ||M z||^2 for R rows at once, M packed lower triangular in LDS (one LDS
// read of an entry feeds R FMAs).
template <int P, int R>
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
    for (int r = 0; r < R; ++r) acc[r] = fma(y[r], y[r], acc[r]);
  }
}

// ||M z||^2 with M read from global memory at uniform, compile-time offsets
// (row stride LDM): the loads go through the scalar unit and every FMA takes
// its M entry from SGPRs.
template <int P>
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
      acc = fma(y, y, acc);
    }
  }
  return acc;
}

template <int P>
__device__ inline double tri_norm2_l(const double* __restrict__ Ml, const double (&z)[P]) {
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    double y = 0.0;
#pragma unroll
    for (int j = 0; j <= i; ++j) y = fma(Ml[i * (i + 1) / 2 + j], z[j], y);
    acc = fma(y, y, acc);
  }
  return acc;
}

// Evaluate rows [r0, r1) of X against NI factors; emit(q, row, d2).
// Mg[q], mug[q]: factor (row stride ldm) and centre in global memory.
template <typename T, int P, int NI, typename Emit>
__device__ inline void dist_rows(const T* __restrict__ X, int64_t ld, int p, int ldm, int64_t r0,
                                 int64_t r1, const double* const (&Mg)[NI],
                                 const double* const (&mug)[NI], double* Ml, double* mul,
                                 T* xs, Emit emit) {
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
            if constexpr (NI == 1 && S::R == 1) acc[0] = tri_norm2_g<P>(Mg[q], ldm, p, z[0]);
            else tri_norm2_r<P, S::R>(Ml + q * (P * (P + 1) / 2), z, acc);
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
          emit(q, rc + tid, tri_norm2_l<P>(Ml + q * (P * (P + 1) / 2), z));
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
        emit(q, r, tri_norm2_l<P>(Ml + q * (P * (P + 1) / 2), z));
      }
    }
  }
}

// C-step distances.  NI = 2: tile.item and tile.item + 1 are the two starts of
// one block (same rows); an inactive start is skipped.
template <typename T, int P, int NI>
__global__ __launch_bounds__(CH) void k_dist(const ItemDesc* __restrict__ items,
                                             const Tile* __restrict__ tiles, int tile_rows,
                                             const double* __restrict__ mtri,
                                             const double* __restrict__ mux,
                                             const int32_t* __restrict__ status,
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
#pragma unroll
  for (int q = 0; q < NI; ++q) {
    const int it = tl.item + q;
    roff[q] = items[it].roff;
    Mg[q] = mtri + (size_t)it * MSTRIDE;
    mug[q] = mux + (size_t)it * PMAX;
  }
  const int64_t r0 = (int64_t)tl.t * tile_rows;
  const int64_t r1 = min(r0 + (int64_t)tile_rows, D.m);
  const T* __restrict__ X = static_cast<const T*>(D.X) + D.row0 * D.ld;
  dist_rows<T, P, NI>(X, D.ld, D.p, PMAX, r0, r1, Mg, mug, Ml, mul, xs,
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
  dist_rows<T, P, 1>(X, D.ld, D.p, PMAX, r0, r1, Mg, mug, Ml, mul, xs,
                           [&](int, int64_t r, double v) {
                             if (od) od[D.row0 + r] = sqrt(v);
                             if (of) of[D.row0 + r] = v > cut ? 1 : 0;
                             if (ow) {
                               const int64_t rr = D.row0 + r - R.row0;
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
  dist_rows<T, P, 1>(X, ld, p, p, r0, r1, Mg, mug, Ml, mul, xs,
                        [&](int, int64_t r, double v) {
                          if (dist) dist[r] = sqrt(v);
                          if (flag) flag[r] = v > cut ? 1 : 0;
                        });
}

}  // namespace

#define RTD_BUCKETS(X) X(4) X(5) X(8) X(10) X(16) X(20) X(24) X(32) X(40) X(48) X(64)

hipError_t launch_dist(int bucket, int dtype, int ipt, const ItemDesc* items, const Tile* tiles,
                       int ntiles, int tile_rows, const double* mtri, const double* mux,
                       const int32_t* status, double* d2, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
#define LAUNCH(T, PB, NI)                                                                       \
  hipLaunchKernelGGL((k_dist<T, PB, NI>), dim3(ntiles), dim3(CH), 0, s, items, tiles, tile_rows, \
                     mtri, mux, status, d2)
#define CASE(PB)                                                                                \
  case PB:                                                                                      \
    if (dtype == 0) {                                                                           \
      if (ipt == 2) LAUNCH(float, PB, 2);                                                       \
      else LAUNCH(float, PB, 1);                                                                \
    } else {                                                                                    \
      if (ipt == 2) LAUNCH(double, PB, 2);                                                      \
      else LAUNCH(double, PB, 1);                                                               \
    }                                                                                           \
    return hipGetLastError();
  switch (bucket) {
    RTD_BUCKETS(CASE)
    default: return hipErrorInvalidValue;
  }
#undef CASE
#undef LAUNCH
}

hipError_t launch_final_dist(int bucket, int dtype, const ItemDesc* items, const Tile* tiles,
                             int ntiles, int tile_rows, const double* mtri, const double* mux,
                             const double* d2, const DsInfo* ds, const rtdetmcd_out* outs,
                             hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
#define CASE(PB)                                                                                \
  case PB:                                                                                      \
    if (dtype == 0)                                                                             \
      hipLaunchKernelGGL((k_final_dist<float, PB>), dim3(ntiles), dim3(CH), 0, s, items, tiles, \
                         tile_rows, mtri, mux, d2, ds, outs);                                   \
    else                                                                                        \
      hipLaunchKernelGGL((k_final_dist<double, PB>), dim3(ntiles), dim3(CH), 0, s, items,       \
                         tiles, tile_rows, mtri, mux, d2, ds, outs);                            \
    return hipGetLastError();
  switch (bucket) {
    RTD_BUCKETS(CASE)
    default: return hipErrorInvalidValue;
  }
#undef CASE
}

hipError_t launch_score(int bucket, int dtype, const void* X, int64_t n, int64_t ld, int p,
                        const double* mu, const double* M, int ldm, double cut, double* dist,
                        uint8_t* flag, hipStream_t s) {
  if (ldm != p) return hipErrorInvalidValue;   // the factor is p x p, row stride p
  // one 256-row chunk per block keeps the most loads in flight for narrow
  // rows (1M x 20: 21 us against 29 us with 2,048-row tiles); wide factors
  // are cheaper to stage in fewer, longer blocks (10M x 40: 675 against 760)
  const int tile_rows = bucket <= 24 ? 256 : 2048;
  const int64_t nb = (n + tile_rows - 1) / tile_rows;
  if (nb <= 0) return hipSuccess;
#define CASE(PB)                                                                                \
  case PB:                                                                                      \
    if (dtype == 0)                                                                             \
      hipLaunchKernelGGL((k_score<float, PB>), dim3((unsigned)nb), dim3(CH), 0, s,              \
                         static_cast<const float*>(X), n, ld, p, mu, M, cut, tile_rows, dist,   \
                         flag);                                                                 \
    else                                                                                        \
      hipLaunchKernelGGL((k_score<double, PB>), dim3((unsigned)nb), dim3(CH), 0, s,             \
                         static_cast<const double*>(X), n, ld, p, mu, M, cut, tile_rows, dist,  \
                         flag);                                                                 \
    return hipGetLastError();
  switch (bucket) {
    RTD_BUCKETS(CASE)
    default: return hipErrorInvalidValue;
  }
#undef CASE
}

}  // namespace rtd
