// Kernels of the full RT-DetMCD fit around the C-step loop: standardisation
// keys, projections for the initial estimators and the refinement, the small
// per-block float64 steps, robust aggregation and reweighting.
#include "../../include/rtdetmcd.h"
#include "fitk.h"
#include "rowload.h"
#include "wave.h"

namespace rtd {

namespace {

__device__ inline uint32_t fkey32(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline uint64_t fkey64(double f) {
  const uint64_t u = (uint64_t)__double_as_longlong(f);
  return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}


// ------------------------------------------------------------ standardisation

// Column-major order keys of the columns of X: a tile of CK_ROWS rows is read
// row by row (contiguous when ld == p), turned into keys in LDS and written
// column by column, so that both sides are coalesced.
constexpr int CK_ROWS = COLKEY_ROWS;
constexpr int CK_NT = 256;

template <typename T, typename K>
__global__ __launch_bounds__(CK_NT) void k_colkeys(const ColJob* __restrict__ jobs, int njobs) {
  __shared__ K tile[CK_ROWS * (PMAX + 1)];   // row-major, row stride p + 1
  // this block's dataset: the last job whose first tile is <= blockIdx.x
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (jobs[mid].tile0 <= (int64_t)blockIdx.x) lo = mid;
    else hi = mid - 1;
  }
  const ColJob J = jobs[lo];
  const T* __restrict__ X = static_cast<const T*>(J.X);
  K* __restrict__ keys = static_cast<K*>(J.keys);
  const int64_t n = J.n, ld = J.ld;
  const int p = J.p;
  const int64_t r0 = ((int64_t)blockIdx.x - J.tile0) * CK_ROWS;
  const int nr = (int)min((int64_t)CK_ROWS, n - r0);
  const int pp = p + 1, tid = threadIdx.x;
  {
    int i = tid / p, j = tid - (tid / p) * p;
    const int di = CK_NT / p, dj = CK_NT - (CK_NT / p) * p;
    const T* __restrict__ xb = X + r0 * ld;
    bool finite = true;   // every value of X passes through here once
    for (int e = tid; e < nr * p; e += CK_NT) {
      const T x = xb[(int64_t)i * ld + j];
      finite = finite && isfinite(x);
      if constexpr (sizeof(K) == 4) tile[i * pp + j] = fkey32((float)x);
      else tile[i * pp + j] = fkey64((double)x);
      i += di;
      j += dj;
      if (j >= p) {
        j -= p;
        ++i;
      }
    }
    if (!finite) *J.err = RTDETMCD_ENONFINITE;
  }
  __syncthreads();
  for (int e = tid; e < p * CK_ROWS; e += CK_NT) {
    const int j = e / CK_ROWS, i = e % CK_ROWS;
    if (i < nr) keys[(size_t)j * n + r0 + i] = tile[i * pp + j];
  }
}

__global__ void k_std_finish(const SegStat* __restrict__ st32, const SegStat* __restrict__ st64,
                             const int32_t* __restrict__ seg0, const int32_t* __restrict__ in64,
                             int D, DsInfo* __restrict__ ds, FitArrays F) {
  const int d = blockIdx.x;
  if (d >= D) return;
  const int p = ds[d].p;
  const SegStat* __restrict__ st = in64[d] ? st64 : st32;
  for (int j = threadIdx.x; j < PMAX; j += blockDim.x) {
    double loc = 0.0, sc = 1.0;
    if (j < p) {
      const SegStat s = st[seg0[d] + j];
      loc = s.mu;
      sc = sqrt(s.var);
      if (!(sc > 0.0) || !(sc < 1e300) || !(fabs(loc) < 1e300)) {
        if (ds[d].err == 0) ds[d].err = RTDETMCD_ESINGULAR;   // keep an earlier ENONFINITE
        loc = 0.0;
        sc = 1.0;
      }
    }
    F.loc[(size_t)d * PMAX + j] = loc;
    F.scale[(size_t)d * PMAX + j] = sc;
  }
}

// ------------------------------------------------------------ projections
// MODE 0: v_j = sum_k W_jk z_k for j < p, one key segment per j (refinement:
//         W = V^T gives the scores T = Z V, W = Sigma^{-1/2} the sphered data).
// MODE 1: v = ||z|| (GSSCM norms), one segment.
// z = (x - loc) / scale, the standardised row (Sec. 3.1, Sec. 4 eq. standardization).
// One row per thread, 256 rows per block (tile_rows / 256 blocks per tile):
// the row's loads all issued before its arithmetic, loc and scale read at
// uniform offsets (scalar unit).
constexpr int PROJ_ROWS = 256;
template <typename T, int P, int MODE>
__global__ __launch_bounds__(PROJ_ROWS) void k_project(const ItemDesc* __restrict__ items,
                                                       const Tile* __restrict__ tiles,
                                                       int tile_rows,
                                                       const int32_t* __restrict__ status,
                                                       const double* __restrict__ W,
                                                       const int64_t* __restrict__ kbase,
                                                       uint64_t* __restrict__ keys) {
  const int nsub = tile_rows / PROJ_ROWS;
  const Tile tl = tiles[blockIdx.x / nsub];
  const int it = tl.item;
  if (status != nullptr && status[it] != ACTIVE) return;
  const ItemDesc D = items[it];
  const int64_t t0 = (int64_t)tl.t * tile_rows;
  const int64_t r = t0 + (int64_t)(blockIdx.x % nsub) * PROJ_ROWS + threadIdx.x;
  if (r >= min(t0 + (int64_t)tile_rows, D.m)) return;
  const int p = D.p;
  const double* __restrict__ loc = D.loc;
  const double* __restrict__ sc = D.scale;
  const double* __restrict__ Wi = W + (size_t)it * MSTRIDE;
  uint64_t* __restrict__ ko = keys + kbase[it];
  const gptr_t<T> xr = as_global(static_cast<const T*>(D.X) + (D.row0 + r) * D.ld);
  T x[P];
#pragma unroll
  for (int k = 0; k < P; ++k) x[k] = k < p ? xr[k] : (T)0;
  all_loaded(x);
  double z[P];
#pragma unroll
  for (int k = 0; k < P; ++k) z[k] = (k < p) ? ((double)x[k] - loc[k]) / sc[k] : 0.0;
  if (MODE == 1) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < P; ++k) s = fma(z[k], z[k], s);
    ko[r] = fkey64(sqrt(s));
  } else {
#pragma unroll
    for (int j = 0; j < P; ++j) {
      if (j < p) {
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < P; ++k) v = fma(Wi[j * PMAX + k], z[k], v);
        ko[(size_t)j * D.m + r] = fkey64(v);
      }
    }
  }
}

// ------------------------------------------------------------ partial sums

__global__ __launch_bounds__(256) void k_reduce_partials(const ItemDesc* __restrict__ items,
                                                         const double* __restrict__ part,
                                                         int first, double* __restrict__ cnt,
                                                         double* __restrict__ sum,
                                                         double* __restrict__ S) {
  const int it = first + blockIdx.x;
  const ItemDesc D = items[it];
  const int p = D.p;
  for (int e = threadIdx.x; e < 1 + p + p * p; e += blockDim.x) {
    int idx;
    if (e == 0) idx = 0;
    else if (e <= p) idx = e;
    else {
      const int q = e - 1 - p, i = q / p, j = q % p;
      const int a = i >= j ? i : j, b = i >= j ? j : i;
      idx = 1 + PMAX + a * (a + 1) / 2 + b;
    }
    const double s = part[(size_t)D.tile0 * PSTRIDE + idx];   // collapsed partial
    if (e == 0) cnt[it] = s;
    else if (e <= p) sum[(size_t)it * PMAX + e - 1] = s;
    else {
      const int q = e - 1 - p;
      S[(size_t)it * MSTRIDE + (q / p) * PMAX + q % p] = s;
    }
  }
}

// mode 0: S1 = classical covariance of the wrapped rows (Sec. 3.2)
// mode 1: S2 = (1/m) sum xi^2 z z^T (eq. LR)
// mode 2: copy the GSSCM cutoffs (A, B) of each block
__global__ void k_init_cov(int mode, const ItemDesc* __restrict__ bitems, int first, FitArrays F,
                           ItemArrays C, const DsInfo* __restrict__ ds, double* __restrict__ cut,
                           const SegStat* __restrict__ gst) {
  const int b = first + blockIdx.x;
  const ItemDesc B = bitems[b];
  const DsInfo d = ds[B.ds];
  const int p = B.p;
  if (mode == 2) {
    if (threadIdx.x == 0) {
      cut[2 * b] = gst[b].mu;
      cut[2 * b + 1] = gst[b].var;
    }
    return;
  }
  const int ci = d.item0 + 2 * (b - d.blk0) + mode;
  const double m = (double)B.m;
  for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
    const int i = e / p, j = e % p;
    const double Sij = F.rS[(size_t)b * MSTRIDE + i * PMAX + j];
    double v;
    if (mode == 0) {
      const double si = F.rsum[(size_t)b * PMAX + i], sj = F.rsum[(size_t)b * PMAX + j];
      v = (Sij - si * sj / m) / (m - 1.0);
    } else {
      v = Sij / m;
    }
    C.sigz[(size_t)ci * MSTRIDE + i * PMAX + j] = v;
  }
}

// ------------------------------------------------------------ refinement (Sec. 3.3)

// Jacobi eigen-decomposition of the initial scatter of each item, one block
// per matrix; eigenvalues in decreasing order (step 1) and the condition check
// lambda_1 / lambda_p <= kappa_max (step 2).
// Parallel cyclic Jacobi on one wave per item: each step applies p/2
// disjoint rotations chosen by the round-robin (circle) ordering, as one
// column pass A J (V too) and one row pass J^T A; p - 1 steps make a sweep
// over all pairs.  A and V sit in LDS with an odd row stride; with a single
// wave the barriers between passes cost almost nothing.
template <int P>
__global__ __launch_bounds__(64) void k_eig(const ItemDesc* __restrict__ items, ItemArrays A,
                                            FitArrays F, int first, double kappa_max) {
  constexpr int LD = P + 1;
  constexpr int NPM = (P + 1) / 2;
  __shared__ double a[P * LD];
  __shared__ double v[P * LD];
  __shared__ double cs_c[NPM], cs_s[NPM];
  __shared__ int pi[NPM], pj[NPM];
  __shared__ int ord[P];
  const int it = first + blockIdx.x;
  if (A.status[it] != ACTIVE) return;
  const int p = items[it].p;          // p <= P
  const int lane = threadIdx.x;
  const double* S = A.sigz + (size_t)it * MSTRIDE;
  if (lane < p) {
    for (int j = 0; j < p; ++j) {
      a[lane * LD + j] = 0.5 * (S[lane * PMAX + j] + S[j * PMAX + lane]);
      v[lane * LD + j] = (lane == j) ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  const int np = (p + 1) & ~1;        // players, a dummy one when p is odd
  const int npair = np / 2;
  for (int sweep = 0; sweep < 60 && p > 1; ++sweep) {
    double off = 0.0, dia = 0.0;
    if (lane < p)
      for (int j = 0; j < p; ++j) {
        const double x = a[lane * LD + j];
        if (j != lane) off = fma(x, x, off);
        else dia = fma(x, x, dia);
      }
    off = wave_sum(off);
    dia = wave_sum(dia);
    // converged once the off-diagonal mass is about 1e-14 of the diagonal's
    // (the rounding floor of the rotations is near 1e-16 per entry, so a much
    // tighter bound may never be met); uniform: every lane holds the sums
    if (!(off > 1e-28 * dia)) break;
    for (int r = 0; r < np - 1; ++r) {
      if (lane < npair) {
        auto pl = [&](int q) { return q == 0 ? 0 : 1 + ((q - 1 + r) % (np - 1)); };
        int i = pl(lane), j = pl(np - 1 - lane);
        if (i > j) { const int t = i; i = j; j = t; }
        double c = 1.0, sn = 0.0;
        if (j < p) {
          const double apq = a[i * LD + j];
          if (apq != 0.0) {
            const double app = a[i * LD + i], aqq = a[j * LD + j];
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            sn = t * c;
          }
        }
        pi[lane] = i;
        pj[lane] = j < p ? j : i;   // a rotation with the dummy is the identity
        cs_c[lane] = c;
        cs_s[lane] = sn;
      }
      __syncthreads();
      // A pass updates p x npair independent (row, pair) elements; the 64
      // lanes take them four at a time (all loads first, then all stores:
      // the pairs of a step touch disjoint columns, and rows).
      const int ne = p * npair;
      const float inv_np = 1.0f / (float)npair;
      for (int e0 = 0; e0 < ne; e0 += 256) {   // columns: A <- A J, V <- V J
        int ri[4], ii[4], jj[4];
        double c[4], sn[4], xi[4], xj[4], yi[4], yj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = min(e0 + 64 * u + lane, ne - 1);
          const int r = (int)(((float)e + 0.5f) * inv_np), k = e - r * npair;
          ri[u] = r * LD;
          ii[u] = pi[k];
          jj[u] = pj[k];
          c[u] = cs_c[k];
          sn[u] = cs_s[k];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          xi[u] = a[ri[u] + ii[u]];
          xj[u] = a[ri[u] + jj[u]];
          yi[u] = v[ri[u] + ii[u]];
          yj[u] = v[ri[u] + jj[u]];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (e0 + 64 * u + lane < ne && ii[u] != jj[u]) {
            a[ri[u] + ii[u]] = c[u] * xi[u] - sn[u] * xj[u];
            a[ri[u] + jj[u]] = sn[u] * xi[u] + c[u] * xj[u];
            v[ri[u] + ii[u]] = c[u] * yi[u] - sn[u] * yj[u];
            v[ri[u] + jj[u]] = sn[u] * yi[u] + c[u] * yj[u];
          }
        }
      }
      __syncthreads();
      for (int e0 = 0; e0 < ne; e0 += 256) {   // rows: A <- J^T A
        int cl[4], ii[4], jj[4];
        double c[4], sn[4], xi[4], xj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = min(e0 + 64 * u + lane, ne - 1);
          const int cc = (int)(((float)e + 0.5f) * inv_np), k = e - cc * npair;
          cl[u] = cc;
          ii[u] = pi[k] * LD;
          jj[u] = pj[k] * LD;
          c[u] = cs_c[k];
          sn[u] = cs_s[k];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          xi[u] = a[ii[u] + cl[u]];
          xj[u] = a[jj[u] + cl[u]];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (e0 + 64 * u + lane < ne && ii[u] != jj[u]) {
            a[ii[u] + cl[u]] = c[u] * xi[u] - sn[u] * xj[u];
            a[jj[u] + cl[u]] = sn[u] * xi[u] + c[u] * xj[u];
          }
        }
      }
      __syncthreads();
      if (lane < npair && pi[lane] != pj[lane] && cs_s[lane] != 0.0) {
        a[pi[lane] * LD + pj[lane]] = 0.0;
        a[pj[lane] * LD + pi[lane]] = 0.0;
      }
      __syncthreads();
    }
  }
  // order by decreasing eigenvalue (stable in the index)
  if (lane < p) {
    const double lk = a[lane * LD + lane];
    int r = 0;
    for (int q = 0; q < p; ++q) {
      const double lq = a[q * LD + q];
      if (lq > lk || (lq == lk && q < lane)) ++r;
    }
    ord[r] = lane;
  }
  __syncthreads();
  double* V = F.vbuf + (size_t)it * MSTRIDE;
  double* W = F.wbuf + (size_t)it * MSTRIDE;
  if (lane < p) {
    for (int c = 0; c < p; ++c) {
      const double x = v[lane * LD + ord[c]];
      V[lane * PMAX + c] = x;       // column c = eigenvector of the c-th largest eigenvalue
      W[c * PMAX + lane] = x;       // W = V^T: scores t_c = sum_i V_ic z_i
    }
  }
  if (lane == 0) {
    const double l1 = a[ord[0] * LD + ord[0]], lp = a[ord[p - 1] * LD + ord[p - 1]];
    if (!(lp > 0.0) || !(l1 / lp <= kappa_max)) A.status[it] = ST_DROP_REFINE;
  }
}

// stage 1 (Sec. 3.3 step 3): D~ = diag(sigma_uni^2(T_j)), Sigma_k = V D~ V^T and
//          the sphering matrix Sigma_k^{-1/2} = V D~^{-1/2} V^T;
// stage 2 (step 4): mu_k = Sigma_k^{1/2} (mu_uni(Z~_1), ..., mu_uni(Z~_p)).
__global__ void k_refine(int stage, const ItemDesc* __restrict__ items, ItemArrays A, FitArrays F,
                         int first, const SegStat* __restrict__ st,
                         const int32_t* __restrict__ seg0) {
  __shared__ double sg[PMAX];
  __shared__ double mt[PMAX];
  __shared__ int bad;
  const int it = first + blockIdx.x;
  if (A.status[it] != ACTIVE) return;
  const int p = items[it].p;
  const double* V = F.vbuf + (size_t)it * MSTRIDE;
  const int s0 = seg0[it];
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  if (stage == 1) {
    for (int j = threadIdx.x; j < p; j += blockDim.x) {
      const double s2 = st[s0 + j].var;
      if (!(s2 > 0.0) || !(s2 < 1e300)) bad = 1;
      sg[j] = s2;
      F.s2buf[(size_t)it * PMAX + j] = s2;
    }
    __syncthreads();
    if (bad) {
      if (threadIdx.x == 0) A.status[it] = ST_DROP_REFINE;
      return;
    }
    double* S = A.sigz + (size_t)it * MSTRIDE;
    double* W = F.wbuf + (size_t)it * MSTRIDE;
    for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
      const int i = e / p, j = e % p;
      double s = 0.0, w = 0.0;
      for (int c = 0; c < p; ++c) {
        const double vv = V[i * PMAX + c] * V[j * PMAX + c];
        s = fma(vv, sg[c], s);
        w = fma(vv, 1.0 / sqrt(sg[c]), w);
      }
      S[i * PMAX + j] = s;
      W[i * PMAX + j] = w;
    }
  } else {
    for (int j = threadIdx.x; j < p; j += blockDim.x) {
      sg[j] = sqrt(F.s2buf[(size_t)it * PMAX + j]);
      mt[j] = st[s0 + j].mu;
    }
    __syncthreads();
    double* mu = A.muz + (size_t)it * PMAX;
    for (int i = threadIdx.x; i < p; i += blockDim.x) {
      double s = 0.0;
      for (int j = 0; j < p; ++j) {
        double r = 0.0;     // (Sigma_k^{1/2})_ij
        for (int c = 0; c < p; ++c) r = fma(V[i * PMAX + c] * V[j * PMAX + c], sg[c], r);
        s = fma(r, mt[j], s);
      }
      mu[i] = s;
    }
  }
}

// ------------------------------------------------------------ start choice (Sec. 4 step 4)
// The start with the smaller determinant; equal subsets or equal log-dets go
// to the first start.  The block fit is scaled by c(alpha) (eq. mcdraw).
__global__ __launch_bounds__(256) void k_choose(const ItemDesc* __restrict__ bitems,
                                                const ItemDesc* __restrict__ citems, ItemArrays A,
                                                FitArrays F, const DsInfo* __restrict__ ds,
                                                int first) {
  __shared__ int diff;
  const int b = first + blockIdx.x;
  const ItemDesc B = bitems[b];
  const DsInfo d = ds[B.ds];
  const int p = B.p;
  const int i0 = d.item0 + 2 * (b - d.blk0), i1 = i0 + 1;
  auto okst = [](int s) { return s == ST_CONVERGED || s == ST_NOTCONV || s == ST_ILLCOND; };
  const bool v0 = okst(A.status[i0]), v1 = okst(A.status[i1]);
  if (threadIdx.x == 0) diff = 0;
  __syncthreads();
  if (v0 && v1) {
    const uint8_t* m0 = A.mask + citems[i0].roff;
    const uint8_t* m1 = A.mask + citems[i1].roff;
    int dl = 0;
    for (int64_t r = threadIdx.x; r < B.m; r += blockDim.x) dl |= (m0[r] != m1[r]);
    if (dl) diff = 1;
  }
  __syncthreads();
  int ch = -1;
  if (v0 && v1) ch = (!diff || !(A.logdet[i1] < A.logdet[i0])) ? i0 : i1;
  else if (v0) ch = i0;
  else if (v1) ch = i1;
  const double lc = log(d.calpha);
  for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
    const int i = e / p, j = e % p;
    F.bsig[(size_t)b * MSTRIDE + i * PMAX + j] =
        ch >= 0 ? d.calpha * A.sigz[(size_t)ch * MSTRIDE + i * PMAX + j] : 0.0;
  }
  for (int j = threadIdx.x; j < p; j += blockDim.x)
    F.bmu[(size_t)b * PMAX + j] = ch >= 0 ? A.muz[(size_t)ch * PMAX + j] : 0.0;
  if (threadIdx.x == 0) {
    F.bitem[b] = ch;
    F.bds[b] = B.ds;
    F.bstat[b] = ch >= 0 ? A.status[ch] : RTDETMCD_BLOCK_INVALID;
    F.bstart[b] = ch < 0 ? -1 : d.warm_mu ? RTDETMCD_START_WARM : ch - i0;
    F.biters[b] = ch >= 0 ? A.iter[ch] : 0;
    F.bld[b] = ch >= 0 ? A.logdet[ch] + p * lc : NAN;
  }
}

// Warm start: block l of dataset d starts its C-steps from the given
// location and scatter, taken into the dataset's standardised units
// (z = (x - loc) / scale); its second start is not used.
__global__ __launch_bounds__(256) void k_warm_start(const DsInfo* __restrict__ ds, int dd,
                                                    ItemArrays C, FitArrays F) {
  const DsInfo d = ds[dd];
  const int p = d.p;
  const int i0 = d.item0 + 2 * blockIdx.x;
  const double* __restrict__ loc = F.loc + (size_t)dd * PMAX;
  const double* __restrict__ sc = F.scale + (size_t)dd * PMAX;
  for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
    const int i = e / p, j = e % p;
    C.sigz[(size_t)i0 * MSTRIDE + i * PMAX + j] =
        0.5 * (d.warm_sigma[i * p + j] + d.warm_sigma[j * p + i]) / (sc[i] * sc[j]);
  }
  for (int j = threadIdx.x; j < p; j += blockDim.x)
    C.muz[(size_t)i0 * PMAX + j] = (d.warm_mu[j] - loc[j]) / sc[j];
  if (threadIdx.x == 0) {
    C.status[i0] = ACTIVE;
    C.status[i0 + 1] = ST_DROP_REFINE;
  }
}

// ------------------------------------------------------------ aggregation (Sec. 4 steps 5-7)

// Entrywise median over the valid blocks of a dataset; an even count takes the
// mean of the two middle values.  One block per (dataset, entry); entry e < p
// is mu_e, otherwise a lower-triangle entry of Sigma.
__global__ __launch_bounds__(256) void k_median(const DsInfo* __restrict__ ds, FitArrays F,
                                                const int2* __restrict__ ent) {
  __shared__ double vs[8192];   // the entry of every valid block (q <= 8192), any order
  __shared__ double lo_v, hi_v;
  __shared__ int nvs;
  const int2 de = ent[blockIdx.x];
  const DsInfo d = ds[de.x];
  const int p = d.p;
  int i = -1, j = -1;
  if (de.y >= p) {
    int k = de.y - p, r = 0;
    while (k > r) { k -= r + 1; ++r; }
    i = r;
    j = k;
  }
  auto val = [&](int b) -> double {
    return i < 0 ? F.bmu[(size_t)b * PMAX + de.y] : F.bsig[(size_t)b * MSTRIDE + i * PMAX + j];
  };
  if (threadIdx.x == 0) nvs = 0;
  __syncthreads();
  // the valid blocks' values, gathered in LDS once (ranks depend on values only)
  for (int b = d.blk0 + threadIdx.x; b < d.blk0 + d.q; b += blockDim.x)
    if (F.bitem[b] >= 0) vs[atomicAdd(&nvs, 1)] = val(b);
  __syncthreads();
  const int nv = nvs;
  if (nv == 0) return;
  const int k1 = (nv - 1) / 2, k2 = nv / 2;
  for (int t = threadIdx.x; t < nv; t += blockDim.x) {
    const double x = vs[t];
    int less = 0, eq = 0;
    for (int c = 0; c < nv; ++c) {
      const double y = vs[c];
      less += y < x;
      eq += y == x;
    }
    if (less <= k1 && k1 < less + eq) lo_v = x;   // all writers store the same value
    if (less <= k2 && k2 < less + eq) hi_v = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double med = 0.5 * (lo_v + hi_v);
    double* M = F.med + (size_t)de.x * (PMAX + MSTRIDE);
    if (i < 0) M[de.y] = med;
    else {
      M[PMAX + i * PMAX + j] = med;
      M[PMAX + j * PMAX + i] = med;
    }
  }
}

// KL'_l = tr(S_med S_l^{-1}) + log det S_l + (mu_med - mu_l)' S_l^{-1} (mu_med - mu_l)
// for the raw block fit S_l = c(alpha) Sigma_l; eq. (KL) without its
// l-independent terms, so that a non-positive-definite S_med is allowed.
// use_sinv: the chosen item's inverse comes from its kept inverse sscp matrix
// (single-swap mode: its last step may not have had a Cholesky factor).
__global__ __launch_bounds__(256) void k_kl(const DsInfo* __restrict__ ds, ItemArrays A,
                                            FitArrays F, int first, int use_sinv) {
  __shared__ double Si[PMAX * PMAX];
  __shared__ double dv[PMAX];
  __shared__ double red[256];
  const int b = first + blockIdx.x;
  const int ch = F.bitem[b];
  if (ch < 0) {
    if (threadIdx.x == 0) F.bkl[b] = INFINITY;
    return;
  }
  const DsInfo d = ds[F.bds[b]];
  const int p = d.p;
  const double* Li = A.linv + (size_t)ch * MSTRIDE;
  const double* M = F.med + (size_t)F.bds[b] * (PMAX + MSTRIDE);
  const double ic = 1.0 / d.calpha;
  if (use_sinv) {
    // Sigma^{-1} = (h-1) D Lam^{-1} D (standardised units)
    const double* Lv = A.sinv + (size_t)ch * MSTRIDE;
    const double* sc = F.scale + (size_t)F.bds[b] * PMAX;
    for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
      const int i = e / p, j = e % p;
      Si[i * PMAX + j] = (double)(d.h - 1) * Lv[i * PMAX + j] * (sc[i] * sc[j]) * ic;
    }
  } else {
    for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
      const int i = e / p, j = e % p;
      const int k0 = i > j ? i : j;
      double s = 0.0;
      for (int k = k0; k < p; ++k) s = fma(Li[k * PMAX + i], Li[k * PMAX + j], s);
      Si[i * PMAX + j] = s * ic;
    }
  }
  for (int j = threadIdx.x; j < p; j += blockDim.x) dv[j] = M[j] - F.bmu[(size_t)b * PMAX + j];
  __syncthreads();
  double acc = 0.0;
  for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
    const int i = e / p, j = e % p;
    acc = fma(M[PMAX + i * PMAX + j] + dv[i] * dv[j], Si[i * PMAX + j], acc);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < 256; ++k) s += red[k];
    F.bkl[b] = s + F.bld[b];
  }
}

// Keep the ceil(q/2) valid blocks of smallest KL' (ties to the lower block)
// and pool them in that order with the single-pass update of Sec. 4 step 7
// (block counts m, Lambda_l = (m-1) S_l).  The result is the start of the
// first global item (reweighting).
__global__ __launch_bounds__(256) void k_pool(DsInfo* __restrict__ ds, ItemArrays G, FitArrays F,
                                              int first_ds, int union_mode) {
  __shared__ int order[4096];   // ceil(q/2) <= 4096 (q <= 8192 is enforced by the planner)
  __shared__ double mu[PMAX];
  __shared__ int nvs;
  const int dd = first_ds + blockIdx.x;
  DsInfo d = ds[dd];
  const int p = d.p, q = d.q;
  if (d.err) return;
  if (threadIdx.x == 0) {
    int c = 0;
    for (int b = d.blk0; b < d.blk0 + q; ++b) c += F.bitem[b] >= 0;
    nvs = c;
  }
  __syncthreads();
  const int nv = nvs;
  if (nv == 0) {
    if (threadIdx.x == 0) ds[dd].err = RTDETMCD_ESINGULAR;
    return;
  }
  const int keep = (nv + 1) / 2;
  for (int b = d.blk0 + threadIdx.x; b < d.blk0 + q; b += blockDim.x) {
    if (F.bitem[b] < 0) continue;
    const double x = F.bkl[b];
    int r = 0;
    for (int c = d.blk0; c < d.blk0 + q; ++c) {
      if (F.bitem[c] < 0) continue;
      const double y = F.bkl[c];
      r += (y < x) || (y == x && c < b);
    }
    if (r < keep && r < 4096) order[r] = b;
  }
  __syncthreads();
  // PRINTED: each kept block counts m rows with Lambda_l = (m - 1) Sigma_raw^(l)
  // (c(alpha) included).  UNION: the kept blocks' h-subsets, disjoint, so
  // pooling their (h, mean, Lambda_l = (h - 1) S_l) gives the classical mean
  // and covariance of the union; S_l is Sigma_raw^(l) without c(alpha), which
  // multiplies the pooled covariance once at the end.
  // The pooled pair in closed form (what merging the blocks one after the
  // other gives, up to rounding): mu = sum_l m mu_l / N and Lambda =
  // sum_l [Lambda_l + m (mu_l - mu)(mu_l - mu)^T]; every entry is its own sum
  // over the kept blocks, taken in KL order.
  const double m = union_mode ? (double)d.h : (double)d.m;
  const double lf = union_mode ? ((double)d.h - 1.0) / d.calpha : (double)d.m - 1.0;
  const int g0 = d.glob0;
  double* Lam = G.sigz + (size_t)g0 * MSTRIDE;   // Lambda_pooled
  const int nk = keep < 4096 ? keep : 4096;
  const double np = m * nk;
  for (int j = threadIdx.x; j < p; j += blockDim.x) {
    double s = 0.0;
    for (int r = 0; r < nk; ++r) s += F.bmu[(size_t)order[r] * PMAX + j];
    mu[j] = s / nk;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
    const int i = e / p, j = e % p;
    double a = 0.0, c = 0.0;
    for (int r = 0; r < nk; ++r) {
      const int b = order[r];
      a += F.bsig[(size_t)b * MSTRIDE + i * PMAX + j];
      c = fma(F.bmu[(size_t)b * PMAX + i] - mu[i], F.bmu[(size_t)b * PMAX + j] - mu[j], c);
    }
    Lam[i * PMAX + j] = lf * a + m * c;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
    const int i = e / p, j = e % p;
    double v = 0.5 * (Lam[i * PMAX + j] + Lam[j * PMAX + i]) / (np - 1.0);
    if (union_mode) v *= d.calpha;
    F.sigraw[(size_t)dd * MSTRIDE + i * PMAX + j] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
    const int i = e / p, j = e % p;
    Lam[i * PMAX + j] = F.sigraw[(size_t)dd * MSTRIDE + i * PMAX + j];
  }
  for (int j = threadIdx.x; j < p; j += blockDim.x) {
    F.muraw[(size_t)dd * PMAX + j] = mu[j];
    G.muz[(size_t)g0 * PMAX + j] = mu[j];
  }
}

// Reweighted location and scatter from the sscp partials of the rows with
// RD^2 <= chi2_{p,q} (Sec. 2.1, Sec. 4 steps 8-9): the classical mean and
// covariance (divisor n_w - 1) of those rows, optionally times c(q).  The
// result is the start of the second global item (final distances).
__global__ __launch_bounds__(256) void k_rew(DsInfo* __restrict__ ds,
                                             const ItemDesc* __restrict__ gitems, ItemArrays G,
                                             FitArrays F, int first_ds) {
  __shared__ double sv[PMAX + 1];
  const int dd = first_ds + blockIdx.x;
  const DsInfo d = ds[dd];
  if (d.err) return;
  const int p = d.p;
  const int g0 = d.glob0, g1 = d.glob1;
  const ItemDesc D = gitems[g0];
  const double* __restrict__ P0 = G.part + (size_t)D.tile0 * PSTRIDE;   // collapsed partial
  for (int e = threadIdx.x; e <= p; e += blockDim.x) sv[e] = P0[e];
  __syncthreads();
  const double nw = sv[0];
  if (!(nw > (double)p)) {
    if (threadIdx.x == 0) ds[dd].err = RTDETMCD_ESINGULAR;
    return;
  }
  const double* c = G.mux + (size_t)g0 * PMAX;
  for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
    const int i = e / p, j = e % p;
    const int a = i >= j ? i : j, bb = i >= j ? j : i;
    const double s = P0[1 + PMAX + a * (a + 1) / 2 + bb];
    const double lam = s - sv[1 + i] * sv[1 + j] / nw;
    const double sx = lam / (nw - 1.0) * d.crew;
    G.sigz[(size_t)g1 * MSTRIDE + i * PMAX + j] =
        sx / (D.scale[i] * D.scale[j]);
  }
  for (int j = threadIdx.x; j < p; j += blockDim.x) {
    const double mx = c[j] + sv[1 + j] / nw;
    G.muz[(size_t)g1 * PMAX + j] = (mx - D.loc[j]) / D.scale[j];
  }
  if (threadIdx.x == 0) F.nw[dd] = (int64_t)nw;
}

// Random partition (Sec. 4): validate the permutation and build its inverse.
__global__ __launch_bounds__(256) void k_perm_check(const int32_t* __restrict__ perm, int64_t n,
                                                    int32_t* __restrict__ inv,
                                                    DsInfo* __restrict__ ds, int d) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int32_t i = perm[k];
  bool bad = i < 0 || (int64_t)i >= n;
  if (!bad) bad = atomicExch(&inv[i], (int32_t)k) != -1;   // a repeated row
  if (bad) ds[d].err = RTDETMCD_EINVAL;
}

// The fitted rows of a randomly partitioned dataset, in block order.
template <typename T>
__global__ __launch_bounds__(256) void k_perm_gather(const T* __restrict__ X, int64_t n,
                                                     int64_t ld, int p,
                                                     const int32_t* __restrict__ perm,
                                                     int64_t rows, T* __restrict__ Xp) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * p) return;
  const int64_t k = e / p;
  const int j = (int)(e - k * p);
  const int32_t i = perm[k];
  Xp[e] = (i >= 0 && (int64_t)i < n) ? X[(int64_t)i * ld + j] : (T)0;
}

// Subset indices of each block's chosen start: rows of X in order of their
// position within the block (ascending rows for contiguous blocks).
__global__ __launch_bounds__(1024) void k_hsub(const ItemDesc* __restrict__ citems, ItemArrays A,
                                               FitArrays F, const DsInfo* __restrict__ ds,
                                               const rtdetmcd_out* __restrict__ outs, int first) {
  __shared__ int wtot[16];
  const int b = first + blockIdx.x;
  const int dd = F.bds[b];
  const DsInfo d = ds[dd];
  int32_t* o = outs[dd].hsubset;
  if (!o) return;
  o += (size_t)(b - d.blk0) * d.h;
  const int ch = F.bitem[b];
  if (ch < 0) {
    for (int64_t k = threadIdx.x; k < d.h; k += blockDim.x) o[k] = -1;
    return;
  }
  const ItemDesc C = citems[ch];
  const uint8_t* mk = A.mask + C.roff;
  int64_t n = 0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int64_t base = 0; base < C.m; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const int f = (i < C.m && mk[i]) ? 1 : 0;
    const uint64_t bal = __ballot(f);
    const int pos = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wtot[wv] = __popcll(bal);
    __syncthreads();
    int off = 0, tot = 0;
    for (int k = 0; k < 16; ++k) {
      if (k < wv) off += wtot[k];
      tot += wtot[k];
    }
    if (f && n + off + pos < d.h)   // block position -> row of X
      o[n + off + pos] = d.perm ? d.perm[C.row0 + i] : (int32_t)(C.row0 + i);
    n += tot;
    __syncthreads();
  }
}

// Outputs in the units of X (affine equivariance: mu_X = loc + scale mu_Z,
// Sigma_X = D Sigma_Z D, distances unchanged).
__global__ __launch_bounds__(256) void k_outputs(const DsInfo* __restrict__ ds, ItemArrays G,
                                                 FitArrays F, const rtdetmcd_out* __restrict__ outs,
                                                 int first_ds) {
  const int dd = first_ds + blockIdx.x;
  const DsInfo d = ds[dd];
  const rtdetmcd_out o = outs[dd];
  const int p = d.p;
  const double* loc = F.loc + (size_t)dd * PMAX;
  const double* sc = F.scale + (size_t)dd * PMAX;
  const int g0 = d.glob0, g1 = d.glob1;
  const bool ok = d.err == 0;
  for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
    const int i = e / p, j = e % p;
    if (o.sigma) o.sigma[e] = ok ? sc[i] * sc[j] * G.sigz[(size_t)g1 * MSTRIDE + i * PMAX + j] : NAN;
    if (o.sigma_raw)
      o.sigma_raw[e] = ok ? sc[i] * sc[j] * F.sigraw[(size_t)dd * MSTRIDE + i * PMAX + j] : NAN;
  }
  for (int j = threadIdx.x; j < p; j += blockDim.x) {
    if (o.mu) o.mu[j] = ok ? loc[j] + sc[j] * G.muz[(size_t)g1 * PMAX + j] : NAN;
    if (o.mu_raw) o.mu_raw[j] = ok ? loc[j] + sc[j] * F.muraw[(size_t)dd * PMAX + j] : NAN;
    if (o.loc) o.loc[j] = loc[j];
    if (o.scale) o.scale[j] = sc[j];
  }
  for (int b = threadIdx.x; b < d.q; b += blockDim.x) {
    if (o.block_status) o.block_status[b] = F.bstat[d.blk0 + b];
    if (o.block_start) o.block_start[b] = F.bstart[d.blk0 + b];
    if (o.block_iters) o.block_iters[b] = F.biters[d.blk0 + b];
  }
  if (threadIdx.x == 0) {
    double ls = 0.0;
    for (int j = 0; j < p; ++j) ls += 2.0 * log(sc[j]);
    if (o.logdet) {
      o.logdet[0] = ok ? G.logdet[g0] + ls : NAN;
      o.logdet[1] = ok ? G.logdet[g1] + ls : NAN;
    }
    if (o.n_w) *o.n_w = ok ? F.nw[dd] : 0;
  }
}

// Diagnostics of a fit, written only where the caller asked for them.
// Blocks [0, nb): per fitted block, the log det of the chosen start's scatter
// at each of its evaluated C-steps (NaN from block_iters on) and the gap
// d2_(h+1) - d2_(h) of its last evaluated distances (smallest distance left
// out minus largest kept).  Blocks [nb, nb + nds): per dataset, the smallest
// |dist^2 - chi2_{p,q}| over the final distances.
__global__ __launch_bounds__(256) void k_diag(const ItemDesc* __restrict__ citems, ItemArrays A,
                                              FitArrays F, const DsInfo* __restrict__ ds,
                                              const rtdetmcd_out* __restrict__ outs, int nb,
                                              int maxs) {
  __shared__ double red[2][4];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double a = -INFINITY, b = INFINITY;   // largest kept, smallest left out (or smallest margin)
  bool want = false;
  double* dst = nullptr;
  if ((int)blockIdx.x < nb) {
    const int bk = blockIdx.x;
    const int dd = F.bds[bk];
    const DsInfo d = ds[dd];
    const rtdetmcd_out o = outs[dd];
    const int lb = bk - d.blk0;
    const int ch = F.bitem[bk];
    if (o.ldtrace) {
      const int iters = ch >= 0 ? F.biters[bk] : 0;
      for (int t = tid; t < maxs; t += blockDim.x)
        o.ldtrace[(size_t)lb * maxs + t] =
            (ch >= 0 && A.ldtr && t < iters && t < A.ldtr_n) ? A.ldtr[(size_t)ch * A.ldtr_n + t]
                                                             : NAN;
    }
    if (o.hmargin && ch >= 0) {   // uniform
      const ItemDesc C = citems[ch];
      const double* __restrict__ d2 = A.d2 + C.roff;
      const uint8_t* __restrict__ mk = A.mask + C.roff;
      for (int64_t i = tid; i < C.m; i += blockDim.x) {
        const double v = d2[i];
        if (mk[i]) a = fmax(a, v);
        else b = fmin(b, v);
      }
      want = true;
      dst = o.hmargin + lb;
    } else if (o.hmargin && tid == 0) {
      o.hmargin[lb] = NAN;
    }
  } else {
    const int dd = blockIdx.x - nb;
    const DsInfo d = ds[dd];
    const rtdetmcd_out o = outs[dd];
    if (o.cmargin) {   // uniform
      if (o.dist && d.err == 0) {
        for (int64_t i = tid; i < d.n; i += blockDim.x) {
          const double v = o.dist[i];
          b = fmin(b, fabs(v * v - d.chi2p));
        }
        want = true;
        dst = o.cmargin;
      } else if (tid == 0) {
        *o.cmargin = NAN;
      }
    }
  }
  if (!want) return;   // uniform
  a = wave_max(a);
  b = -wave_max(-b);
  if (lane == 0) {
    red[0][w] = a;
    red[1][w] = b;
  }
  __syncthreads();
  if (tid == 0) {
    for (int k = 1; k < 4; ++k) {
      a = fmax(a, red[0][k]);
      b = fmin(b, red[1][k]);
    }
    const bool cm = (int)blockIdx.x >= nb;
    *dst = cm ? b : ((a > -INFINITY && b < INFINITY) ? b - a : NAN);
  }
}

// MODE 0 for p >= 16 on the float64 matrix cores: the scores of 16 rows at a
// time, D = W_tile (16 output columns x 4) x Z^T (4 x 16 rows) over the k
// steps (16x16x4 MFMA).  Each wave stages chunks of its rows in its own LDS
// region; lane l supplies z of row (l mod 16), column 4 s + l/16 (each
// element standardised once) and receives output columns 16 t + l/16 + 4 v
// of that row, which it stores as keys (16 consecutive rows of a column per
// 16 lanes).
typedef double dbl4 __attribute__((ext_vector_type(4)));

template <typename T, int P>
struct PShape {
  static constexpr int NG = (P + 15) / 16;
  static constexpr int KS = (P + 3) / 4;
  static constexpr int CR = P <= 32 ? 64 : 32;   // rows per wave chunk
};

template <typename T, int P>
__global__ __launch_bounds__(256) void k_project_mfma(const ItemDesc* __restrict__ items,
                                                      const Tile* __restrict__ tiles,
                                                      int tile_rows,
                                                      const int32_t* __restrict__ status,
                                                      const double* __restrict__ W,
                                                      const int64_t* __restrict__ kbase,
                                                      uint64_t* __restrict__ keys) {
  using S = PShape<T, P>;
  constexpr int NG = S::NG, KS = S::KS, CR = S::CR;
  __shared__ double Wl[NG * KS * 64];
  __shared__ double sloc[P], sisc[P];
  __shared__ T xw[4 * CR * P];
  const Tile tl = tiles[blockIdx.x];
  const int it = tl.item;
  if (status != nullptr && status[it] != ACTIVE) return;
  const ItemDesc D = items[it];
  const int p = D.p;
  const T* __restrict__ X = static_cast<const T*>(D.X) + D.row0 * D.ld;
  const double* __restrict__ Wi = W + (size_t)it * MSTRIDE;
  uint64_t* __restrict__ ko = keys + kbase[it];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  for (int e = tid; e < NG * KS * 64; e += 256) {
    const int l = e & 63, ts = e >> 6, t = ts / KS, sidx = ts % KS;
    const int i = 16 * t + (l & 15), k = 4 * sidx + (l >> 4);
    Wl[e] = (i < p && k < p) ? Wi[i * PMAX + k] : 0.0;
  }
  for (int j = tid; j < P; j += 256) {
    sloc[j] = j < p ? D.loc[j] : 0.0;
    sisc[j] = j < p ? D.scale[j] : 1.0;
  }
  __syncthreads();
  const int64_t r0 = (int64_t)tl.t * tile_rows;
  const int64_t r1 = min(r0 + (int64_t)tile_rows, D.m);
  const int64_t per = (((r1 - r0) + 3) / 4 + 15) / 16 * 16;
  const int64_t w0 = r0 + wv * per, w1 = min(w0 + per, r1);
  T* __restrict__ xs = xw + wv * CR * P;
  const bool vec = p == P && D.ld == P && ((reinterpret_cast<uintptr_t>(X) & 15) == 0);
  for (int64_t base = w0; base < w1; base += CR) {
    const int n = (int)min((int64_t)CR, w1 - base);
    __syncwarp();   // the previous chunk's reads of xs are done
    if (vec) {
      typedef unsigned V __attribute__((ext_vector_type(4)));
      const V* __restrict__ src = reinterpret_cast<const V*>(X + base * P);
      V* __restrict__ dst = reinterpret_cast<V*>(xs);
      const int nv = (n * P * (int)sizeof(T)) / 16;
      for (int k = lane; k < nv; k += 64) dst[k] = src[k];
      for (int e = nv * (16 / (int)sizeof(T)) + lane; e < n * P; e += 64) xs[e] = X[base * P + e];
    } else {
      for (int e = lane; e < n * P; e += 64) {
        const int r = e / P, j = e - r * P;
        xs[e] = j < p ? X[(base + r) * D.ld + j] : (T)0;
      }
    }
    __syncwarp();   // staged rows visible to the whole wave
    for (int g = 0; g < n; g += 16) {
      const int rb = g + lr;
      double zb[KS];
#pragma unroll
      for (int sidx = 0; sidx < KS; ++sidx) {
        const int k = 4 * sidx + lk;
        zb[sidx] = (rb < n && k < p) ? ((double)xs[rb * P + k] - sloc[k]) / sisc[k] : 0.0;
      }
#pragma unroll
      for (int t = 0; t < NG; ++t) {
        dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int sidx = 0; sidx < KS; ++sidx)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Wl[(t * KS + sidx) * 64 + lane], zb[sidx],
                                                     acc, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int col = 16 * t + lk + 4 * v;
          if (col < p && rb < n) ko[(size_t)col * D.m + base + rb] = fkey64(acc[v]);
        }
      }
    }
  }
}

template <typename T, int P, int MODE>
hipError_t project_t(const ItemDesc* items, const Tile* tiles, int ntiles, int tile_rows,
                     const int32_t* status, const double* W, const int64_t* kbase, uint64_t* keys,
                     hipStream_t s) {
  if constexpr (MODE == 0 && P >= 16)
    hipLaunchKernelGGL((k_project_mfma<T, P>), dim3(ntiles), dim3(256), 0, s, items, tiles,
                       tile_rows, status, W, kbase, keys);
  else {
    if (tile_rows % PROJ_ROWS != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_project<T, P, MODE>), dim3(ntiles * (tile_rows / PROJ_ROWS)),
                       dim3(PROJ_ROWS), 0, s, items, tiles, tile_rows, status, W, kbase, keys);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_colkeys(int dtype, const ColJob* jobs, int njobs, int64_t ntiles,
                          hipStream_t s) {
  if (njobs <= 0 || ntiles <= 0) return hipSuccess;
  if (ntiles > 0x7fffffff) return hipErrorInvalidValue;
  if (dtype == 0)
    hipLaunchKernelGGL((k_colkeys<float, uint32_t>), dim3((unsigned)ntiles), dim3(CK_NT), 0, s,
                       jobs, njobs);
  else
    hipLaunchKernelGGL((k_colkeys<double, uint64_t>), dim3((unsigned)ntiles), dim3(CK_NT), 0, s,
                       jobs, njobs);
  return hipGetLastError();
}

hipError_t launch_std_finish(const SegStat* st32, const SegStat* st64, const int32_t* seg0,
                             const int32_t* in64, int D, DsInfo* ds, FitArrays F, hipStream_t s) {
  hipLaunchKernelGGL(k_std_finish, dim3(D), dim3(64), 0, s, st32, st64, seg0, in64, D, ds, F);
  return hipGetLastError();
}

hipError_t launch_project(int bucket, int dtype, int mode, const ItemDesc* items,
                          const Tile* tiles, int ntiles, int tile_rows, const int32_t* status,
                          const double* W, const int64_t* kbase, uint64_t* keys, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
#define CASE(PB)                                                                               \
  case PB:                                                                                     \
    if (dtype == 0)                                                                            \
      return mode == 0 ? project_t<float, PB, 0>(items, tiles, ntiles, tile_rows, status, W,   \
                                                 kbase, keys, s)                               \
                       : project_t<float, PB, 1>(items, tiles, ntiles, tile_rows, status, W,   \
                                                 kbase, keys, s);                              \
    return mode == 0 ? project_t<double, PB, 0>(items, tiles, ntiles, tile_rows, status, W,    \
                                                kbase, keys, s)                                \
                     : project_t<double, PB, 1>(items, tiles, ntiles, tile_rows, status, W,    \
                                                kbase, keys, s);
  switch (bucket) {
    CASE(4) CASE(5) CASE(8) CASE(10) CASE(16) CASE(20) CASE(24) CASE(32) CASE(40) CASE(48)
    CASE(64)
    default: return hipErrorInvalidValue;
  }
#undef CASE
}

hipError_t launch_reduce_partials(const ItemDesc* items, const double* part, int first, int n,
                                  double* cnt, double* sum, double* S, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_partials, dim3(n), dim3(256), 0, s, items, part, first, cnt, sum, S);
  return hipGetLastError();
}

hipError_t launch_init_cov(int mode, const ItemDesc* bitems, int first, int n, FitArrays F,
                           ItemArrays C, const DsInfo* ds, double* cut, const SegStat* gst,
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_init_cov, dim3(n), dim3(256), 0, s, mode, bitems, first, F, C, ds, cut, gst);
  return hipGetLastError();
}

hipError_t launch_eig(int bucket, const ItemDesc* items, ItemArrays A, FitArrays F, int first,
                      int n, double kappa_max, hipStream_t s) {
  if (n <= 0) return hipSuccess;
#define CASE(PB)                                                                             \
  case PB:                                                                                   \
    hipLaunchKernelGGL((k_eig<PB>), dim3(n), dim3(64), 0, s, items, A, F, first, kappa_max); \
    break;
  switch (bucket) {
    CASE(4) CASE(5) CASE(8) CASE(10) CASE(16) CASE(20) CASE(24) CASE(32) CASE(40) CASE(48)
    CASE(64)
    default: return hipErrorInvalidValue;
  }
#undef CASE
  return hipGetLastError();
}

hipError_t launch_refine(int stage, const ItemDesc* items, ItemArrays A, FitArrays F, int first,
                         int n, const SegStat* st, const int32_t* seg0, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_refine, dim3(n), dim3(256), 0, s, stage, items, A, F, first, st, seg0);
  return hipGetLastError();
}

hipError_t launch_choose(const ItemDesc* bitems, const ItemDesc* citems, ItemArrays A,
                         FitArrays F, const DsInfo* ds, int first, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_choose, dim3(n), dim3(256), 0, s, bitems, citems, A, F, ds, first);
  return hipGetLastError();
}

hipError_t launch_warm_start(const DsInfo* ds, int d, int q, ItemArrays C, FitArrays F,
                             hipStream_t s) {
  if (q <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_warm_start, dim3(q), dim3(256), 0, s, ds, d, C, F);
  return hipGetLastError();
}

hipError_t launch_median(const DsInfo* ds, FitArrays F, const int2* ent, int nent,
                         hipStream_t s) {
  if (nent <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_median, dim3(nent), dim3(256), 0, s, ds, F, ent);
  return hipGetLastError();
}

hipError_t launch_kl(const DsInfo* ds, ItemArrays A, FitArrays F, int first_blk, int nblk,
                     int use_sinv, hipStream_t s) {
  if (nblk <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_kl, dim3(nblk), dim3(256), 0, s, ds, A, F, first_blk, use_sinv);
  return hipGetLastError();
}

hipError_t launch_pool(DsInfo* ds, ItemArrays G, FitArrays F, int first_ds, int nds, int pool_mode,
                       hipStream_t s) {
  if (nds <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pool, dim3(nds), dim3(256), 0, s, ds, G, F, first_ds,
                     pool_mode == RTDETMCD_POOL_UNION ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_rew(DsInfo* ds, const ItemDesc* gitems, ItemArrays G, FitArrays F, int first_ds,
                      int nds, hipStream_t s) {
  if (nds <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rew, dim3(nds), dim3(256), 0, s, ds, gitems, G, F, first_ds);
  return hipGetLastError();
}

hipError_t launch_perm_check(const int32_t* perm, int64_t n, int32_t* inv, DsInfo* ds, int d,
                             hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_perm_check, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, perm, n,
                     inv, ds, d);
  return hipGetLastError();
}

hipError_t launch_perm_gather(int dtype, const void* X, int64_t n, int64_t ld, int p,
                              const int32_t* perm, int64_t rows, void* Xp, hipStream_t s) {
  const int64_t ne = rows * p;
  if (ne <= 0) return hipSuccess;
  const dim3 g((unsigned)((ne + 255) / 256));
  if (dtype == 0)
    hipLaunchKernelGGL(k_perm_gather<float>, g, dim3(256), 0, s, static_cast<const float*>(X), n,
                       ld, p, perm, rows, static_cast<float*>(Xp));
  else
    hipLaunchKernelGGL(k_perm_gather<double>, g, dim3(256), 0, s, static_cast<const double*>(X),
                       n, ld, p, perm, rows, static_cast<double*>(Xp));
  return hipGetLastError();
}

hipError_t launch_hsub(const ItemDesc* citems, ItemArrays A, FitArrays F, const DsInfo* ds,
                       const rtdetmcd_out* outs, int first, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hsub, dim3(n), dim3(1024), 0, s, citems, A, F, ds, outs, first);
  return hipGetLastError();
}

hipError_t launch_outputs(const DsInfo* ds, ItemArrays G, FitArrays F, const rtdetmcd_out* outs,
                          int first_ds, int nds, hipStream_t s) {
  if (nds <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_outputs, dim3(nds), dim3(256), 0, s, ds, G, F, outs, first_ds);
  return hipGetLastError();
}

hipError_t launch_diag(const ItemDesc* citems, ItemArrays A, FitArrays F, const DsInfo* ds,
                       const rtdetmcd_out* outs, int nb, int nds, int maxs, hipStream_t s) {
  if (nb + nds <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_diag, dim3(nb + nds), dim3(256), 0, s, citems, A, F, ds, outs, nb, maxs);
  return hipGetLastError();
}

}  // namespace rtd
