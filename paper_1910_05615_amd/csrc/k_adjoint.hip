// Adjoint of the end of the fit (Sec. 4 steps 9-10) with respect to X, with
// the reweighting set W held fixed.
//
// The fit ends with  mu = mean of the rows of W,  Sigma = c cov(rows of W)
// (divisor n_w - 1), and  d_i = sqrt(r_i^T P r_i),  r_i = x_i - mu,
// P = Sigma^{-1}, for every row (eq. statdist).  W is a step function of X
// (constant away from ties at the cutoff, as are the h-subsets before it),
// so where the fit is differentiable its derivative is that of these
// formulas.  With cotangents v (of d), gbar_mu, Gbar_Sigma and w_i = v_i/d_i:
//
//   direct term   g_i  = w_i P r_i                              (every row)
//   g_mu = gbar_mu - P s,            s = sum_i w_i r_i
//   G    = Gbar_Sigma - 1/2 P B P,   B = sum_i w_i r_i r_i^T
//   rows of W     g_j += g_mu / n_w + c/(n_w - 1) (G + G^T) r_j
//
// s and B are a weighted sscp about mu: the matrix-core sscp kernel in its
// SSCP_ADJ mode computes them (weights w_i), the tile partials are collapsed,
// one block forms g_mu, G and the row coefficients, and one pass over the rows
// writes the gradient.  Everything in float64.
#include <algorithm>

#include "common.h"
#include "driver.h"

namespace rtd {

namespace {

constexpr int BW_NT = 256;

__global__ void k_bw_copy(const double* __restrict__ src, int p, double* __restrict__ dst) {
  for (int j = threadIdx.x; j < PMAX; j += blockDim.x) dst[j] = j < p ? src[j] : 0.0;
}

// P = Sigma^{-1} (full, row stride PMAX) by Cholesky, L^{-1} and L^{-T} L^{-1}.
// A Sigma that is not positive definite gives NaN (the fit never returns one).
__global__ __launch_bounds__(BW_NT) void k_bw_prep(const double* __restrict__ sigma, int p,
                                                   double* __restrict__ Pm) {
  __shared__ double Sg[PMAX * PMAX];
  __shared__ double Li[PMAX * PMAX];
  __shared__ int fail;
  const int tid = threadIdx.x;
  for (int e = tid; e < p * p; e += BW_NT) {
    const int i = e / p, j = e % p;
    Sg[i * PMAX + j] = 0.5 * (sigma[i * p + j] + sigma[j * p + i]);
  }
  if (tid == 0) fail = 0;
  __syncthreads();
  for (int k = 0; k < p; ++k) {
    if (tid == 0) {
      const double d = Sg[k * PMAX + k];
      if (!(d > 0.0)) fail = 1;
      else Sg[k * PMAX + k] = sqrt(d);
    }
    __syncthreads();
    if (fail) break;
    const double lkk = Sg[k * PMAX + k];
    for (int i = k + 1 + tid; i < p; i += BW_NT) Sg[i * PMAX + k] /= lkk;
    __syncthreads();
    const int nn = p - k - 1;
    for (int e = tid; e < nn * nn; e += BW_NT) {
      const int i = k + 1 + e / nn, j = k + 1 + e % nn;
      if (j <= i) Sg[i * PMAX + j] -= Sg[i * PMAX + k] * Sg[j * PMAX + k];
    }
    __syncthreads();
  }
  if (fail) {
    for (int e = tid; e < PMAX * PMAX; e += BW_NT) Pm[e] = NAN;
    return;
  }
  for (int j = tid; j < p; j += BW_NT) {   // column j of L^{-1}
    for (int i = 0; i < j; ++i) Li[i * PMAX + j] = 0.0;
    Li[j * PMAX + j] = 1.0 / Sg[j * PMAX + j];
    for (int i = j + 1; i < p; ++i) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s = fma(Sg[i * PMAX + k], Li[k * PMAX + j], s);
      Li[i * PMAX + j] = -s / Sg[i * PMAX + i];
    }
  }
  __syncthreads();
  for (int e = tid; e < PMAX * PMAX; e += BW_NT) {
    const int i = e / PMAX, j = e % PMAX;
    double v = 0.0;
    if (i < p && j < p) {
      for (int k = i > j ? i : j; k < p; ++k) v = fma(Li[k * PMAX + i], Li[k * PMAX + j], v);
    }
    Pm[e] = v;
  }
}

// g_mu, G and the coefficients of the rows of W:  u = g_mu / n_w and
// K = c/(n_w - 1) (G + G^T).  part0: collapsed sscp partial (count, s, packed
// B) or null when there is no distance cotangent.
__global__ __launch_bounds__(BW_NT) void k_bw_mid(const double* __restrict__ part0,
                                                  const double* __restrict__ Pm,
                                                  const double* __restrict__ g_mu,
                                                  const double* __restrict__ g_sigma,
                                                  const int64_t* __restrict__ n_w, double c, int p,
                                                  double* __restrict__ u, double* __restrict__ K) {
  __shared__ double Ps[PMAX * PMAX];
  __shared__ double Bs[PMAX * PMAX];
  __shared__ double T1[PMAX * PMAX];
  __shared__ double sv[PMAX];
  const int tid = threadIdx.x;
  for (int e = tid; e < p * p; e += BW_NT) {
    const int i = e / p, j = e % p;
    Ps[i * PMAX + j] = Pm[i * PMAX + j];
    const int a = i >= j ? i : j, b = i >= j ? j : i;
    Bs[i * PMAX + j] = part0 ? part0[1 + PMAX + a * (a + 1) / 2 + b] : 0.0;
  }
  for (int j = tid; j < p; j += BW_NT) sv[j] = part0 ? part0[1 + j] : 0.0;
  __syncthreads();
  for (int e = tid; e < p * p; e += BW_NT) {   // T1 = P B
    const int i = e / p, j = e % p;
    double v = 0.0;
    for (int k = 0; k < p; ++k) v = fma(Ps[i * PMAX + k], Bs[k * PMAX + j], v);
    T1[i * PMAX + j] = v;
  }
  __syncthreads();
  const double nw = (double)*n_w;
  for (int e = tid; e < p * p; e += BW_NT) {   // G = Gbar - 1/2 (P B) P, K = c/(nw-1)(G + G^T)
    const int i = e / p, j = e % p;
    double a = 0.0, b = 0.0;
    for (int k = 0; k < p; ++k) {
      a = fma(T1[i * PMAX + k], Ps[k * PMAX + j], a);
      b = fma(T1[j * PMAX + k], Ps[k * PMAX + i], b);
    }
    const double gij = (g_sigma ? g_sigma[i * p + j] : 0.0) - 0.5 * a;
    const double gji = (g_sigma ? g_sigma[j * p + i] : 0.0) - 0.5 * b;
    K[i * PMAX + j] = c / (nw - 1.0) * (gij + gji);
  }
  for (int j = tid; j < p; j += BW_NT) {
    double v = 0.0;
    for (int k = 0; k < p; ++k) v = fma(Ps[j * PMAX + k], sv[k], v);
    u[j] = ((g_mu ? g_mu[j] : 0.0) - v) / nw;
  }
}

// g_X row by row: w_i P r_i + [i in W] (u + K r_i); one row per thread.
template <typename T, int P>
__global__ __launch_bounds__(BW_NT) void k_bw_rows(const T* __restrict__ X, int64_t n, int64_t ld,
                                                   int p, const double* __restrict__ mu,
                                                   const double* __restrict__ Pm,
                                                   const double* __restrict__ K,
                                                   const double* __restrict__ u,
                                                   const double* __restrict__ dist,
                                                   const double* __restrict__ g_dist,
                                                   const uint8_t* __restrict__ W,
                                                   double* __restrict__ gX) {
  __shared__ double Ps[P * P], Ks[P * P], mus[P], us[P];
  for (int e = threadIdx.x; e < P * P; e += BW_NT) {
    const int i = e / P, j = e % P;
    const bool in = i < p && j < p;
    Ps[e] = in ? Pm[i * PMAX + j] : 0.0;
    Ks[e] = in ? K[i * PMAX + j] : 0.0;
  }
  for (int j = threadIdx.x; j < P; j += BW_NT) {
    mus[j] = j < p ? mu[j] : 0.0;
    us[j] = j < p ? u[j] : 0.0;
  }
  __syncthreads();
  for (int64_t r = (int64_t)blockIdx.x * BW_NT + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * BW_NT) {
    const T* __restrict__ xr = X + r * ld;
    double rv[P];
#pragma unroll
    for (int j = 0; j < P; ++j) rv[j] = j < p ? (double)xr[j] - mus[j] : 0.0;
    double w = 0.0;
    if (g_dist) {
      const double d = dist[r];
      w = d > 0.0 ? g_dist[r] / d : 0.0;
    }
    const bool inw = W[r] != 0;
    double* __restrict__ go = gX + r * p;
#pragma unroll 1
    for (int j = 0; j < p; ++j) {
      double y = 0.0, t = 0.0;
#pragma unroll
      for (int k = 0; k < P; ++k) {
        y = fma(Ps[j * P + k], rv[k], y);
        t = fma(Ks[j * P + k], rv[k], t);
      }
      go[j] = w * y + (inw ? us[j] + t : 0.0);
    }
  }
}

template <typename T>
hipError_t bw_rows_t(int bucket, const T* X, int64_t n, int64_t ld, int p, const double* mu,
                     const double* Pm, const double* K, const double* u, const double* dist,
                     const double* g_dist, const uint8_t* W, double* gX, hipStream_t s) {
  int64_t nb = (n + BW_NT - 1) / BW_NT;
  nb = std::min<int64_t>(nb, 16384);
#define CASE(PB)                                                                           \
  case PB:                                                                                 \
    hipLaunchKernelGGL((k_bw_rows<T, PB>), dim3((unsigned)nb), dim3(BW_NT), 0, s, X, n, ld, p, \
                       mu, Pm, K, u, dist, g_dist, W, gX);                                 \
    return hipGetLastError();
  switch (bucket) {
    CASE(4) CASE(5) CASE(8) CASE(10) CASE(16) CASE(20) CASE(24) CASE(32) CASE(40) CASE(48)
    CASE(64)
    default: return hipErrorInvalidValue;
  }
#undef CASE
}

}  // namespace

}  // namespace rtd

using namespace rtd;

extern "C" rtdetmcd_status rtdetmcd_backward(rtdetmcd_handle ctx, const void* X, int32_t dtype,
                                             int64_t n, int32_t p, int64_t ld, const double* mu,
                                             const double* sigma, const double* dist,
                                             const uint8_t* rew_mask, const int64_t* n_w,
                                             double c_rew, const double* g_dist,
                                             const double* g_mu, const double* g_sigma,
                                             double* g_X) {
  if (!ctx) return RTDETMCD_EINVAL;
  if (!X || !mu || !sigma || !dist || !rew_mask || !n_w || !g_X || n < 2 || p < 1 || ld < p ||
      (dtype != 0 && dtype != 1) || !(c_rew > 0.0)) {
    ctx->err = "rtdetmcd_backward: bad argument";
    return RTDETMCD_EINVAL;
  }
  if (p > RTDETMCD_MAX_P) return RTDETMCD_EUNSUPPORTED;
  RTD_HIP(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  // one item over all rows, for the weighted sscp about mu
  ItemSet S;
  ItemDesc d{};
  d.X = X; d.ld = ld; d.row0 = 0; d.m = n; d.h = n - 1; d.p = p; d.dtype = dtype; d.start = -1;
  S.add(d);
  Layout L0;
  size_t off[NOFF];
  layout_items(L0, S, off);
  const size_t o_P = L0.add(PMAX * PMAX * 8);
  const size_t o_K = L0.add(PMAX * PMAX * 8);
  const size_t o_u = L0.add(PMAX * 8);
  RTD_TRY(ensure_ws(ctx, L0.off));
  char* base = static_cast<char*>(ctx->ws);
  ItemDev D;
  bind_items(base, S, off, D);
  double* Pm = reinterpret_cast<double*>(base + o_P);
  double* Km = reinterpret_cast<double*>(base + o_K);
  double* uv = reinterpret_cast<double*>(base + o_u);
  Uploader up;
  up.add(D.items, S.items.data(), S.items.size());
  up.add(D.stiles, S.stiles.data(), S.stiles.size());
  RTD_TRY(up.flush(ctx));
  const int bucket = bucket_of(p);
  hipLaunchKernelGGL(k_bw_copy, dim3(1), dim3(64), 0, st, mu, p, D.A.mux);
  RTD_HIP(hipGetLastError());
  const double* part0 = nullptr;
  if (g_dist) {
    ItemArrays A = D.A;
    A.d2 = const_cast<double*>(dist);   // read only: the distances d_i
    RTD_HIP(launch_sscp(bucket, dtype, SSCP_ADJ, D.items, A, D.stiles, (int)S.stiles.size(),
                        SSCP_TILE, g_dist, nullptr, st));
    RTD_HIP(launch_collapse(D.items, A, 0, 1, S.max_ntiles(0, 1), 0, SSCP_TILE, st));
    part0 = D.A.part;   // the item's first tile
  }
  hipLaunchKernelGGL(k_bw_prep, dim3(1), dim3(BW_NT), 0, st, sigma, p, Pm);
  RTD_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_bw_mid, dim3(1), dim3(BW_NT), 0, st, part0, Pm, g_mu, g_sigma, n_w, c_rew,
                     p, uv, Km);
  RTD_HIP(hipGetLastError());
  if (dtype == 0)
    RTD_HIP(bw_rows_t<float>(bucket, static_cast<const float*>(X), n, ld, p, mu, Pm, Km, uv, dist,
                             g_dist, rew_mask, g_X, st));
  else
    RTD_HIP(bw_rows_t<double>(bucket, static_cast<const double*>(X), n, ld, p, mu, Pm, Km, uv,
                              dist, g_dist, rew_mask, g_X, st));
  return RTDETMCD_OK;
}
