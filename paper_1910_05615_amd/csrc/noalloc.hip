// Allocation-free C-step entry point (rtdetmcd_cstep_noalloc): the C-steps of
// rtdetmcd_cstep with every piece of device memory beyond the caller's inputs
// and outputs taken from a fixed file-scope array, for callers that cannot
// allocate (code under stream capture, tight serving loops).
#include <algorithm>
#include <mutex>
#include <string>

#include "driver.h"

namespace rtd {
namespace {

// Fixed scratch: item table, tile tables, per-item state (p x p matrices at
// a row stride of PMAX), per-row distances, mask and swap list, and the sscp
// tile partials of one block of at most NOALLOC_MAX_M rows.
constexpr size_t NOALLOC_BYTES = (size_t)8 << 20;
constexpr int64_t NOALLOC_MAX_M = 131072;
__device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

// Device address of `scratch`, per device.  In host code the array's name is
// only a host-side stand-in: kernels and copies take this address.
constexpr int MAX_DEV = 64;
std::mutex g_mu;
bool g_done[MAX_DEV];
void* g_ptr[MAX_DEV];

// Item table and tile tables written from kernel arguments (no staging copy).
__global__ void k_noalloc_tables(ItemDesc d, ItemDesc* __restrict__ items,
                                 Tile* __restrict__ dtiles, int ndt, Tile* __restrict__ stiles,
                                 int nst) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) items[0] = d;
  if (t < ndt) dtiles[t] = Tile{0, t};
  if (t < nst) stiles[t] = Tile{0, t};
}

}  // namespace

void* noalloc_scratch(int device, size_t* bytes) {
  *bytes = 0;
  if (device < 0 || device >= MAX_DEV) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_done[device]) {
    // the caller (rtdetmcd_create) has made `device` current
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
    g_ptr[device] = p;
    g_done[device] = true;
  }
  if (g_ptr[device]) *bytes = NOALLOC_BYTES;
  return g_ptr[device];
}

}  // namespace rtd

using namespace rtd;

extern "C" rtdetmcd_status rtdetmcd_cstep_noalloc(
    rtdetmcd_handle ctx, const void* X, int32_t dtype, int64_t m, int32_t p, int64_t ld,
    int64_t h_sub, const double* mu0, const double* sigma0, const double* kappa_scale,
    const rtdetmcd_opts* o_in, double* mu, double* sigma, int32_t* hsubset, int32_t* status,
    int32_t* iters, double* logdet) {
  if (!ctx) return RTDETMCD_EINVAL;
  rtdetmcd_opts o;
  RTD_TRY(check_opts(ctx, o_in, o));
  o.graph = 0;   // capturing a graph allocates
  o.tune = 0;    // so does a tuned plan
  if (!X || !mu0 || !sigma0 || p < 1 || ld < p || !(h_sub > p && h_sub < m) ||
      (dtype != 0 && dtype != 1)) {
    ctx->err = "rtdetmcd_cstep_noalloc: bad argument (need p < h < m)";
    return RTDETMCD_EINVAL;
  }
  if (p > RTDETMCD_MAX_P) return RTDETMCD_EUNSUPPORTED;
  if (m > NOALLOC_MAX_M) {
    ctx->err = "rtdetmcd_cstep_noalloc: m = " + std::to_string(m) + " exceeds the limit of " +
               std::to_string(NOALLOC_MAX_M) + " rows";
    return RTDETMCD_EINVAL;
  }
  if (!ctx->scratch) {
    ctx->err = "rtdetmcd_cstep_noalloc: no scratch array on this device";
    return RTDETMCD_EDEVICE;
  }
  RTD_HIP(hipSetDevice(ctx->device));
  ItemSet S;
  ItemDesc d{};
  d.X = X; d.ld = ld; d.row0 = 0; d.m = m; d.h = h_sub; d.p = p; d.dtype = dtype; d.start = -1;
  S.add(d);
  Layout L0;
  size_t off[NOFF];
  layout_items(L0, S, off);
  const size_t o_loc = L0.add(PMAX * 8), o_scale = L0.add(PMAX * 8);
  if (L0.off > ctx->scratch_bytes) {   // cannot happen for m <= NOALLOC_MAX_M
    ctx->err = "rtdetmcd_cstep_noalloc: scratch array too small";
    return RTDETMCD_EINVAL;
  }
  char* base = static_cast<char*>(ctx->scratch);
  ItemDev D;
  bind_items(base, S, off, D);
  double* loc = reinterpret_cast<double*>(base + o_loc);
  double* scale = reinterpret_cast<double*>(base + o_scale);
  S.items[0].loc = loc;
  S.items[0].scale = scale;
  hipStream_t st = ctx->stream;
  const int ndt = (int)S.dtiles.size(), nst = (int)S.stiles.size();
  const int nt = std::max(ndt, nst);
  hipLaunchKernelGGL(k_noalloc_tables, dim3((nt + 255) / 256), dim3(256), 0, st, S.items[0],
                     D.items, D.dtiles, ndt, D.stiles, nst);
  RTD_HIP(hipGetLastError());
  RTD_HIP(launch_cstep_init(mu0, sigma0, kappa_scale, p, D.A, loc, scale, st));
  RTD_HIP(launch_fill_i32(D.A.status, ACTIVE, 1, st));
  RTD_HIP(launch_fill_i32(D.A.iter, 0, 1, st));
  RTD_HIP(launch_fill_u8(D.A.mask, 0, m, st));
  RTD_TRY(run_csteps(ctx, S, D, bucket_of(p), dtype, 0, 1, o, ctx->flag));
  RTD_HIP(launch_cstep_out(D.A, scale, p, (double)h_sub, mu, sigma, status, iters, logdet, st));
  if (hsubset) RTD_HIP(launch_extract_subset(D.items, D.A, 0, 1, hsubset, h_sub, 0, st));
  return RTDETMCD_OK;
}
