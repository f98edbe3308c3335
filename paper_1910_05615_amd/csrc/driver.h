// Host driver pieces shared by the C entry points: workspace layout, uploads
// through pinned staging, item tables and the C-step loop.
#pragma once

#include <cstring>
#include <string>
#include <vector>

#include "../../include/rtdetmcd.h"
#include "host_util.h"

namespace rtd {

constexpr int DIST_TILE = 1024;   // rows per block of the distance kernel
constexpr int SSCP_TILE = 1024;   // candidate rows per block of the sscp kernel

#define RTD_HIP(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);                \
      return RTDETMCD_EDEVICE;                                                     \
    }                                                                              \
  } while (0)

#define RTD_TRY(expr)                     \
  do {                                    \
    rtdetmcd_status s_ = (expr);          \
    if (s_ != RTDETMCD_OK) return s_;     \
  } while (0)

struct Layout {
  size_t off = 0;
  size_t add(size_t bytes) {
    const size_t o = (off + 255) & ~(size_t)255;
    off = o + (bytes ? bytes : 1);
    return o;
  }
};

rtdetmcd_status ensure_ws(rtdetmcd_ctx* ctx, size_t bytes);
void drop_graphs(rtdetmcd_ctx* ctx);   // destroy the captured C-step rounds

// Collects host->device copies and issues them from pinned staging.
struct Uploader {
  struct E { void* dst; size_t off; size_t bytes; };
  std::vector<E> ents;
  std::vector<char> buf;
  template <typename T>
  void add(void* dst, const T* src, size_t n) {
    const size_t bytes = n * sizeof(T);
    const size_t off = (buf.size() + 15) & ~(size_t)15;
    buf.resize(off + bytes);
    if (bytes) std::memcpy(buf.data() + off, src, bytes);
    ents.push_back({dst, off, bytes});
  }
  rtdetmcd_status flush(rtdetmcd_ctx* ctx);
};

// Items of one C-step run plus their tile tables (host copies kept for
// per-item launches).
struct ItemSet {
  std::vector<ItemDesc> items;
  std::vector<Tile> dtiles, stiles;
  std::vector<int> dt_first, dt_count;   // per item, into dtiles
  int64_t rows = 0;                      // sum of m
  int32_t ldtr_n = 0;                    // log det trace entries per item (0: none kept)
  void add(const ItemDesc& d) {
    ItemDesc e = d;
    e.roff = rows;
    e.tile0 = (int)stiles.size();
    const int ns = (int)((e.m + SSCP_TILE - 1) / SSCP_TILE);
    e.ntiles = ns < 1 ? 1 : ns;
    for (int t = 0; t < e.ntiles; ++t) stiles.push_back({(int)items.size(), t});
    dt_first.push_back((int)dtiles.size());
    const int nd = (int)((e.m + DIST_TILE - 1) / DIST_TILE);
    for (int t = 0; t < nd; ++t) dtiles.push_back({(int)items.size(), t});
    dt_count.push_back(nd);
    rows += e.m;
    items.push_back(e);
  }
  int max_ntiles(int a, int b) const {   // over items [a, b)
    int r = 0;
    for (int i = a; i < b; ++i) r = items[i].ntiles > r ? items[i].ntiles : r;
    return r;
  }
  // Items [a, b) all hold dense rows of exactly `bucket` columns (ld == p ==
  // bucket) at a base aligned for whole-row vector loads: the distance
  // kernels then take their row-load path only.
  bool rows_dense(int a, int b, int bucket) const {
    for (int i = a; i < b; ++i)
      if (!rows_dense_at(items[i].X, items[i].ld, items[i].p, items[i].dtype, bucket)) return false;
    return true;
  }
};

// Device copies of an ItemSet and its state arrays inside the workspace.
struct ItemDev {
  ItemDesc* items = nullptr;
  Tile* dtiles = nullptr;
  Tile* stiles = nullptr;
  ItemArrays A{};
};

constexpr int NOFF = 22;   // workspace offsets of one item set
void layout_items(Layout& L, const ItemSet& S, size_t off[NOFF]);
void bind_items(char* base, const ItemSet& S, const size_t off[NOFF], ItemDev& D);

// Enqueue the C-step loop for items [first, first+n) of a bucket/dtype class.
// Batched: all items in each launch, host checks convergence every
// rounds_per_sync steps.  Plain: one item at a time, host check every step.
rtdetmcd_status run_csteps(rtdetmcd_ctx* ctx, const ItemSet& S, ItemDev& D, int bucket, int dtype,
                           int first, int n, const rtdetmcd_opts& o, int32_t* pin_flag);

rtdetmcd_status check_opts(rtdetmcd_ctx* ctx, const rtdetmcd_opts* in, rtdetmcd_opts& o);

// Kernel timing: while rtdetmcd_profile is on (and no graph is being
// captured), a ProfMark records a HIP event on the launching stream before
// a launch and another after it (end), with the launch's algorithmic bytes
// and flops.  Off, it does nothing.
struct ProfMark {
  rtdetmcd_ctx* ctx = nullptr;
  int idx = -1;
  ProfMark(rtdetmcd_ctx* c, int kind, hipStream_t s, double bytes, double flops_useful = 0.0,
           double flops_exec = 0.0);
  void end(hipStream_t s);
};

// Start of rtdetmcd_cstep: (mu0, sigma0) divided by the condition-check
// scales into the item's muz / sigz, loc = 0 and scale = kscale (or 1).
hipError_t launch_cstep_init(const double* mu0, const double* sigma0, const double* kscale,
                             int p, const ItemArrays& A, double* loc, double* scale,
                             hipStream_t s);
// End of rtdetmcd_cstep: the item's mean, covariance (lamx / (h-1)), status,
// iterations and log det in data units (NaN for a dropped start).
hipError_t launch_cstep_out(const ItemArrays& A, const double* scale, int p, double h_sub,
                            double* mu, double* sigma, int32_t* status, int32_t* iters,
                            double* logdet, hipStream_t s);

// Address of this device's allocation-free scratch array (rtdetmcd_cstep_noalloc),
// looked up once per device; null (and *bytes = 0) if the lookup failed.
void* noalloc_scratch(int device, size_t* bytes);

}  // namespace rtd
