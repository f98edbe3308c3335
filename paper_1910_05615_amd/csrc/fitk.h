// Kernels of the full fit (declarations).
#pragma once

#include "common.h"
#include "sortseg.h"
#include "../../include/rtdetmcd.h"

namespace rtd {

// Per-dataset device record.
struct DsInfo {
  const void* X;
  int64_t n, ld, m, h;
  int32_t p, dtype, q, glob1;   // glob1: second global item (final distances)
  double chi2p;      // chi2_{p, cutoff_q}
  double calpha;     // c(h/m) for p
  double crew;       // reweighted-scatter factor (1 or c(cutoff_q) for p)
  int32_t item0;     // first C-step item (2 per block)
  int32_t blk0;      // first block item
  int32_t glob0;     // first of the two global items
  int32_t err;       // 0 ok, else a status code
  const int32_t* perm;  // random partition: dataset row of block position k, or null
  int32_t* inv;         // its inverse: block position of dataset row i (valid perm only)
  const double* warm_mu;     // warm start (units of X), or null
  const double* warm_sigma;
};

// Per-dataset and per-block result arrays.
struct FitArrays {
  double* loc;       // [D*PMAX]
  double* scale;     // [D*PMAX]
  double* muraw;     // [D*PMAX]  aggregated raw fit, standardised units
  double* sigraw;    // [D*MSTRIDE]
  int64_t* nw;       // [D]
  double* bmu;       // [B*PMAX]   block raw fits (standardised), c(alpha) applied
  double* bsig;      // [B*MSTRIDE]
  double* bld;       // [B] log det of the block raw scatter
  double* bkl;       // [B] KL' key
  int32_t* bitem;    // [B] chosen C-step item or -1
  int32_t* bstat;    // [B]
  int32_t* bstart;   // [B]
  int32_t* biters;   // [B]
  int32_t* bds;      // [B] dataset of each block
  double* med;       // [D*(PMAX + MSTRIDE)] entrywise medians (mu then Sigma)
  double* vbuf;      // [I*MSTRIDE] eigenvectors of the initial scatter
  double* wbuf;      // [I*MSTRIDE] projection matrix of the refinement
  double* s2buf;     // [I*PMAX]    refined score variances
  double* rcnt;      // [I] reduced partial counts (block items)
  double* rsum;      // [I*PMAX]
  double* rS;        // [I*MSTRIDE]
};

// One dataset of a column-key launch: its n x p rows (stride ld) become p
// columns of order keys at `keys` (column j at keys + j n); a NaN or Inf
// sets *err = RTDETMCD_ENONFINITE.  tile0: its first block in the launch
// (CK tiles of 128 rows; jobs in increasing tile0).
struct ColJob {
  const void* X;
  void* keys;
  int32_t* err;
  int64_t n, ld;
  int64_t tile0;
  int32_t p, pad;
};
constexpr int COLKEY_ROWS = 128;   // rows per block of the column-key kernel
// Column-major order keys of the datasets of one element type (0 = f32 with
// 32-bit keys, 1 = f64 with 64-bit keys) for the standardisation sort.
hipError_t launch_colkeys(int dtype, const ColJob* jobs, int njobs, int64_t ntiles,
                          hipStream_t s);
hipError_t launch_std_finish(const SegStat* st32, const SegStat* st64, const int32_t* seg0,
                             const int32_t* in64, int D, DsInfo* ds, FitArrays F, hipStream_t s);
hipError_t launch_project(int bucket, int dtype, int mode, const ItemDesc* items,
                          const Tile* tiles, int ntiles, int tile_rows, const int32_t* status,
                          const double* W, const int64_t* kbase, uint64_t* keys, hipStream_t s);
hipError_t launch_reduce_partials(const ItemDesc* items, const double* part, int first, int n,
                                  double* cnt, double* sum, double* S, hipStream_t s);
hipError_t launch_init_cov(int mode, const ItemDesc* bitems, int first, int n, FitArrays F,
                           ItemArrays C, const DsInfo* ds, double* cut, const SegStat* gst,
                           hipStream_t s);
hipError_t launch_eig(int bucket, const ItemDesc* items, ItemArrays A, FitArrays F, int first,
                      int n, double kappa_max, hipStream_t s);
hipError_t launch_refine(int stage, const ItemDesc* items, ItemArrays A, FitArrays F, int first,
                         int n, const SegStat* st, const int32_t* seg0, hipStream_t s);
hipError_t launch_choose(const ItemDesc* bitems, const ItemDesc* citems, ItemArrays A,
                         FitArrays F, const DsInfo* ds, int first, int n, hipStream_t s);
hipError_t launch_median(const DsInfo* ds, FitArrays F, const int2* ent, int nent,
                         hipStream_t s);
hipError_t launch_kl(const DsInfo* ds, ItemArrays A, FitArrays F, int first_blk, int nblk,
                     int use_sinv, hipStream_t s);
hipError_t launch_pool(DsInfo* ds, ItemArrays G, FitArrays F, int first_ds, int nds, int pool_mode,
                       hipStream_t s);
hipError_t launch_rew(DsInfo* ds, const ItemDesc* gitems, ItemArrays G, FitArrays F, int first_ds,
                      int nds, hipStream_t s);
// form: per-item distance form of the items (ItemArrays::form), or null.
hipError_t launch_final_dist(int bucket, int dtype, int dense, const ItemDesc* items,
                             const Tile* tiles,
                             int ntiles, int tile_rows, const double* mtri, const double* mux,
                             const int32_t* form, const double* d2, const DsInfo* ds,
                             const struct rtdetmcd_out* outs, hipStream_t s);
// Random partition (Sec. 4) of dataset d: check that perm is a permutation
// of 0..n-1 (inv prefilled with -1 receives its inverse; a bad entry sets
// ds[d].err = RTDETMCD_EINVAL), and copy the q m fitted rows into Xp
// (row-major, row stride p) in block order; a bad entry copies zeros.
hipError_t launch_perm_check(const int32_t* perm, int64_t n, int32_t* inv, DsInfo* ds, int d,
                             hipStream_t s);
hipError_t launch_perm_gather(int dtype, const void* X, int64_t n, int64_t ld, int p,
                              const int32_t* perm, int64_t rows, void* Xp, hipStream_t s);
// Warm start (last paragraph of Sec. 4) of dataset d's q blocks: the first
// item of each block starts from (warm_mu, warm_sigma) in standardised units,
// the second is dropped.
hipError_t launch_warm_start(const DsInfo* ds, int d, int q, ItemArrays C, FitArrays F,
                             hipStream_t s);
hipError_t launch_hsub(const ItemDesc* citems, ItemArrays A, FitArrays F, const DsInfo* ds,
                       const struct rtdetmcd_out* outs, int first, int n, hipStream_t s);
hipError_t launch_outputs(const DsInfo* ds, ItemArrays G, FitArrays F,
                          const struct rtdetmcd_out* outs, int first_ds, int nds, hipStream_t s);
// The requested diagnostics of every block and dataset of a fit (the log
// det trace, the selection gap, the flag margin of rtdetmcd_out).
hipError_t launch_diag(const ItemDesc* citems, ItemArrays A, FitArrays F, const DsInfo* ds,
                       const struct rtdetmcd_out* outs, int nb, int nds, int maxs,
                       hipStream_t s);

}  // namespace rtd
