// Internal declarations shared by the librtdetmcd HIP sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace rtd {

constexpr int PMAX = 64;                 // largest supported p
constexpr int MSTRIDE = PMAX * PMAX;     // per-item stride of p x p matrices
constexpr int TRI = PMAX * (PMAX + 1) / 2;  // packed lower triangle
constexpr int ACTIVE = -1;               // item still iterating

// Status values (same numbering as the public header).
constexpr int ST_CONVERGED = 0, ST_NOTCONV = 1, ST_ILLCOND = 2, ST_DROP_REFINE = 3,
              ST_DROP_FIRST = 4, ST_SINGULAR = 5;

// One C-step work item: a (dataset, block, start) triple, or a plain row set
// (reweighting, final scoring, low-level calls) with start = -1.
struct ItemDesc {
  const void* X;     // dataset base (device), row-major
  int64_t ld;        // row stride in elements
  int64_t row0;      // first dataset row of the block
  int64_t m;         // rows of the block
  int64_t h;         // subset size
  int64_t roff;      // offset of this item's rows in the per-row work arrays
  const double* loc;    // [p] standardisation location of the dataset
  const double* scale;  // [p] standardisation scale of the dataset
  int32_t p;
  int32_t dtype;     // 0 = f32, 1 = f64
  int32_t ds;        // dataset index
  int32_t blk;       // block index within the dataset
  int32_t start;     // 0 = wrapping start, 1 = GSSCM start, -1 = none
  int32_t tile0;     // first tile of this item in the SSCP tile table
  int32_t ntiles;    // number of SSCP tiles of this item
  int32_t pad;
};

// Per-item state (device arrays, item-major).
struct ItemArrays {
  int32_t* status;   // [I] ACTIVE or a terminal status
  int32_t* iter;     // [I] C-steps evaluated
  int32_t* kswap;    // [I] rows that entered the subset in the last step
  int32_t* full;     // [I] 1: next statistics are recomputed in full
  double* logdet;    // [I] log det of the current scatter (standardised units)
  double* mux;       // [I*PMAX] current mean, data units
  double* lamx;      // [I*MSTRIDE] sscp about mux, data units
  double* muz;       // [I*PMAX] current mean, standardised units
  double* sigz;      // [I*MSTRIDE] current covariance, standardised units
  double* linv;      // [I*MSTRIDE] inverse Cholesky factor of sigz
  double* mtri;      // [I*MSTRIDE] L^{-1} D^{-1} (lower, row stride PMAX): distances in data units
  double* d2;        // [rows] squared distances
  uint8_t* mask;     // [rows] current subset
  int32_t* swap;     // [rows] entering rows from 0, leaving rows from m/2
  double* part;      // [tiles * PSTRIDE] SSCP tile partials
  int32_t* nactive;  // [1] items still active after the last finalize
  int32_t* form;     // [I] 0: mtri holds L^{-1} D^{-1}; 1: the packed explicit inverse P~
  double* sinv;      // [I*MSTRIDE] inverse of lamx (data units), kept by the single-swap mode
  double* ldtr;      // [I*ldtr_n] log det of the scatter at each evaluated C-step, or null
  int32_t ldtr_n;    // entries per item (the C-step limit)
};

constexpr int PSTRIDE = 1 + PMAX + TRI;  // count, sum, packed sscp

// Row-source modes of the SSCP kernel.
enum SscpMode : int {
  SSCP_CSTEP = 0,    // subset rows (full) or swapped rows (update), about mux
  SSCP_D2CUT = 1,    // rows with d2 <= cut, about the item's mean (reweighting)
  SSCP_WRAP = 2,     // all rows, wrapped standardised values, about 0
  SSCP_GSSCM = 3,    // all rows, standardised values weighted by xi^2(||z||)
  SSCP_ADJ = 4,      // all rows about the item's mean, weight wsrc_i / d_i (0 if d_i = 0)
};

struct Tile {
  int32_t item;
  int32_t t;         // tile index within the item
};

inline int bucket_of(int p) {
  if (p <= 4) return 4;
  if (p <= 5) return 5;
  if (p <= 8) return 8;
  if (p <= 10) return 10;
  if (p <= 16) return 16;
  if (p <= 20) return 20;
  if (p <= 24) return 24;
  if (p <= 32) return 32;
  if (p <= 40) return 40;
  if (p <= 48) return 48;
  return 64;
}

// Launch helpers implemented in the .hip files (all enqueue on `s`).
// Largest power-of-two load (16, 8 or the element size) that divides a row of
// `bucket` elements: the distance kernels read whole rows with it.
inline int dist_row_align(int bucket, int dtype) {
  const int es = dtype == 0 ? 4 : 8;
  const int bytes = bucket * es;
  return bytes % 16 == 0 ? 16 : bytes % 8 == 0 ? 8 : es;
}
inline bool rows_dense_at(const void* X, int64_t ld, int p, int dtype, int bucket) {
  return p == bucket && ld == p &&
         reinterpret_cast<uintptr_t>(X) % (uintptr_t)dist_row_align(bucket, dtype) == 0;
}
// dense: every item of the launch satisfies rows_dense_at (the kernels then
// skip the per-element path for narrower or strided rows).  One item per
// tile: the C-step pass runs over both starts' items of a block, reading
// each row twice (10^6 x 20: 35 against 37 us for one read feeding both
// factors; x 40: 130 against 154).
// form: per-item distance form (ItemArrays::form), or null when every item
// holds L^{-1} D^{-1} (the launch then takes the kernels without the
// explicit-inverse evaluation).
hipError_t launch_dist(int bucket, int dtype, int dense, const ItemDesc* items,
                       const Tile* tiles,
                       int ntiles, int tile_rows, const double* mtri, const double* mux,
                       const int32_t* status, const int32_t* form, double* d2, hipStream_t s);
// max_m: largest m among the items (picks the register-resident variant).
// reset_nactive: the first block zeroes *A.nactive before anything else (the
// C-step loop counts the items left active by the step's finalize).
hipError_t launch_select(const ItemDesc* items, ItemArrays A, int first_item, int nitems,
                         int64_t max_m, int cstep_mode, hipStream_t s, int reset_nactive = 0);
// wsrc: per-row cotangents of SSCP_ADJ (rows indexed like d2), else unused.
hipError_t launch_sscp(int bucket, int dtype, int mode, const ItemDesc* items, ItemArrays A,
                       const Tile* tiles, int ntiles, int tile_rows, const double* wsrc,
                       const double* cut, hipStream_t s);
// Sums each item's sscp tile partials into the partial of its first tile
// (every consumer of the partials reads that one only).  cstep: the partials
// come from the C-step sscp (valid tiles depend on full/kswap, inactive
// items skipped).  max_ntiles: largest ntiles among the items.
hipError_t launch_collapse(const ItemDesc* items, ItemArrays A, int first, int nitems,
                           int max_ntiles, int cstep, int tile_rows, hipStream_t s);
// bucket: a p bucket (bucket_of) no smaller than any item's p.
// cstep_mode: RTDETMCD_CSTEP_*; with RTDETMCD_CSTEP_SMW a step that swapped
// one row in and one out takes the single-swap update (Sec. 3.5) and the
// inverse form.  dist_form: 1 writes the explicit-inverse form P~ for every
// other step too (the distance switch), 0 the Cholesky form.
hipError_t launch_finalize(int bucket, const ItemDesc* items, ItemArrays A, int first_item,
                           int nitems, int from_start, int max_csteps, double kappa_max,
                           int cstep_mode, int dist_form, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
// stage: n records (dst, offset, bytes) of 3 uint64 each, then the payload at
// those offsets from stage; copies every record's bytes to its dst.
hipError_t launch_upload_scatter(const void* stage, int n, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t s);
hipError_t launch_chol_factor(const double* sigma, int p, double* mtri, hipStream_t s);
hipError_t launch_extract_subset(const ItemDesc* items, ItemArrays A, int first_item, int nitems,
                                 int32_t* out, int64_t out_stride, int global_rows,
                                 hipStream_t s);
hipError_t launch_score(int bucket, int dtype, const void* X, int64_t n, int64_t ld, int p,
                        const double* mu, const double* M, int ldm, double cut, double* dist,
                        uint8_t* flag, hipStream_t s);

}  // namespace rtd
