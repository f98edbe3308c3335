// Segmented sort and order-statistic estimators (declarations).
#pragma once

#include "common.h"

namespace rtd {

struct SegTile {
  int32_t seg;
  int32_t tile;
};

// One sort call: nseg segments of keys, segment s at [seg_off[s], +seg_len[s]).
struct SortPlan {
  int key_bytes = 8;            // 4: keys of float32 values, 8: keys of float64 values
  int nseg = 0;
  int ntiles = 0;
  void* keys = nullptr;         // in/out
  void* tmp = nullptr;          // ping-pong buffer of the same size
  const SegTile* tiles = nullptr;
  const int64_t* seg_off = nullptr;
  const int64_t* seg_len = nullptr;
  const int32_t* seg_tile0 = nullptr;   // [nseg + 1] first tile of each segment
  int32_t* counts = nullptr;    // [ntiles * 256]
  int32_t* offs = nullptr;      // [ntiles * 256]
};

struct SegStat {
  double mu_raw, var_raw, mu, var;
  int64_t start, n_kept;
};

enum : int { SEGSTAT_UNIMCD = 0, SEGSTAT_MEDMAD = 1, SEGSTAT_GSSCM = 2 };

int sort_tile_keys();
hipError_t sort_segments(SortPlan& P, hipStream_t s);
// UNIMCD: seg_craw[s] = c(h~/L) for p = 1, q1 = chi2_{1,q}, crew = c(q) for p = 1.
// MEDMAD: mu = median, var = (1.4826 MAD)^2.  GSSCM: mu = A, var = B.
hipError_t launch_segstats(const SortPlan& P, const double* seg_craw, double q1, double crew,
                           int mode, SegStat* out, hipStream_t s);

}  // namespace rtd
