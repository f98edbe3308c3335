// Segmented sort and order-statistic estimators (declarations).
#pragma once

#include <algorithm>

#include "common.h"

namespace rtd {

struct SegTile {
  int32_t seg;
  int32_t tile;
};

// Scratch of the multi-block univariate MCD (per tile / per segment arrays).
struct MbScratch {
  double *bs1, *bs2;     // [ntiles] block sums, then exclusive prefixes
  double *wbest;         // [ntiles] smallest window criterion hd s2 - s1^2 per block
  int64_t* wj;           // [ntiles] its window start
  double *k0, *k1, *k2;  // [ntiles] kept-row partial sums
  double* tot;           // [2 nseg] segment totals
  double* prm;           // [5 nseg] per-segment parameters
};

// One sort call: nseg segments of keys, segment s at [seg_off[s], +seg_len[s]).
struct SortPlan {
  const MbScratch* mb = nullptr;   // device pointers, for the multi-block estimator
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
  int tile_first = 0;           // absolute index of tiles[0] (seg_tile0 holds absolute indices)
  int safe = 0;                 // 1: rank equal digits with ballots, not LDS atomics
  int32_t* flag = nullptr;      // set to 1 when a sorted segment is found out of order
  int seg_first = 0;            // absolute index of the first segment of the plan
  // Buckets of the sample sort (sort_buckets): segment s owns the buckets
  // [bk0[s], bk0[s + 1]) (absolute), bucket j is (bk_tab[j].seg, bk_tab[j].tile =
  // its rank within the segment).  Of a plan, buckets [bk_first, + nbk).
  const int32_t* bk0 = nullptr;     // [nseg + 1]
  const SegTile* bk_tab = nullptr;
  int bk_first = 0;
  int nbk = 0;
  int bk_max = 0;                   // most buckets of one segment
  // The plan restricted to segments [a, b): pointers offset, tile and
  // bucket counts given by the host copies of the absolute seg_tile0 and
  // bk0 tables.
  SortPlan sub(int a, int b, const int32_t* host_seg_tile0, const int32_t* host_bk0) const {
    SortPlan r = *this;
    const int ta = host_seg_tile0[a], tb = host_seg_tile0[b];
    r.nseg = b - a;
    r.ntiles = tb - ta;
    r.tiles = tiles + ta;
    // tiles carry absolute segment ids, so seg_off / seg_len stay absolute;
    // kernels that index segments by block use seg_first
    r.seg_first = seg_first + a;
    r.seg_tile0 = seg_tile0 + a;
    r.counts = counts + (size_t)ta * 256;
    r.offs = offs + (size_t)ta * 256;
    r.tile_first = ta;
    r.bk_first = host_bk0[a];
    r.nbk = host_bk0[b] - host_bk0[a];
    r.bk_max = 0;
    for (int k = a; k < b; ++k) r.bk_max = std::max(r.bk_max, host_bk0[k + 1] - host_bk0[k]);
    return r;
  }
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
// Sort and estimator in one launch for plans whose segments all hold at most
// lds_sort_capacity() keys (the sort happens in LDS; P.keys is left unsorted).
int lds_sort_capacity();
// Univariate MCD over sorted segments of any length, spread over the tiles.
hipError_t launch_unimcd_multiblock(const SortPlan& P, const double* seg_craw, double q1,
                                    double crew, SegStat* out, hipStream_t s);
hipError_t launch_seg_lds(const SortPlan& P, const double* seg_craw, double q1, double crew,
                          int mode, SegStat* out, int64_t max_len, hipStream_t s);

// Sample sort of segments of at most bucket_max_len() keys (P.keys sorted
// in place): bucket_count(L) buckets per segment of L keys,
// each sorted in LDS, with P.tmp holding nbk * bucket_capacity() keys and
// P.counts at least 5 nbk ints.  A bucket that outgrows its capacity sets
// *P.flag (the caller then sorts again with the radix passes).
int64_t bucket_count(int64_t L);
int bucket_capacity();
int64_t bucket_max_len();
hipError_t sort_buckets(SortPlan& P, hipStream_t s);

}  // namespace rtd
