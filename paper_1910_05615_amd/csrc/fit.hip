// Host orchestration of the RT-DetMCD fit (Sec. 4 steps 1-10) for one or
// many datasets.  Every step runs in the library's kernels; the host only
// builds tables, enqueues launches and reads convergence words.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "driver.h"
#include "fitk.h"
#include "sortseg.h"

namespace rtd {
namespace {

struct DsHost {
  const rtdetmcd_dataset* in;
  const int32_t* perm;   // random partition (Sec. 4), or null for contiguous blocks
  bool warm;             // warm start (last paragraph of Sec. 4)
  int p, dtype, bucket, q;
  int64_t n, m, h, ld;
  double chi2p, calpha, crew;
  int item0, blk0, glob0;
};

// Host description of one sort call (segments and their tiles).
struct SortHost {
  int key_bytes = 8;
  std::vector<int64_t> off, len;
  std::vector<int32_t> tile0;     // nseg + 1, absolute
  std::vector<SegTile> tiles;
  std::vector<double> craw;
  std::vector<int32_t> bk0;       // nseg + 1: buckets of the sample sort, absolute
  std::vector<SegTile> bktab;     // (segment, rank within it) of every bucket
  int64_t keys = 0;               // total keys
  int64_t maxlen = 0;
  bool buckets = false;           // the sample sort may take the long segments
  void add(int64_t L, double cr) {
    const int T = sort_tile_keys();
    if (tile0.empty()) tile0.push_back(0);
    if (bk0.empty()) bk0.push_back(0);
    const int64_t nb = bucket_count(L);
    for (int64_t b = 0; b < nb; ++b) bktab.push_back({(int)off.size(), (int)b});
    bk0.push_back((int32_t)bktab.size());
    maxlen = std::max(maxlen, L);
    off.push_back(keys);
    len.push_back(L);
    craw.push_back(cr);
    const int nt = (int)std::max<int64_t>(1, (L + T - 1) / T);
    for (int t = 0; t < nt; ++t) tiles.push_back({(int)off.size() - 1, t});
    tile0.push_back((int32_t)tiles.size());
    keys += L;
  }
  int nseg() const { return (int)off.size(); }
  // Staging keys of the sample sort (zero where it cannot be used): a
  // plan with a segment too long for one LDS segment and none too long for
  // the buckets.
  int64_t bucket_keys() const {
    if (!buckets || maxlen <= lds_sort_capacity() || maxlen > bucket_max_len()) return 0;
    return (int64_t)bktab.size() * bucket_capacity();
  }
};

struct SortDev {
  SortPlan plan;
  SegStat* st = nullptr;
  double* craw = nullptr;
  size_t o_off = 0, o_len = 0, o_t0 = 0, o_tiles = 0, o_st = 0, o_craw = 0, o_bk0 = 0, o_bkt = 0;
};

void layout_sort(Layout& L, const SortHost& H, SortDev& D) {
  D.o_off = L.add(H.off.size() * 8);
  D.o_len = L.add(H.len.size() * 8);
  D.o_t0 = L.add(H.tile0.size() * 4);
  D.o_tiles = L.add(H.tiles.size() * sizeof(SegTile));
  D.o_st = L.add(H.off.size() * sizeof(SegStat));
  D.o_craw = L.add(H.craw.size() * 8);
  D.o_bk0 = L.add(H.bk0.size() * 4);
  D.o_bkt = L.add(H.bktab.size() * sizeof(SegTile));
}

void bind_sort(char* base, const SortHost& H, SortDev& D, void* keys, void* tmp, int32_t* counts,
               int32_t* offs) {
  SortPlan& P = D.plan;
  P.key_bytes = H.key_bytes;
  P.nseg = H.nseg();
  P.ntiles = (int)H.tiles.size();
  P.keys = keys;
  P.tmp = tmp;
  P.tiles = reinterpret_cast<SegTile*>(base + D.o_tiles);
  P.seg_off = reinterpret_cast<int64_t*>(base + D.o_off);
  P.seg_len = reinterpret_cast<int64_t*>(base + D.o_len);
  P.seg_tile0 = reinterpret_cast<int32_t*>(base + D.o_t0);
  P.counts = counts;
  P.offs = offs;
  P.tile_first = 0;
  P.bk0 = reinterpret_cast<int32_t*>(base + D.o_bk0);
  P.bk_tab = reinterpret_cast<SegTile*>(base + D.o_bkt);
  P.bk_first = 0;
  P.nbk = (int)H.bktab.size();
  P.bk_max = 0;
  for (size_t k = 0; k + 1 < H.bk0.size(); ++k) P.bk_max = std::max(P.bk_max, H.bk0[k + 1] - H.bk0[k]);
  D.st = reinterpret_cast<SegStat*>(base + D.o_st);
  D.craw = reinterpret_cast<double*>(base + D.o_craw);
}

void upload_sort(Uploader& up, const SortHost& H, SortDev& D) {
  up.add(const_cast<int64_t*>(D.plan.seg_off), H.off.data(), H.off.size());
  up.add(const_cast<int64_t*>(D.plan.seg_len), H.len.data(), H.len.size());
  up.add(const_cast<int32_t*>(D.plan.seg_tile0), H.tile0.data(), H.tile0.size());
  up.add(const_cast<SegTile*>(D.plan.tiles), H.tiles.data(), H.tiles.size());
  up.add(D.craw, H.craw.data(), H.craw.size());
  up.add(const_cast<int32_t*>(D.plan.bk0), H.bk0.data(), H.bk0.size());
  up.add(const_cast<SegTile*>(D.plan.bk_tab), H.bktab.data(), H.bktab.size());
}

// Sort + estimator over the segments [a, b) of a plan.
rtdetmcd_status sort_stats(rtdetmcd_ctx* ctx, const SortHost& H, SortDev& D, int a, int b,
                           int mode, double q1, double crew1) {
  if (b <= a) return RTDETMCD_OK;
  SortPlan P = D.plan.sub(a, b, H.tile0.data(), H.bk0.data());
  const int64_t maxlen = *std::max_element(H.len.begin() + a, H.len.begin() + b);
  if (maxlen <= lds_sort_capacity()) {
    double keys = 0.0;
    for (int k = a; k < b; ++k) keys += (double)H.len[k];
    ProfMark pm(ctx, RTDETMCD_PROF_SEGSORT, ctx->stream,
                keys * H.key_bytes + (double)(b - a) * sizeof(SegStat));
    RTD_HIP(launch_seg_lds(P, D.craw + a, q1, crew1, mode, D.st + a, maxlen, ctx->stream));
    pm.end(ctx->stream);
    return RTDETMCD_OK;
  }
  if (H.bucket_keys() > 0 && !ctx->sort_safe)
    RTD_HIP(sort_buckets(P, ctx->stream));
  else
    RTD_HIP(sort_segments(P, ctx->stream));
  if (mode == SEGSTAT_UNIMCD)
    RTD_HIP(launch_unimcd_multiblock(P, D.craw + a, q1, crew1, D.st + a, ctx->stream));
  else
    RTD_HIP(launch_segstats(P, D.craw + a, q1, crew1, mode, D.st + a, ctx->stream));
  return RTDETMCD_OK;
}

struct Group {   // datasets sharing a kernel instantiation (p bucket, dtype)
  int bucket, dtype;
  int ds0, ds1;          // dataset range (in fit order)
  int c0, c1;            // C-step items
  int b0, b1;            // block items
  bool all_warm;         // every dataset warm-started: no starts to compute
};

}  // namespace

rtdetmcd_status fit_many(rtdetmcd_ctx* ctx, int nd, const rtdetmcd_dataset* sets,
                         const rtdetmcd_opts& o, rtdetmcd_status* status) {
  hipStream_t st = ctx->stream;
  RTD_HIP(hipSetDevice(ctx->device));
  // ---------------------------------------------------------------- plan
  std::vector<DsHost> dsh;
  std::vector<int> order;
  for (int i = 0; i < nd; ++i) {
    const rtdetmcd_dataset& s = sets[i];
    if (status) status[i] = RTDETMCD_OK;
    int32_t q;
    int64_t m, h;
    rtdetmcd_status ps = rtdetmcd_plan(s.n, s.p, s.h_sub, s.n_chunks, &o, &q, &m, &h);
    if (ps == RTDETMCD_OK && (!s.X || s.ld < s.p || (s.dtype != 0 && s.dtype != 1) ||
                              (!s.warm_mu) != (!s.warm_sigma)))
      ps = RTDETMCD_EINVAL;
    if (ps != RTDETMCD_OK) {
      if (status) status[i] = ps;
      ctx->err = "dataset " + std::to_string(i) + ": invalid sizes or pointers";
      if (nd == 1) return ps;
      continue;
    }
    DsHost d{};
    d.in = &s;
    d.perm = s.perm;
    d.warm = s.warm_mu != nullptr;
    d.p = s.p;
    d.dtype = s.dtype;
    d.bucket = bucket_of(s.p);
    d.q = q;
    d.n = s.n;
    d.m = m;
    d.h = h;
    d.ld = s.ld;
    d.chi2p = chi2_quantile_memo(o.cutoff_q, s.p);
    d.calpha = consistency_memo((double)h / (double)m, s.p);
    d.crew = o.rew_consistency ? consistency_memo(o.cutoff_q, s.p) : 1.0;
    order.push_back((int)dsh.size());
    dsh.push_back(d);
  }
  if (dsh.empty()) return RTDETMCD_EINVAL;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (dsh[a].bucket != dsh[b].bucket) return dsh[a].bucket < dsh[b].bucket;
    return dsh[a].dtype < dsh[b].dtype;
  });
  std::vector<DsHost> D;
  for (int i : order) D.push_back(dsh[i]);
  const int ND = (int)D.size();

  ItemSet C, B, G;
  std::vector<Group> groups;
  for (int k = 0; k < ND; ++k) {
    DsHost& d = D[k];
    if (groups.empty() || groups.back().bucket != d.bucket || groups.back().dtype != d.dtype)
      groups.push_back({d.bucket, d.dtype, k, k, (int)C.items.size(), (int)C.items.size(),
                        (int)B.items.size(), (int)B.items.size(), true});
    groups.back().all_warm = groups.back().all_warm && d.warm;
    d.item0 = (int)C.items.size();
    d.blk0 = (int)B.items.size();
    for (int l = 0; l < d.q; ++l) {
      ItemDesc e{};
      e.X = d.in->X; e.ld = d.ld; e.row0 = (int64_t)l * d.m; e.m = d.m; e.h = d.h;
      e.p = d.p; e.dtype = d.dtype; e.ds = k; e.blk = l;
      e.start = -1;
      B.add(e);
      e.start = 0;
      C.add(e);
      e.start = 1;
      C.add(e);
    }
    Group& g = groups.back();
    g.ds1 = k + 1;
    g.c1 = (int)C.items.size();
    g.b1 = (int)B.items.size();
  }
  // global items: [0, ND) reweighting rows (q m), [ND, 2 ND) all rows
  for (int k = 0; k < ND; ++k) {
    ItemDesc e{};
    e.X = D[k].in->X; e.ld = D[k].ld; e.row0 = 0; e.m = (int64_t)D[k].q * D[k].m; e.h = 0;
    e.p = D[k].p; e.dtype = D[k].dtype; e.ds = k; e.blk = -1; e.start = -1;
    G.add(e);
    D[k].glob0 = k;
  }
  for (int k = 0; k < ND; ++k) {
    ItemDesc e{};
    e.X = D[k].in->X; e.ld = D[k].ld; e.row0 = 0; e.m = D[k].n; e.h = 0;
    e.p = D[k].p; e.dtype = D[k].dtype; e.ds = k; e.blk = -1; e.start = -1;
    G.add(e);
  }
  const int NB = (int)B.items.size(), NC = (int)C.items.size(), NG = (int)G.items.size();

  // sort plans
  SortHost S32, S64, SN, SR;
  S32.key_bytes = 4;
  S64.key_bytes = 8;
  SN.key_bytes = 8;
  SR.key_bytes = 8;
  S32.buckets = S64.buckets = SN.buckets = SR.buckets = true;
  std::vector<int32_t> std_seg0(ND);
  std::vector<int> std_in64(ND);
  for (int k = 0; k < ND; ++k) {
    SortHost& Hs = D[k].dtype == 0 ? S32 : S64;
    std_in64[k] = D[k].dtype;
    std_seg0[k] = Hs.nseg();
    const double cr = consistency_memo((double)(D[k].n / 2 + 1) / (double)D[k].n, 1);
    for (int j = 0; j < D[k].p; ++j) Hs.add(D[k].n, cr);
  }
  std::vector<int64_t> nkbase(NB), rkbase(NC);
  std::vector<int32_t> rseg0(NC);
  for (int b = 0; b < NB; ++b) {
    nkbase[b] = SN.keys;
    SN.add(B.items[b].m, 0.0);
  }
  for (int c = 0; c < NC; ++c) {
    const ItemDesc& e = C.items[c];
    rkbase[c] = SR.keys;
    rseg0[c] = SR.nseg();
    const double cr = consistency_memo((double)(e.m / 2 + 1) / (double)e.m, 1);
    for (int j = 0; j < e.p; ++j) SR.add(e.m, cr);
  }
  // aggregation entries
  std::vector<int2> ent;
  for (int k = 0; k < ND; ++k)
    for (int e = 0; e < D[k].p + D[k].p * (D[k].p + 1) / 2; ++e) ent.push_back(make_int2(k, e));

  // ---------------------------------------------------------------- workspace
  Layout L;
  size_t offC[NOFF], offB[NOFF], offG[NOFF];
  // diagnostics: the C-step items keep their log det trace when a dataset
  // asks for it
  bool want_trace = false, want_diag = false;
  for (int k = 0; k < nd; ++k) {
    const rtdetmcd_out& ok = sets[k].out;
    want_trace = want_trace || ok.ldtrace != nullptr;
    want_diag = want_diag || ok.ldtrace || ok.hmargin || ok.cmargin;
  }
  C.ldtr_n = want_trace ? o.max_csteps : 0;
  layout_items(L, C, offC);
  layout_items(L, B, offB);
  layout_items(L, G, offG);
  const size_t o_ds = L.add(ND * sizeof(DsInfo));
  const size_t o_outs = L.add(ND * sizeof(rtdetmcd_out));
  const size_t o_loc = L.add((size_t)ND * PMAX * 8), o_scale = L.add((size_t)ND * PMAX * 8);
  const size_t o_muraw = L.add((size_t)ND * PMAX * 8), o_sigraw = L.add((size_t)ND * MSTRIDE * 8);
  const size_t o_nw = L.add((size_t)ND * 8);
  const size_t o_bmu = L.add((size_t)NB * PMAX * 8), o_bsig = L.add((size_t)NB * MSTRIDE * 8);
  const size_t o_bld = L.add((size_t)NB * 8), o_bkl = L.add((size_t)NB * 8);
  const size_t o_bitem = L.add((size_t)NB * 4), o_bstat = L.add((size_t)NB * 4);
  const size_t o_bstart = L.add((size_t)NB * 4), o_biters = L.add((size_t)NB * 4);
  const size_t o_bds = L.add((size_t)NB * 4);
  const size_t o_med = L.add((size_t)ND * (PMAX + MSTRIDE) * 8);
  const size_t o_vbuf = L.add((size_t)NC * MSTRIDE * 8), o_wbuf = L.add((size_t)NC * MSTRIDE * 8);
  const size_t o_s2 = L.add((size_t)NC * PMAX * 8);
  const size_t o_rcnt = L.add((size_t)NB * 8), o_rsum = L.add((size_t)NB * PMAX * 8);
  const size_t o_rS = L.add((size_t)NB * MSTRIDE * 8);
  const size_t o_cut = L.add((size_t)NB * 2 * 8);
  const size_t o_chi = L.add((size_t)ND * 8);
  const size_t o_ent = L.add(ent.size() * sizeof(int2));
  const size_t o_std_seg0 = L.add((size_t)ND * 4), o_in64 = L.add((size_t)ND * 4);
  const size_t o_nkb = L.add((size_t)NB * 8), o_rkb = L.add((size_t)NC * 8);
  const size_t o_rseg0 = L.add((size_t)NC * 4);
  const size_t o_sflag = L.add(8);
  const size_t o_cjobs = L.add((size_t)ND * sizeof(ColJob));
  SortDev D32, D64, DN, DR;
  layout_sort(L, S32, D32);
  layout_sort(L, S64, D64);
  layout_sort(L, SN, DN);
  layout_sort(L, SR, DR);
  const int64_t kbytes = std::max({S32.keys * 4 + S64.keys * 8, SN.keys * 8, SR.keys * 8});
  // the staging slots of the sample sort live in the ping-pong buffer (the
  // 64-bit standardisation plan's part of it starts after the 32-bit keys)
  const int64_t tbytes = std::max({kbytes, S32.bucket_keys() * 4,
                                   S32.keys * 4 + S64.bucket_keys() * 8, SN.bucket_keys() * 8,
                                   SR.bucket_keys() * 8});
  const size_t maxtiles = std::max({S32.tiles.size() + S64.tiles.size(), SN.tiles.size(),
                                    SR.tiles.size()});
  const size_t o_keys = L.add((size_t)kbytes), o_tmp = L.add((size_t)tbytes);
  const size_t o_counts = L.add(maxtiles * 256 * 4), o_offs = L.add(maxtiles * 256 * 4);
  const size_t maxseg = std::max({(size_t)S32.nseg() + S64.nseg(), (size_t)SN.nseg(),
                                  (size_t)SR.nseg()});
  size_t o_mb[9];
  for (int k = 0; k < 7; ++k) o_mb[k] = L.add(maxtiles * 8);
  o_mb[7] = L.add(maxseg * 2 * 8);
  o_mb[8] = L.add(maxseg * 5 * 8);
  // random partitions: the fitted rows in block order (dense, row stride p)
  // and the inverse permutation
  std::vector<size_t> o_xp(ND, 0), o_inv(ND, 0);
  for (int k = 0; k < ND; ++k)
    if (D[k].perm) {
      o_xp[k] = L.add((size_t)D[k].q * D[k].m * D[k].p * (D[k].dtype == 0 ? 4 : 8));
      o_inv[k] = L.add((size_t)D[k].n * 4);
    }
  RTD_TRY(ensure_ws(ctx, L.off));
  char* base = static_cast<char*>(ctx->ws);

  FitArrays F{};
  F.loc = reinterpret_cast<double*>(base + o_loc);
  F.scale = reinterpret_cast<double*>(base + o_scale);
  F.muraw = reinterpret_cast<double*>(base + o_muraw);
  F.sigraw = reinterpret_cast<double*>(base + o_sigraw);
  F.nw = reinterpret_cast<int64_t*>(base + o_nw);
  F.bmu = reinterpret_cast<double*>(base + o_bmu);
  F.bsig = reinterpret_cast<double*>(base + o_bsig);
  F.bld = reinterpret_cast<double*>(base + o_bld);
  F.bkl = reinterpret_cast<double*>(base + o_bkl);
  F.bitem = reinterpret_cast<int32_t*>(base + o_bitem);
  F.bstat = reinterpret_cast<int32_t*>(base + o_bstat);
  F.bstart = reinterpret_cast<int32_t*>(base + o_bstart);
  F.biters = reinterpret_cast<int32_t*>(base + o_biters);
  F.bds = reinterpret_cast<int32_t*>(base + o_bds);
  F.med = reinterpret_cast<double*>(base + o_med);
  F.vbuf = reinterpret_cast<double*>(base + o_vbuf);
  F.wbuf = reinterpret_cast<double*>(base + o_wbuf);
  F.s2buf = reinterpret_cast<double*>(base + o_s2);
  F.rcnt = reinterpret_cast<double*>(base + o_rcnt);
  F.rsum = reinterpret_cast<double*>(base + o_rsum);
  F.rS = reinterpret_cast<double*>(base + o_rS);
  double* cut = reinterpret_cast<double*>(base + o_cut);
  double* dchi = reinterpret_cast<double*>(base + o_chi);
  int2* dent = reinterpret_cast<int2*>(base + o_ent);
  int32_t* dstd_seg0 = reinterpret_cast<int32_t*>(base + o_std_seg0);
  int32_t* din64 = reinterpret_cast<int32_t*>(base + o_in64);
  int64_t* dnkb = reinterpret_cast<int64_t*>(base + o_nkb);
  int64_t* drkb = reinterpret_cast<int64_t*>(base + o_rkb);
  int32_t* drseg0 = reinterpret_cast<int32_t*>(base + o_rseg0);
  DsInfo* dds = reinterpret_cast<DsInfo*>(base + o_ds);
  rtdetmcd_out* douts = reinterpret_cast<rtdetmcd_out*>(base + o_outs);
  char* keys = base + o_keys;
  char* tmp = base + o_tmp;
  int32_t* counts = reinterpret_cast<int32_t*>(base + o_counts);
  int32_t* offs = reinterpret_cast<int32_t*>(base + o_offs);
  MbScratch mbs;
  mbs.bs1 = reinterpret_cast<double*>(base + o_mb[0]);
  mbs.bs2 = reinterpret_cast<double*>(base + o_mb[1]);
  mbs.wbest = reinterpret_cast<double*>(base + o_mb[2]);
  mbs.wj = reinterpret_cast<int64_t*>(base + o_mb[3]);
  mbs.k0 = reinterpret_cast<double*>(base + o_mb[4]);
  mbs.k1 = reinterpret_cast<double*>(base + o_mb[5]);
  mbs.k2 = reinterpret_cast<double*>(base + o_mb[6]);
  mbs.tot = reinterpret_cast<double*>(base + o_mb[7]);
  mbs.prm = reinterpret_cast<double*>(base + o_mb[8]);
  // the 32-bit and 64-bit standardisation sorts share the key buffer
  bind_sort(base, S32, D32, keys, tmp, counts, offs);
  bind_sort(base, S64, D64, keys + S32.keys * 4, tmp + S32.keys * 4,
            counts + S32.tiles.size() * 256, offs + S32.tiles.size() * 256);
  bind_sort(base, SN, DN, keys, tmp, counts, offs);
  bind_sort(base, SR, DR, keys, tmp, counts, offs);
  D32.plan.mb = D64.plan.mb = DN.plan.mb = DR.plan.mb = &mbs;
  int32_t* sflag = reinterpret_cast<int32_t*>(base + o_sflag);
  for (SortDev* sd : {&D32, &D64, &DN, &DR}) {
    sd->plan.safe = ctx->sort_safe;
    sd->plan.flag = sflag;
  }

  ItemDev CD, BD, GD;
  bind_items(base, C, offC, CD);
  bind_items(base, B, offB, BD);
  bind_items(base, G, offG, GD);
  // loc/scale pointers of every item; the blocks, starts and reweighting
  // rows of a randomly partitioned dataset read its gathered copy
  for (auto* set : {&C, &B, &G})
    for (ItemDesc& e : set->items) {
      e.loc = F.loc + (size_t)e.ds * PMAX;
      e.scale = F.scale + (size_t)e.ds * PMAX;
    }
  for (int k = 0; k < ND; ++k) {
    if (!D[k].perm) continue;
    auto repoint = [&](ItemDesc& e) {
      e.X = base + o_xp[k];
      e.ld = D[k].p;
    };
    for (int i = D[k].item0; i < D[k].item0 + 2 * D[k].q; ++i) repoint(C.items[i]);
    for (int i = D[k].blk0; i < D[k].blk0 + D[k].q; ++i) repoint(B.items[i]);
    repoint(G.items[D[k].glob0]);
  }
  std::vector<DsInfo> dinfo(ND);
  std::vector<rtdetmcd_out> houts(ND);
  std::vector<double> hchi(ND);
  for (int k = 0; k < ND; ++k) {
    DsInfo& x = dinfo[k];
    std::memset(&x, 0, sizeof(x));
    x.X = D[k].in->X; x.n = D[k].n; x.ld = D[k].ld; x.m = D[k].m; x.h = D[k].h;
    x.p = D[k].p; x.dtype = D[k].dtype; x.q = D[k].q;
    x.chi2p = D[k].chi2p; x.calpha = D[k].calpha; x.crew = D[k].crew;
    x.item0 = D[k].item0; x.blk0 = D[k].blk0; x.glob0 = D[k].glob0; x.glob1 = ND + k;
    x.err = 0;
    x.perm = D[k].perm;
    x.inv = D[k].perm ? reinterpret_cast<int32_t*>(base + o_inv[k]) : nullptr;
    x.warm_mu = D[k].warm ? D[k].in->warm_mu : nullptr;
    x.warm_sigma = D[k].warm ? D[k].in->warm_sigma : nullptr;
    houts[k] = D[k].in->out;
    hchi[k] = D[k].chi2p;
  }
  // column-key jobs of the standardisation: float datasets, then double ones
  std::vector<ColJob> cjobs;
  int64_t ctiles[2] = {0, 0};
  int ncjobs[2] = {0, 0};
  for (int t = 0; t < 2; ++t)
    for (int k = 0; k < ND; ++k) {
      if (D[k].dtype != t) continue;
      const SortHost& Hs = t == 0 ? S32 : S64;
      const SortDev& Ds = t == 0 ? D32 : D64;
      ColJob j{};
      j.X = D[k].in->X;
      j.keys = static_cast<char*>(Ds.plan.keys) + Hs.off[std_seg0[k]] * Hs.key_bytes;
      j.err = &dds[k].err;
      j.n = D[k].n;
      j.ld = D[k].ld;
      j.p = D[k].p;
      j.tile0 = ctiles[t];
      ctiles[t] += (D[k].n + COLKEY_ROWS - 1) / COLKEY_ROWS;
      ++ncjobs[t];
      cjobs.push_back(j);
    }
  ColJob* dcjobs = reinterpret_cast<ColJob*>(base + o_cjobs);
  Uploader up;
  up.add(dcjobs, cjobs.data(), cjobs.size());
  up.add(CD.items, C.items.data(), C.items.size());
  up.add(CD.dtiles, C.dtiles.data(), C.dtiles.size());
  up.add(CD.stiles, C.stiles.data(), C.stiles.size());
  up.add(BD.items, B.items.data(), B.items.size());
  up.add(BD.dtiles, B.dtiles.data(), B.dtiles.size());
  up.add(BD.stiles, B.stiles.data(), B.stiles.size());
  up.add(GD.items, G.items.data(), G.items.size());
  up.add(GD.dtiles, G.dtiles.data(), G.dtiles.size());
  up.add(GD.stiles, G.stiles.data(), G.stiles.size());
  up.add(dds, dinfo.data(), ND);
  up.add(douts, houts.data(), ND);
  up.add(dchi, hchi.data(), ND);
  up.add(dent, ent.data(), ent.size());
  up.add(dstd_seg0, std_seg0.data(), ND);
  up.add(din64, std_in64.data(), ND);
  up.add(dnkb, nkbase.data(), NB);
  up.add(drkb, rkbase.data(), NC);
  up.add(drseg0, rseg0.data(), NC);
  upload_sort(up, S32, D32);
  upload_sort(up, S64, D64);
  upload_sort(up, SN, DN);
  upload_sort(up, SR, DR);
  RTD_TRY(up.flush(ctx));

  const bool plain = o.launch == RTDETMCD_LAUNCH_PLAIN;
  const double q1 = chi2_quantile_memo(o.cutoff_q, 1);
  const double crew1 = consistency_memo(o.cutoff_q, 1);
  const int smode = o.standardize == RTDETMCD_STD_MEDMAD ? SEGSTAT_MEDMAD : SEGSTAT_UNIMCD;

  ProfMark pm_fit(ctx, RTDETMCD_PROF_FIT, st, 0.0);
  // ---------------------------------------------------------------- random partitions
  for (int k = 0; k < ND; ++k) {
    if (!D[k].perm) continue;
    int32_t* inv = reinterpret_cast<int32_t*>(base + o_inv[k]);
    RTD_HIP(launch_fill_i32(inv, -1, D[k].n, st));
    RTD_HIP(launch_perm_check(D[k].perm, D[k].n, inv, dds, k, st));
    RTD_HIP(launch_perm_gather(D[k].dtype, D[k].in->X, D[k].n, D[k].ld, D[k].p, D[k].perm,
                               (int64_t)D[k].q * D[k].m, base + o_xp[k], st));
  }
  // ---------------------------------------------------------------- step 0: standardisation
  RTD_HIP(launch_fill_i32(sflag, 0, 1, st));
  RTD_HIP(launch_colkeys(0, dcjobs, ncjobs[0], ctiles[0], st));
  RTD_HIP(launch_colkeys(1, dcjobs + ncjobs[0], ncjobs[1], ctiles[1], st));
  RTD_TRY(sort_stats(ctx, S32, D32, 0, S32.nseg(), smode, q1, crew1));
  RTD_TRY(sort_stats(ctx, S64, D64, 0, S64.nseg(), smode, q1, crew1));
  RTD_HIP(launch_std_finish(D32.st, D64.st, dstd_seg0, din64, ND, dds, F, st));

  // ---------------------------------------------------------------- steps 1-2: starts
  auto group_of_block = [&](int b) -> const Group& {
    for (const Group& g : groups)
      if (b >= g.b0 && b < g.b1) return g;
    return groups.front();
  };
  auto group_of_item = [&](int c) -> const Group& {
    for (const Group& g : groups)
      if (c >= g.c0 && c < g.c1) return g;
    return groups.front();
  };
  // block phases over [b0, b1) (a whole group when batched, one block when plain)
  auto blocks_phase = [&](int b0, int b1) -> rtdetmcd_status {
    const Group& g = group_of_block(b0);
    const int st0 = B.items[b0].tile0, stn = B.items[b1 - 1].tile0 + B.items[b1 - 1].ntiles - st0;
    const int dt0 = B.dt_first[b0], dtn = B.dt_first[b1 - 1] + B.dt_count[b1 - 1] - dt0;
    RTD_HIP(launch_sscp(g.bucket, g.dtype, SSCP_WRAP, BD.items, BD.A, BD.stiles + st0, stn,
                        SSCP_TILE, nullptr, nullptr, st));
    RTD_HIP(launch_collapse(BD.items, BD.A, b0, b1 - b0, B.max_ntiles(b0, b1), 0, SSCP_TILE, st));
    RTD_HIP(launch_reduce_partials(BD.items, BD.A.part, b0, b1 - b0, F.rcnt, F.rsum, F.rS, st));
    RTD_HIP(launch_init_cov(0, BD.items, b0, b1 - b0, F, CD.A, dds, cut, DN.st, st));
    RTD_HIP(launch_project(g.bucket, g.dtype, 1, BD.items, BD.dtiles + dt0, dtn, DIST_TILE,
                           nullptr, nullptr, dnkb, reinterpret_cast<uint64_t*>(DN.plan.keys), st));
    RTD_TRY(sort_stats(ctx, SN, DN, b0, b1, SEGSTAT_GSSCM, 0.0, 1.0));
    RTD_HIP(launch_init_cov(2, BD.items, b0, b1 - b0, F, CD.A, dds, cut, DN.st, st));
    RTD_HIP(launch_sscp(g.bucket, g.dtype, SSCP_GSSCM, BD.items, BD.A, BD.stiles + st0, stn,
                        SSCP_TILE, nullptr, cut, st));
    RTD_HIP(launch_collapse(BD.items, BD.A, b0, b1 - b0, B.max_ntiles(b0, b1), 0, SSCP_TILE, st));
    RTD_HIP(launch_reduce_partials(BD.items, BD.A.part, b0, b1 - b0, F.rcnt, F.rsum, F.rS, st));
    RTD_HIP(launch_init_cov(1, BD.items, b0, b1 - b0, F, CD.A, dds, cut, DN.st, st));
    return RTDETMCD_OK;
  };
  // refinement of the starts [c0, c1) (Sec. 3.3)
  auto refine_phase = [&](int c0, int c1) -> rtdetmcd_status {
    const Group& g = group_of_item(c0);
    const int dt0 = C.dt_first[c0], dtn = C.dt_first[c1 - 1] + C.dt_count[c1 - 1] - dt0;
    const int s0 = rseg0[c0], s1 = rseg0[c1 - 1] + C.items[c1 - 1].p;
    uint64_t* rk = reinterpret_cast<uint64_t*>(DR.plan.keys);
    RTD_HIP(launch_eig(g.bucket, CD.items, CD.A, F, c0, c1 - c0, o.kappa_max, st));
    RTD_HIP(launch_project(g.bucket, g.dtype, 0, CD.items, CD.dtiles + dt0, dtn, DIST_TILE,
                           CD.A.status, F.wbuf, drkb, rk, st));
    RTD_TRY(sort_stats(ctx, SR, DR, s0, s1, SEGSTAT_UNIMCD, q1, crew1));
    RTD_HIP(launch_refine(1, CD.items, CD.A, F, c0, c1 - c0, DR.st, drseg0, st));
    RTD_HIP(launch_project(g.bucket, g.dtype, 0, CD.items, CD.dtiles + dt0, dtn, DIST_TILE,
                           CD.A.status, F.wbuf, drkb, rk, st));
    RTD_TRY(sort_stats(ctx, SR, DR, s0, s1, SEGSTAT_UNIMCD, q1, crew1));
    RTD_HIP(launch_refine(2, CD.items, CD.A, F, c0, c1 - c0, DR.st, drseg0, st));
    return RTDETMCD_OK;
  };

  RTD_HIP(launch_fill_i32(CD.A.status, ACTIVE, NC, st));
  RTD_HIP(launch_fill_i32(CD.A.iter, 0, NC, st));
  RTD_HIP(launch_fill_u8(CD.A.mask, 0, C.rows, st));
  if (!plain) {
    for (const Group& g : groups) {
      if (g.all_warm) continue;   // steps 1-2 are not needed
      if (g.b1 > g.b0) RTD_TRY(blocks_phase(g.b0, g.b1));
      if (g.c1 > g.c0) RTD_TRY(refine_phase(g.c0, g.c1));
    }
    for (int k = 0; k < ND; ++k)
      if (D[k].warm) RTD_HIP(launch_warm_start(dds, k, D[k].q, CD.A, F, st));
    // ---------------------------------------------------------------- step 3: C-steps
    for (const Group& g : groups)
      if (g.c1 > g.c0)
        RTD_TRY(run_csteps(ctx, C, CD, g.bucket, g.dtype, g.c0, g.c1 - g.c0, o, ctx->flag));
    RTD_HIP(launch_choose(BD.items, CD.items, CD.A, F, dds, 0, NB, st));
  } else {
    for (int b = 0; b < NB; ++b) {
      const int k = B.items[b].ds;
      if (D[k].warm) {
        // the dataset's blocks in one go, at its first block
        if (b == D[k].blk0) RTD_HIP(launch_warm_start(dds, k, D[k].q, CD.A, F, st));
      } else {
        RTD_TRY(blocks_phase(b, b + 1));
      }
      for (int c = 2 * b; c < 2 * b + 2; ++c) {
        if (!D[k].warm) RTD_TRY(refine_phase(c, c + 1));
        const Group& g = group_of_item(c);
        RTD_TRY(run_csteps(ctx, C, CD, g.bucket, g.dtype, c, 1, o, ctx->flag));
      }
      RTD_HIP(launch_choose(BD.items, CD.items, CD.A, F, dds, b, 1, st));
    }
  }

  // ---------------------------------------------------------------- steps 5-7: aggregation
  RTD_HIP(launch_median(dds, F, dent, (int)ent.size(), st));
  RTD_HIP(launch_kl(dds, CD.A, F, 0, NB, o.cstep_mode == RTDETMCD_CSTEP_SMW, st));
  RTD_HIP(launch_fill_i32(GD.A.status, ACTIVE, NG, st));
  RTD_HIP(launch_pool(dds, GD.A, F, 0, ND, o.pool_mode, st));
  for (const Group& g : groups)
    RTD_HIP(launch_finalize(g.bucket, GD.items, GD.A, g.ds0, g.ds1 - g.ds0, 1, 1, 1e300,
                            RTDETMCD_CSTEP_FULL, o.distance, st));
  // ---------------------------------------------------------------- steps 8-9: reweighting
  for (const Group& g : groups) {
    const int a = g.ds0, b = g.ds1;
    const int dt0 = G.dt_first[a], dtn = G.dt_first[b - 1] + G.dt_count[b - 1] - dt0;
    const int st0 = G.items[a].tile0, stn = G.items[b - 1].tile0 + G.items[b - 1].ntiles - st0;
    RTD_HIP(launch_dist(g.bucket, g.dtype, G.rows_dense(a, b, g.bucket), GD.items,
                        GD.dtiles + dt0, dtn, DIST_TILE, GD.A.mtri, GD.A.mux, nullptr,
                        o.distance ? GD.A.form : nullptr, GD.A.d2, st));
    RTD_HIP(launch_sscp(g.bucket, g.dtype, SSCP_D2CUT, GD.items, GD.A, GD.stiles + st0, stn,
                        SSCP_TILE, nullptr, dchi, st));
    RTD_HIP(launch_collapse(GD.items, GD.A, a, b - a, G.max_ntiles(a, b), 0, SSCP_TILE, st));
  }
  RTD_HIP(launch_rew(dds, GD.items, GD.A, F, 0, ND, st));
  RTD_HIP(launch_fill_i32(GD.A.status + ND, ACTIVE, ND, st));
  for (const Group& g : groups)
    RTD_HIP(launch_finalize(g.bucket, GD.items, GD.A, ND + g.ds0, g.ds1 - g.ds0, 1, 1, 1e300,
                            RTDETMCD_CSTEP_FULL, o.distance, st));
  // ---------------------------------------------------------------- step 10: distances, flags
  for (const Group& g : groups) {
    const int a = ND + g.ds0, b = ND + g.ds1;
    const int dt0 = G.dt_first[a], dtn = G.dt_first[b - 1] + G.dt_count[b - 1] - dt0;
    double byt = 0.0;
    for (int k = g.ds0; k < g.ds1; ++k)
      byt += (double)D[k].n * ((D[k].dtype == 0 ? 4.0 : 8.0) * D[k].p + 10.0) +
             (double)D[k].q * D[k].m * 8.0;
    ProfMark pm(ctx, RTDETMCD_PROF_FINAL_DIST, st, byt);
    RTD_HIP(launch_final_dist(g.bucket, g.dtype, G.rows_dense(a, b, g.bucket), GD.items,
                              GD.dtiles + dt0, dtn, DIST_TILE,
                              GD.A.mtri, GD.A.mux, o.distance ? GD.A.form : nullptr, GD.A.d2,
                              dds, douts, st));
    pm.end(st);
  }
  RTD_HIP(launch_hsub(CD.items, CD.A, F, dds, douts, 0, NB, st));
  RTD_HIP(launch_outputs(dds, GD.A, F, douts, 0, ND, st));
  if (want_diag) RTD_HIP(launch_diag(CD.items, CD.A, F, dds, douts, NB, ND, o.max_csteps, st));
  pm_fit.end(st);
  // ---------------------------------------------------------------- status
  RTD_HIP(hipMemcpyAsync(dinfo.data(), dds, ND * sizeof(DsInfo), hipMemcpyDeviceToHost, st));
  RTD_HIP(hipMemcpyAsync(ctx->flag, sflag, 4, hipMemcpyDeviceToHost, st));
  RTD_HIP(hipStreamSynchronize(st));
  if (*ctx->flag && !ctx->sort_safe) {
    // a sort whose atomic ranks came out of lane order: fit again with
    // ballot ranking throughout
    ctx->sort_safe = 1;
    ++ctx->sort_reruns;
    const rtdetmcd_status again = fit_many(ctx, nd, sets, o, status);
    ctx->sort_safe = 0;
    return again;
  }
  rtdetmcd_status ret = RTDETMCD_OK;
  for (int k = 0; k < ND; ++k) {
    const int orig = (int)(D[k].in - sets);
    const rtdetmcd_status s = dinfo[k].err ? (rtdetmcd_status)dinfo[k].err : RTDETMCD_OK;
    if (status) status[orig] = s;
    if (s != RTDETMCD_OK) {
      ret = s;
      ctx->err = "dataset " + std::to_string(orig) +
                 (s == RTDETMCD_EINVAL       ? ": perm is not a permutation of the rows"
                  : s == RTDETMCD_ENONFINITE ? ": X holds NaN or Inf values"
                                             : ": no valid fit (degenerate data)");
    }
  }
  return nd == 1 ? ret : RTDETMCD_OK;
}

}  // namespace rtd

using namespace rtd;

extern "C" {

rtdetmcd_status rtdetmcd_fit(rtdetmcd_handle ctx, const void* X, int32_t dtype, int64_t n,
                             int32_t p, int64_t ld, int64_t h_sub, int32_t n_chunks,
                             const rtdetmcd_opts* o_in, const rtdetmcd_out* out) {
  if (!ctx) return RTDETMCD_EINVAL;
  rtdetmcd_opts o;
  RTD_TRY(check_opts(ctx, o_in, o));
  if (!out) {
    ctx->err = "rtdetmcd_fit: out is NULL";
    return RTDETMCD_EINVAL;
  }
  rtdetmcd_dataset d{};
  d.X = X; d.dtype = dtype; d.n = n; d.p = p; d.ld = ld; d.h_sub = h_sub; d.n_chunks = n_chunks;
  d.out = *out;
  return fit_many(ctx, 1, &d, o, nullptr);
}

rtdetmcd_status rtdetmcd_fit_batched(rtdetmcd_handle ctx, int32_t n_datasets,
                                     const rtdetmcd_dataset* sets, const rtdetmcd_opts* o_in,
                                     rtdetmcd_status* status) {
  if (!ctx) return RTDETMCD_EINVAL;
  rtdetmcd_opts o;
  RTD_TRY(check_opts(ctx, o_in, o));
  if (n_datasets < 1 || !sets) {
    ctx->err = "rtdetmcd_fit_batched: no datasets";
    return RTDETMCD_EINVAL;
  }
  return fit_many(ctx, n_datasets, sets, o, status);
}

}  // extern "C"
