// C entry points of librtdetmcd: handle management, options, low-level steps
// and the C-step loop driver.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "driver.h"

namespace rtd {

static hipEvent_t prof_event(rtdetmcd_ctx* ctx) {
  if (ctx->prof_next < ctx->prof_events.size()) return ctx->prof_events[ctx->prof_next++];
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  ctx->prof_events.push_back(e);
  ctx->prof_next = ctx->prof_events.size();
  return e;
}

ProfMark::ProfMark(rtdetmcd_ctx* c, int kind, hipStream_t s, double bytes, double flops_useful,
                   double flops_exec) {
  if (!c || !c->prof_on) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  hipEvent_t e0 = prof_event(c), e1 = prof_event(c);
  if (!e0 || !e1 || hipEventRecord(e0, s) != hipSuccess) return;
  ctx = c;
  idx = (int)c->prof.size();
  c->prof.push_back({kind, e0, e1, bytes, flops_useful, flops_exec});
}

void ProfMark::end(hipStream_t s) {
  if (idx >= 0 && hipEventRecord(ctx->prof[idx].e1, s) != hipSuccess) ctx->prof[idx].e1 = nullptr;
}

void drop_graphs(rtdetmcd_ctx* ctx) {
  for (rtd_graph& g : ctx->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  ctx->graphs.clear();
}

rtdetmcd_status ensure_ws(rtdetmcd_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->ws_size) return RTDETMCD_OK;
  RTD_HIP(hipSetDevice(ctx->device));
  if (ctx->ws) {
    RTD_HIP(hipStreamSynchronize(ctx->stream));
    if (ctx->gstream) RTD_HIP(hipStreamSynchronize(ctx->gstream));
    drop_graphs(ctx);   // their kernel arguments point into the old workspace
    RTD_HIP(hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_size = 0;
  }
  const size_t want = bytes + bytes / 4 + (1u << 20);
  if (hipMalloc(&ctx->ws, want) != hipSuccess) {
    ctx->ws = nullptr;
    ctx->err = "workspace allocation of " + std::to_string(want) + " bytes failed";
    (void)hipGetLastError();
    return RTDETMCD_ENOMEM;
  }
  ctx->ws_size = want;
  return RTDETMCD_OK;
}

// All tables of a flush go to the device in one copy (header of (dst,
// offset, bytes) records, then the payload) into a staging buffer, and one
// kernel scatters them to their places: one copy and one launch instead of
// one copy per table.
rtdetmcd_status Uploader::flush(rtdetmcd_ctx* ctx) {
  if (ents.empty()) return RTDETMCD_OK;
  if (ctx->pin_pending) {
    RTD_HIP(hipEventSynchronize(ctx->pin_ev));
    ctx->pin_pending = false;
  }
  const size_t n = ents.size();
  const size_t hdr = (n * 3 * sizeof(uint64_t) + 255) & ~(size_t)255;
  const size_t total = hdr + buf.size();
  if (total > ctx->pin_size) {
    if (ctx->pin) RTD_HIP(hipHostFree(ctx->pin));
    ctx->pin = nullptr;
    const size_t want = total + (1u << 16);
    RTD_HIP(hipHostMalloc(&ctx->pin, want, hipHostMallocDefault));
    ctx->pin_size = want;
  }
  if (total > ctx->stage_size) {
    if (ctx->stage) {
      RTD_HIP(hipStreamSynchronize(ctx->stream));
      RTD_HIP(hipFree(ctx->stage));
    }
    ctx->stage = nullptr;
    ctx->stage_size = 0;
    const size_t want = total + (1u << 16);
    RTD_HIP(hipMalloc(&ctx->stage, want));
    ctx->stage_size = want;
  }
  uint64_t* h = static_cast<uint64_t*>(ctx->pin);
  for (size_t k = 0; k < n; ++k) {
    h[3 * k] = (uint64_t)(uintptr_t)ents[k].dst;
    h[3 * k + 1] = (uint64_t)(hdr + ents[k].off);
    h[3 * k + 2] = (uint64_t)ents[k].bytes;
  }
  std::memcpy(static_cast<char*>(ctx->pin) + hdr, buf.data(), buf.size());
  RTD_HIP(hipMemcpyAsync(ctx->stage, ctx->pin, total, hipMemcpyHostToDevice, ctx->stream));
  RTD_HIP(launch_upload_scatter(ctx->stage, (int)n, ctx->stream));
  RTD_HIP(hipEventRecord(ctx->pin_ev, ctx->stream));
  ctx->pin_pending = true;
  ents.clear();
  buf.clear();
  return RTDETMCD_OK;
}

void layout_items(Layout& L, const ItemSet& S, size_t off[NOFF]) {
  const size_t I = S.items.size();
  off[0] = L.add(I * sizeof(ItemDesc));
  off[1] = L.add(S.dtiles.size() * sizeof(Tile));
  off[2] = L.add(S.stiles.size() * sizeof(Tile));
  off[3] = L.add(I * 4);             // status
  off[4] = L.add(I * 4);             // iter
  off[5] = L.add(I * 4);             // kswap
  off[6] = L.add(I * 4);             // full
  off[7] = L.add(I * 8);             // logdet
  off[8] = L.add(I * PMAX * 8);      // mux
  off[9] = L.add(I * MSTRIDE * 8);   // lamx
  off[10] = L.add(I * PMAX * 8);     // muz
  off[11] = L.add(I * MSTRIDE * 8);  // sigz
  off[12] = L.add(I * MSTRIDE * 8);  // linv
  off[13] = L.add(I * MSTRIDE * 8);  // mtri
  off[14] = L.add((size_t)S.rows * 8);   // d2
  off[15] = L.add((size_t)S.rows);       // mask
  off[16] = L.add((size_t)S.rows * 4);   // swap
  off[17] = L.add(S.stiles.size() * PSTRIDE * 8);  // partials
  off[18] = L.add(64);                   // nactive
  off[19] = L.add(I * 4);             // form
  off[20] = L.add(I * MSTRIDE * 8);   // sinv
  off[21] = L.add(I * (size_t)S.ldtr_n * 8);   // log det trace
}

void bind_items(char* base, const ItemSet& S, const size_t off[NOFF], ItemDev& D) {
  D.items = reinterpret_cast<ItemDesc*>(base + off[0]);
  D.dtiles = reinterpret_cast<Tile*>(base + off[1]);
  D.stiles = reinterpret_cast<Tile*>(base + off[2]);
  ItemArrays& A = D.A;
  A.status = reinterpret_cast<int32_t*>(base + off[3]);
  A.iter = reinterpret_cast<int32_t*>(base + off[4]);
  A.kswap = reinterpret_cast<int32_t*>(base + off[5]);
  A.full = reinterpret_cast<int32_t*>(base + off[6]);
  A.logdet = reinterpret_cast<double*>(base + off[7]);
  A.mux = reinterpret_cast<double*>(base + off[8]);
  A.lamx = reinterpret_cast<double*>(base + off[9]);
  A.muz = reinterpret_cast<double*>(base + off[10]);
  A.sigz = reinterpret_cast<double*>(base + off[11]);
  A.linv = reinterpret_cast<double*>(base + off[12]);
  A.mtri = reinterpret_cast<double*>(base + off[13]);
  A.d2 = reinterpret_cast<double*>(base + off[14]);
  A.mask = reinterpret_cast<uint8_t*>(base + off[15]);
  A.swap = reinterpret_cast<int32_t*>(base + off[16]);
  A.part = reinterpret_cast<double*>(base + off[17]);
  A.nactive = reinterpret_cast<int32_t*>(base + off[18]);
  A.form = reinterpret_cast<int32_t*>(base + off[19]);
  A.sinv = reinterpret_cast<double*>(base + off[20]);
  A.ldtr = S.ldtr_n > 0 ? reinterpret_cast<double*>(base + off[21]) : nullptr;
  A.ldtr_n = S.ldtr_n;
}

// The executable graph of R C-steps for `key`: from the cache, or captured
// now on the handle's replay stream (no memset nodes: counters are cleared by
// a fill kernel).
template <typename Step>
rtdetmcd_status graph_for(rtdetmcd_ctx* ctx, const std::vector<int64_t>& key, int R, Step& step,
                          hipGraphExec_t* out) {
  for (rtd_graph& g : ctx->graphs) {
    if (g.key == key) {
      *out = g.exec;
      return RTDETMCD_OK;
    }
  }
  if (!ctx->gstream) {
    RTD_HIP(hipStreamCreateWithFlags(&ctx->gstream, hipStreamNonBlocking));
    RTD_HIP(hipEventCreateWithFlags(&ctx->gev[0], hipEventDisableTiming));
    RTD_HIP(hipEventCreateWithFlags(&ctx->gev[1], hipEventDisableTiming));
  }
  constexpr size_t kMaxGraphs = 16;
  if (ctx->graphs.size() >= kMaxGraphs) {
    RTD_HIP(hipStreamSynchronize(ctx->gstream));
    (void)hipGraphExecDestroy(ctx->graphs.front().exec);
    ctx->graphs.erase(ctx->graphs.begin());
  }
  hipGraph_t g = nullptr;
  RTD_HIP(hipStreamBeginCapture(ctx->gstream, hipStreamCaptureModeThreadLocal));
  rtdetmcd_status s = RTDETMCD_OK;
  for (int r = 0; r < R && s == RTDETMCD_OK; ++r) s = step(ctx->gstream);
  const hipError_t ec = hipStreamEndCapture(ctx->gstream, &g);
  if (s != RTDETMCD_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  RTD_HIP(ec);
  hipGraphExec_t ge = nullptr;
  const hipError_t ei = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  RTD_HIP(ei);
  rtd_graph e;
  e.key = key;
  e.exec = ge;
  ctx->graphs.push_back(e);
  *out = ge;
  return RTDETMCD_OK;
}

// Distance tiling of a batched C-step loop under opts.tune: the kept plan
// of this shape, or a new one measured on the first C-step's distance pass
// (every candidate timed twice with HIP events on the handle's stream, the
// faster kept).  The distance pass only writes the distances, which the
// loop's own first pass writes again, so the measurement leaves no trace.
// *idx: the plan's index in ctx->tune.
rtdetmcd_status tuned_dist_plan(rtdetmcd_ctx* ctx, const ItemSet& S, ItemDev& D, int bucket,
                                int dtype, int first, int n, bool dense,
                                const int32_t* form, int* idx) {
  int64_t rows = 0, max_m = 0;
  for (int i = first; i < first + n; ++i) {
    rows += S.items[i].m;
    max_m = std::max(max_m, S.items[i].m);
  }
  const std::vector<int64_t> key = {bucket, dtype, n, rows, max_m, dense ? 1 : 0, form ? 1 : 0};
  for (size_t k = 0; k < ctx->tune.size(); ++k)
    if (ctx->tune[k].key == key) {
      *idx = (int)k;
      return RTDETMCD_OK;
    }
  auto table = [&](int T) {
    std::vector<Tile> t;
    for (int i = first; i < first + n; ++i) {
      const int nd = (int)((S.items[i].m + T - 1) / T);
      for (int k = 0; k < nd; ++k) t.push_back({i, k});
    }
    return t;
  };
  const int rows_c[] = {256, 512, 1024, 2048, 4096};
  Tile* tmp = nullptr;
  RTD_HIP(hipMalloc(&tmp, table(256).size() * sizeof(Tile)));
  hipEvent_t e[2] = {nullptr, nullptr};
  RTD_HIP(hipEventCreate(&e[0]));
  RTD_HIP(hipEventCreate(&e[1]));
  int best_T = DIST_TILE;
  float best = 1e30f;
  hipError_t err = hipSuccess;
  for (const int T : rows_c) {
    const std::vector<Tile> t = table(T);
    err = hipMemcpy(tmp, t.data(), t.size() * sizeof(Tile), hipMemcpyHostToDevice);
    for (int rep = 0; rep < 2 && err == hipSuccess; ++rep) {
      err = hipEventRecord(e[0], ctx->stream);
      if (err == hipSuccess)
        err = launch_dist(bucket, dtype, dense, D.items, tmp, (int)t.size(), T, D.A.mtri,
                          D.A.mux, D.A.status, form, D.A.d2, ctx->stream);
      if (err == hipSuccess) err = hipEventRecord(e[1], ctx->stream);
      if (err == hipSuccess) err = hipEventSynchronize(e[1]);
      float ms = 0.0f;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e[0], e[1]);
      if (err == hipSuccess && ms < best) {
        best = ms;
        best_T = T;
      }
    }
    if (err != hipSuccess) break;
  }
  (void)hipEventDestroy(e[0]);
  (void)hipEventDestroy(e[1]);
  (void)hipFree(tmp);
  RTD_HIP(err);
  rtdetmcd_ctx::TunePlan tp;
  tp.key = key;
  tp.bucket = bucket;
  tp.tile_rows = best_T;
  tp.mode = 1;   // one factor per pass
  const std::vector<Tile> t = table(best_T);
  tp.ntiles = (int)t.size();
  RTD_HIP(hipMalloc(&tp.tiles, t.size() * sizeof(Tile)));
  RTD_HIP(hipMemcpy(tp.tiles, t.data(), t.size() * sizeof(Tile), hipMemcpyHostToDevice));
  constexpr size_t kMaxPlans = 64;
  if (ctx->tune.size() >= kMaxPlans) {   // the oldest plan goes (its graphs with it)
    drop_graphs(ctx);
    (void)hipFree(ctx->tune.front().tiles);
    ctx->tune.erase(ctx->tune.begin());
  }
  ctx->tune.push_back(tp);
  *idx = (int)ctx->tune.size() - 1;
  return RTDETMCD_OK;
}

rtdetmcd_status run_csteps(rtdetmcd_ctx* ctx, const ItemSet& S, ItemDev& D, int bucket,
                           int dtype, int first, int n, const rtdetmcd_opts& o,
                           int32_t* pin_flag) {
  hipStream_t st = ctx->stream;
  const int maxs = o.max_csteps;
  if (o.launch == RTDETMCD_LAUNCH_BATCHED) {
    // tiles of the items [first, first+n) are contiguous in all tables
    const int dt0 = S.dt_first[first];
    const int dtn = S.dt_first[first + n - 1] + S.dt_count[first + n - 1] - dt0;
    const int st0 = S.items[first].tile0;
    const int stn = S.items[first + n - 1].tile0 + S.items[first + n - 1].ntiles - st0;
    int64_t max_m = 0;
    for (int i = first; i < first + n; ++i) max_m = std::max(max_m, S.items[i].m);
    const int max_nt = S.max_ntiles(first, first + n);
    const bool dense = S.rows_dense(first, first + n, bucket);
    RTD_HIP(launch_finalize(bucket, D.items, D.A, first, n, 1, maxs, o.kappa_max, o.cstep_mode,
                            o.distance, st));
    int R = std::max(1, o.rounds_per_sync);
    // items may hold the explicit-inverse form only with the distance switch
    // or the single-swap mode
    const int32_t* form =
        (o.distance || o.cstep_mode == RTDETMCD_CSTEP_SMW) ? D.A.form : nullptr;
    // distance tiling: the plan's tables, or the tuned ones
    const Tile* dtab = D.dtiles + dt0;
    int dntab = dtn, dtile = DIST_TILE, tix = -1;
    if (o.tune) {
      RTD_TRY(tuned_dist_plan(ctx, S, D, bucket, dtype, first, n, dense, form, &tix));
      const rtdetmcd_ctx::TunePlan& tp = ctx->tune[tix];
      dtab = tp.tiles;
      dntab = tp.ntiles;
      dtile = tp.tile_rows;
      R = std::max(R, tp.iters);   // the first check after the previous fit's C-step count
    }
    // one C-step of every active item
    // one C-step of every active item; the selection zeroes the active count
    auto step = [&](hipStream_t s) -> rtdetmcd_status {
      RTD_HIP(launch_dist(bucket, dtype, dense, D.items, dtab, dntab, dtile, D.A.mtri,
                          D.A.mux, D.A.status, form, D.A.d2, s));
      RTD_HIP(launch_select(D.items, D.A, first, n, max_m, o.cstep_mode, s, 1));
      RTD_HIP(launch_sscp(bucket, dtype, SSCP_CSTEP, D.items, D.A, D.stiles + st0, stn,
                          SSCP_TILE, nullptr, nullptr, s));
      RTD_HIP(launch_collapse(D.items, D.A, first, n, max_nt, 1, SSCP_TILE, s));
      RTD_HIP(launch_finalize(bucket, D.items, D.A, first, n, 0, maxs, o.kappa_max,
                              o.cstep_mode, o.distance, s));
      return RTDETMCD_OK;
    };
    // kernel timing of the first C-step (every start still active): the
    // distance pass, the selection and the full sscp
    auto step1 = [&](hipStream_t s) -> rtdetmcd_status {
      double rows = 0.0, byt_d = 0.0, fl_d = 0.0, fl_su = 0.0, fl_se = 0.0;
      for (int i = first; i < first + n; ++i) {
        const ItemDesc& e = S.items[i];
        const double m = (double)e.m, p = (double)e.p, es = e.dtype == 0 ? 4.0 : 8.0;
        rows += m;
        byt_d += m * (es * p + 8.0);
        fl_d += m * (p * (p + 1.0) + 3.0 * p);
        // useful: h rows of the lower triangle of the sscp (with the sum and
        // count); executed: the matrix-core blocks over every candidate row
        const double g = std::ceil((p + 1.0) / 16.0);
        fl_su += (double)e.h * (p + 1.0) * (p + 2.0);
        fl_se += std::ceil(m / 4.0) * g * (g + 1.0) / 2.0 * 2048.0;
      }
      {
        ProfMark pm(ctx, RTDETMCD_PROF_CSTEP_DIST, s, byt_d, fl_d, fl_d);
        RTD_HIP(launch_dist(bucket, dtype, dense, D.items, dtab, dntab, dtile, D.A.mtri,
                            D.A.mux, D.A.status, form, D.A.d2, s));
        pm.end(s);
      }
      {
        ProfMark pm(ctx, RTDETMCD_PROF_SELECT, s, rows * 9.0);
        RTD_HIP(launch_select(D.items, D.A, first, n, max_m, o.cstep_mode, s, 1));
        pm.end(s);
      }
      double byt_s = 0.0;
      for (int i = first; i < first + n; ++i)
        byt_s += (double)S.items[i].m * ((S.items[i].dtype == 0 ? 4.0 : 8.0) * S.items[i].p + 1.0);
      {
        ProfMark pm(ctx, RTDETMCD_PROF_SSCP, s, byt_s, fl_su, fl_se);
        RTD_HIP(launch_sscp(bucket, dtype, SSCP_CSTEP, D.items, D.A, D.stiles + st0, stn,
                            SSCP_TILE, nullptr, nullptr, s));
        pm.end(s);
      }
      RTD_HIP(launch_collapse(D.items, D.A, first, n, max_nt, 1, SSCP_TILE, s));
      {
        ProfMark pm(ctx, RTDETMCD_PROF_FINALIZE, s, 0.0);
        RTD_HIP(launch_finalize(bucket, D.items, D.A, first, n, 0, maxs, o.kappa_max,
                                o.cstep_mode, o.distance, s));
        pm.end(s);
      }
      return RTDETMCD_OK;
    };
    int t = 1;
    if (ctx->prof_on) {
      RTD_TRY(step1(st));
      if (maxs == 1) {
        RTD_HIP(hipMemcpyAsync(pin_flag, D.A.nactive, 4, hipMemcpyDeviceToHost, st));
        RTD_HIP(hipStreamSynchronize(st));
        return RTDETMCD_OK;
      }
      t = 2;
    }
    if (o.graph && maxs >= R) {
      // whole rounds of R steps replayed from a captured graph on the
      // handle's replay stream, ordered after / before the caller's stream
      // every argument of every captured launch: the tables and the per-item
      // and per-row state arrays (their offsets in the workspace depend on
      // the item count and the total row count of the set), the grid sizes
      // and the options
      const ItemArrays& A = D.A;
      const void* ptrs[] = {ctx->ws,   D.items,  dtab,     D.stiles, A.status, A.iter,
                            A.kswap,   A.full,   A.logdet, A.mux,    A.lamx,   A.muz,
                            A.sigz,    A.linv,   A.mtri,   A.d2,     A.mask,   A.swap,
                            A.part,    A.nactive, A.form,  A.sinv,   A.ldtr};
      std::vector<int64_t> key;
      for (const void* q : ptrs) key.push_back((int64_t)(uintptr_t)q);
      int64_t kbits;
      std::memcpy(&kbits, &o.kappa_max, 8);
      const int64_t scal[] = {bucket, dtype, first, n, dense ? 1 : 0,
                              dntab, dtile, st0, stn, max_nt, max_m, (int64_t)S.items.size(),
                              S.rows, o.cstep_mode, maxs, R, kbits, o.distance};
      key.insert(key.end(), std::begin(scal), std::end(scal));
      hipGraphExec_t ge = nullptr;
      RTD_TRY(graph_for(ctx, key, R, step, &ge));
      RTD_HIP(hipEventRecord(ctx->gev[0], st));
      RTD_HIP(hipStreamWaitEvent(ctx->gstream, ctx->gev[0], 0));
      bool done = false;
      for (; t + R - 1 <= maxs; t += R) {   // (t = 2 after a profiled first step)
        RTD_HIP(hipGraphLaunch(ge, ctx->gstream));
        RTD_HIP(hipMemcpyAsync(pin_flag, D.A.nactive, 4, hipMemcpyDeviceToHost, ctx->gstream));
        RTD_HIP(hipStreamSynchronize(ctx->gstream));
        if (*pin_flag == 0) { done = true; break; }
      }
      RTD_HIP(hipEventRecord(ctx->gev[1], ctx->gstream));
      RTD_HIP(hipStreamWaitEvent(st, ctx->gev[1], 0));
      if (done) {
        if (tix >= 0) ctx->tune[tix].iters = t + R - 1;
        return RTDETMCD_OK;
      }
    }
    for (; t <= maxs; ++t) {
      RTD_TRY(step(st));
      if (t % R == 0 || t == maxs) {
        RTD_HIP(hipMemcpyAsync(pin_flag, D.A.nactive, 4, hipMemcpyDeviceToHost, st));
        RTD_HIP(hipStreamSynchronize(st));
        if (*pin_flag == 0) break;
      }
    }
    if (tix >= 0) ctx->tune[tix].iters = std::min(t, maxs);
    return RTDETMCD_OK;
  }
  // plain: one item at a time, host-driven, one host check per step
  for (int i = first; i < first + n; ++i) {
    const ItemDesc& d = S.items[i];
    RTD_HIP(launch_finalize(bucket, D.items, D.A, i, 1, 1, maxs, o.kappa_max, o.cstep_mode,
                            o.distance, st));
    RTD_HIP(hipMemcpyAsync(pin_flag, D.A.status + i, 4, hipMemcpyDeviceToHost, st));
    RTD_HIP(hipStreamSynchronize(st));
    if (*pin_flag != ACTIVE) continue;
    for (int t = 1; t <= maxs; ++t) {
      RTD_HIP(launch_dist(bucket, dtype, S.rows_dense(i, i + 1, bucket), D.items,
                          D.dtiles + S.dt_first[i], S.dt_count[i],
                          DIST_TILE, D.A.mtri, D.A.mux, D.A.status,
                          (o.distance || o.cstep_mode == RTDETMCD_CSTEP_SMW) ? D.A.form : nullptr,
                          D.A.d2, st));
      RTD_HIP(launch_select(D.items, D.A, i, 1, d.m, o.cstep_mode, st));
      RTD_HIP(launch_sscp(bucket, dtype, SSCP_CSTEP, D.items, D.A, D.stiles + d.tile0,
                          d.ntiles, SSCP_TILE, nullptr, nullptr, st));
      RTD_HIP(launch_collapse(D.items, D.A, i, 1, d.ntiles, 1, SSCP_TILE, st));
      RTD_HIP(launch_finalize(bucket, D.items, D.A, i, 1, 0, maxs, o.kappa_max, o.cstep_mode,
                              o.distance, st));
      RTD_HIP(hipMemcpyAsync(pin_flag, D.A.status + i, 4, hipMemcpyDeviceToHost, st));
      RTD_HIP(hipStreamSynchronize(st));
      if (*pin_flag != ACTIVE) break;
    }
  }
  return RTDETMCD_OK;
}

rtdetmcd_status check_opts(rtdetmcd_ctx* ctx, const rtdetmcd_opts* in, rtdetmcd_opts& o) {
  rtdetmcd_default_opts(&o);
  if (in) {
    if (in->struct_size != (int32_t)sizeof(rtdetmcd_opts)) {
      ctx->err = "rtdetmcd_opts.struct_size mismatch";
      return RTDETMCD_EINVAL;
    }
    o = *in;
  }
  if (!(o.alpha > 0.5 && o.alpha <= 1.0) || o.max_csteps < 1 || !(o.kappa_max > 1.0) ||
      !(o.cutoff_q > 0.0 && o.cutoff_q < 1.0) || o.omega < 1 || o.standardize < 0 ||
      o.standardize > 1 || o.cstep_mode < 0 || o.cstep_mode > 3 || o.pool_mode < 0 ||
      o.pool_mode > 1 || o.launch < 0 || o.launch > 1 || o.distance < 0 || o.distance > 1 ||
      o.tune < 0 || o.tune > 1) {
    ctx->err = "invalid option value";
    return RTDETMCD_EINVAL;
  }
  return RTDETMCD_OK;
}

namespace {

__global__ void k_cstep_init(const double* __restrict__ mu0, const double* __restrict__ s0,
                             const double* __restrict__ sc, int p, double* __restrict__ muz,
                             double* __restrict__ sigz, double* __restrict__ loc,
                             double* __restrict__ scale) {
  for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
    const int i = e / p, j = e % p;
    const double si = sc ? sc[i] : 1.0, sj = sc ? sc[j] : 1.0;
    sigz[i * PMAX + j] = s0[i * p + j] / (si * sj);
  }
  for (int j = threadIdx.x; j < p; j += blockDim.x) {
    const double s = sc ? sc[j] : 1.0;
    muz[j] = mu0[j] / s;
    loc[j] = 0.0;
    scale[j] = s;
  }
}

__global__ void k_cstep_out(const double* __restrict__ mux, const double* __restrict__ lamx,
                            const double* __restrict__ scale, const int32_t* __restrict__ status,
                            const int32_t* __restrict__ iter, const double* __restrict__ logdet,
                            int p, double h, double* mu, double* sigma, int32_t* st,
                            int32_t* its, double* ld) {
  const int s = *status;
  const bool ok = (s == ST_CONVERGED || s == ST_NOTCONV || s == ST_ILLCOND);
  for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
    const int i = e / p, j = e % p;
    if (sigma) sigma[e] = ok ? lamx[i * PMAX + j] / (h - 1.0) : NAN;
  }
  for (int j = threadIdx.x; j < p; j += blockDim.x)
    if (mu) mu[j] = ok ? mux[j] : NAN;
  if (threadIdx.x == 0) {
    if (st) *st = s;
    if (its) *its = *iter;
    if (ld) {
      double a = *logdet;
      for (int j = 0; j < p; ++j) a += 2.0 * log(scale[j]);
      *ld = ok ? a : NAN;
    }
  }
}

__global__ void k_copy_pad(const double* __restrict__ src, int p, double* __restrict__ dst) {
  for (int j = threadIdx.x; j < PMAX; j += blockDim.x) dst[j] = j < p ? src[j] : 0.0;
}

}  // namespace

hipError_t launch_cstep_init(const double* mu0, const double* sigma0, const double* kscale,
                             int p, const ItemArrays& A, double* loc, double* scale,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_cstep_init, dim3(1), dim3(256), 0, s, mu0, sigma0, kscale, p, A.muz,
                     A.sigz, loc, scale);
  return hipGetLastError();
}

hipError_t launch_cstep_out(const ItemArrays& A, const double* scale, int p, double h_sub,
                            double* mu, double* sigma, int32_t* status, int32_t* iters,
                            double* logdet, hipStream_t s) {
  hipLaunchKernelGGL(k_cstep_out, dim3(1), dim3(256), 0, s, A.mux, A.lamx, scale, A.status,
                     A.iter, A.logdet, p, h_sub, mu, sigma, status, iters, logdet);
  return hipGetLastError();
}

}  // namespace rtd

using namespace rtd;

extern "C" {

void rtdetmcd_default_opts(rtdetmcd_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = (int32_t)sizeof(rtdetmcd_opts);
  o->alpha = 0.75;
  o->standardize = RTDETMCD_STD_UNIMCD;
  o->cstep_mode = RTDETMCD_CSTEP_AUTO;
  o->max_csteps = 100;
  o->kappa_max = 1000.0;
  o->cutoff_q = 0.975;
  o->pool_mode = RTDETMCD_POOL_PRINTED;
  o->rew_consistency = 0;
  o->omega = 4096;
  o->launch = RTDETMCD_LAUNCH_BATCHED;
  o->graph = 0;
  o->rounds_per_sync = 4;
  o->distance = RTDETMCD_DIST_CHOLESKY;
  o->tune = 0;
}

rtdetmcd_status rtdetmcd_create(rtdetmcd_handle* out, int32_t device, void* hip_stream) {
  if (!out) return RTDETMCD_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return RTDETMCD_EDEVICE;
  rtdetmcd_ctx* c = new rtdetmcd_ctx();
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  const char* safe = std::getenv("RTDETMCD_SAFE_SORT");
  c->sort_safe = (safe && safe[0] == '1') ? 1 : 0;
  if (hipSetDevice(device) != hipSuccess ||
      hipEventCreateWithFlags(&c->pin_ev, hipEventDisableTiming) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&c->flag), 256, hipHostMallocDefault) != hipSuccess) {
    delete c;
    return RTDETMCD_EDEVICE;
  }
  // the allocation-free entry point's array on this device (looked up once
  // per device, with the device current)
  c->scratch = noalloc_scratch(device, &c->scratch_bytes);
  *out = c;
  return RTDETMCD_OK;
}

rtdetmcd_status rtdetmcd_destroy(rtdetmcd_handle ctx) {
  if (!ctx) return RTDETMCD_EINVAL;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->gstream) (void)hipStreamSynchronize(ctx->gstream);
  drop_graphs(ctx);
  if (ctx->gstream) (void)hipStreamDestroy(ctx->gstream);
  for (hipEvent_t e : ctx->gev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->pin) (void)hipHostFree(ctx->pin);
  if (ctx->pin_ev) (void)hipEventDestroy(ctx->pin_ev);
  if (ctx->flag) (void)hipHostFree(ctx->flag);
  if (ctx->stage) (void)hipFree(ctx->stage);
  for (hipEvent_t e : ctx->prof_events) (void)hipEventDestroy(e);
  for (const auto& tp : ctx->tune) (void)hipFree(tp.tiles);
  delete ctx;
  return RTDETMCD_OK;
}

rtdetmcd_status rtdetmcd_tuned_plans(rtdetmcd_handle ctx, int64_t* out, int32_t cap,
                                     int32_t* count) {
  if (!ctx || !count || cap < 0 || (cap > 0 && !out)) return RTDETMCD_EINVAL;
  *count = (int32_t)ctx->tune.size();
  for (int k = 0; k < (int)ctx->tune.size() && k < cap; ++k) {
    const auto& tp = ctx->tune[k];
    out[4 * k] = tp.bucket;
    out[4 * k + 1] = tp.tile_rows;
    out[4 * k + 2] = tp.mode;
    out[4 * k + 3] = tp.iters;
  }
  return RTDETMCD_OK;
}

rtdetmcd_status rtdetmcd_set_stream(rtdetmcd_handle ctx, void* hip_stream) {
  if (!ctx) return RTDETMCD_EINVAL;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return RTDETMCD_OK;
}

const char* rtdetmcd_last_error(rtdetmcd_handle ctx) { return ctx ? ctx->err.c_str() : "null handle"; }

double rtdetmcd_chi2_quantile(double q, int32_t df) { return rtd::chi2_quantile(q, df); }
double rtdetmcd_chi2_cdf(double x, int32_t df) { return rtd::chi2_cdf(x, df); }
double rtdetmcd_consistency(double alpha, int32_t p) { return rtd::consistency(alpha, p); }

rtdetmcd_status rtdetmcd_plan(int64_t n, int32_t p, int64_t h_sub, int32_t n_chunks,
                              const rtdetmcd_opts* o_in, int32_t* q, int64_t* m, int64_t* h) {
  rtdetmcd_opts o;
  rtdetmcd_default_opts(&o);
  if (o_in) o = *o_in;
  if (p < 1 || n <= 2 * (int64_t)p || n_chunks < 0 || h_sub < 0) return RTDETMCD_EINVAL;
  if (p > RTDETMCD_MAX_P) return RTDETMCD_EUNSUPPORTED;
  int64_t qq = n_chunks > 0 ? n_chunks : std::max<int64_t>(n / ((int64_t)p * o.omega), 1);
  if (qq > n) return RTDETMCD_EINVAL;
  if (qq > 8192) return RTDETMCD_EUNSUPPORTED;   // aggregation keeps at most 4096 blocks
  const int64_t mm = n / qq;
  int64_t hh = h_sub;
  if (hh == 0) {
    hh = (int64_t)std::floor(o.alpha * (double)mm);
    hh = std::max<int64_t>(hh, (mm + p + 1) / 2);
    hh = std::min<int64_t>(hh, mm - 1);
  }
  if (!(hh > p && hh < mm)) return RTDETMCD_EINVAL;
  if (mm > INT32_MAX) return RTDETMCD_EUNSUPPORTED;
  if (q) *q = (int32_t)qq;
  if (m) *m = mm;
  if (h) *h = hh;
  return RTDETMCD_OK;
}

rtdetmcd_status rtdetmcd_distances(rtdetmcd_handle ctx, const void* X, int32_t dtype, int64_t n,
                                   int32_t p, int64_t ld, const double* mu, const double* L,
                                   double* d2) {
  if (!ctx) return RTDETMCD_EINVAL;
  if (n == 0 && p >= 1 && p <= RTDETMCD_MAX_P && (dtype == 0 || dtype == 1))
    return RTDETMCD_OK;   // no rows: nothing is read or written
  if (!X || !mu || !L || !d2 || n < 0 || p < 1 || ld < p || (dtype != 0 && dtype != 1)) {
    ctx->err = "rtdetmcd_distances: bad argument";
    return RTDETMCD_EINVAL;
  }
  if (p > RTDETMCD_MAX_P) return RTDETMCD_EUNSUPPORTED;
  RTD_HIP(hipSetDevice(ctx->device));
  ItemSet S;
  ItemDesc d{};
  d.X = X; d.ld = ld; d.row0 = 0; d.m = n; d.h = 0; d.p = p; d.dtype = dtype; d.start = -1;
  S.add(d);
  Layout L0;
  size_t off[NOFF];
  layout_items(L0, S, off);
  // only items, tiles, mux and mtri are used
  RTD_TRY(ensure_ws(ctx, L0.off));
  ItemDev D;
  bind_items(static_cast<char*>(ctx->ws), S, off, D);
  Uploader up;
  up.add(D.items, S.items.data(), S.items.size());
  up.add(D.dtiles, S.dtiles.data(), S.dtiles.size());
  RTD_TRY(up.flush(ctx));
  hipLaunchKernelGGL(k_copy_pad, dim3(1), dim3(64), 0, ctx->stream, mu, p, D.A.mux);
  RTD_HIP(hipGetLastError());
  RTD_HIP(launch_chol_factor(L, p, D.A.mtri, ctx->stream));
  // the distance kernel writes d2 + roff with roff = 0
  const double es = dtype == 0 ? 4.0 : 8.0;
  ProfMark pm(ctx, RTDETMCD_PROF_DISTANCES, ctx->stream, (double)n * (es * p + 8.0),
              (double)n * (p * (p + 1.0) + 3.0 * p));
  RTD_HIP(launch_dist(bucket_of(p), dtype, S.rows_dense(0, (int)S.items.size(), bucket_of(p)),
                      D.items, D.dtiles, (int)S.dtiles.size(), DIST_TILE,
                      D.A.mtri, D.A.mux, nullptr, nullptr, d2, ctx->stream));
  pm.end(ctx->stream);
  return RTDETMCD_OK;
}

rtdetmcd_status rtdetmcd_score(rtdetmcd_handle ctx, const void* X, int32_t dtype, int64_t n,
                               int32_t p, int64_t ld, const double* mu, const double* Linv,
                               double cut, double* dist, uint8_t* outlier) {
  if (!ctx) return RTDETMCD_EINVAL;
  if (n == 0 && p >= 1 && p <= RTDETMCD_MAX_P && (dtype == 0 || dtype == 1))
    return RTDETMCD_OK;   // no rows: nothing is read or written
  if (!X || !mu || !Linv || n < 0 || p < 1 || ld < p || (dtype != 0 && dtype != 1)) {
    ctx->err = "rtdetmcd_score: bad argument";
    return RTDETMCD_EINVAL;
  }
  if (p > RTDETMCD_MAX_P) return RTDETMCD_EUNSUPPORTED;
  RTD_HIP(hipSetDevice(ctx->device));
  const double c = cut > 0.0 ? cut : chi2_quantile(0.975, p);
  const double es = dtype == 0 ? 4.0 : 8.0;
  ProfMark pm(ctx, RTDETMCD_PROF_DISTANCES, ctx->stream,
              (double)n * (es * p + (dist ? 8.0 : 0.0) + (outlier ? 1.0 : 0.0)),
              (double)n * (p * (p + 1.0) + 3.0 * p));
  RTD_HIP(launch_score(bucket_of(p), dtype, X, n, ld, p, mu, Linv, p, c, dist, outlier,
                       ctx->stream));
  pm.end(ctx->stream);
  return RTDETMCD_OK;
}

rtdetmcd_status rtdetmcd_select(rtdetmcd_handle ctx, const double* d2, int64_t m, int64_t h_sub,
                                int32_t* idx, uint8_t* mask) {
  if (!ctx) return RTDETMCD_EINVAL;
  if (!d2 || !idx || m < 1 || h_sub < 1 || h_sub > m || m > INT32_MAX) {
    ctx->err = "rtdetmcd_select: bad argument";
    return RTDETMCD_EINVAL;
  }
  RTD_HIP(hipSetDevice(ctx->device));
  ItemSet S;
  ItemDesc d{};
  d.m = m; d.h = h_sub; d.p = 1; d.start = -1;
  S.add(d);
  Layout L0;
  size_t off[NOFF];
  layout_items(L0, S, off);
  RTD_TRY(ensure_ws(ctx, L0.off));
  ItemDev D;
  bind_items(static_cast<char*>(ctx->ws), S, off, D);
  Uploader up;
  up.add(D.items, S.items.data(), 1);
  RTD_TRY(up.flush(ctx));
  hipStream_t st = ctx->stream;
  ItemArrays A = D.A;
  A.d2 = const_cast<double*>(d2);
  RTD_HIP(launch_fill_i32(A.status, ACTIVE, 1, st));
  RTD_HIP(launch_fill_i32(A.iter, 0, 1, st));
  RTD_HIP(launch_fill_u8(A.mask, 0, m, st));
  RTD_HIP(launch_select(D.items, A, 0, 1, m, RTDETMCD_CSTEP_FULL, st));
  RTD_HIP(launch_extract_subset(D.items, A, 0, 1, idx, h_sub, 0, st));
  if (mask) RTD_HIP(hipMemcpyAsync(mask, A.mask, (size_t)m, hipMemcpyDeviceToDevice, st));
  return RTDETMCD_OK;
}

rtdetmcd_status rtdetmcd_cstep(rtdetmcd_handle ctx, const void* X, int32_t dtype, int64_t m,
                               int32_t p, int64_t ld, int64_t h_sub, const double* mu0,
                               const double* sigma0, const double* kappa_scale,
                               const rtdetmcd_opts* o_in, double* mu, double* sigma,
                               int32_t* hsubset, int32_t* status, int32_t* iters,
                               double* logdet) {
  if (!ctx) return RTDETMCD_EINVAL;
  rtdetmcd_opts o;
  RTD_TRY(check_opts(ctx, o_in, o));
  if (!X || !mu0 || !sigma0 || p < 1 || ld < p || !(h_sub > p && h_sub < m) ||
      m > INT32_MAX || (dtype != 0 && dtype != 1)) {
    ctx->err = "rtdetmcd_cstep: bad argument (need p < h < m)";
    return RTDETMCD_EINVAL;
  }
  if (p > RTDETMCD_MAX_P) return RTDETMCD_EUNSUPPORTED;
  RTD_HIP(hipSetDevice(ctx->device));
  ItemSet S;
  ItemDesc d{};
  d.X = X; d.ld = ld; d.row0 = 0; d.m = m; d.h = h_sub; d.p = p; d.dtype = dtype; d.start = -1;
  S.add(d);
  Layout L0;
  size_t off[NOFF];
  layout_items(L0, S, off);
  const size_t o_loc = L0.add(PMAX * 8), o_scale = L0.add(PMAX * 8), o_flag = L0.add(64);
  RTD_TRY(ensure_ws(ctx, L0.off));
  char* base = static_cast<char*>(ctx->ws);
  ItemDev D;
  bind_items(base, S, off, D);
  double* loc = reinterpret_cast<double*>(base + o_loc);
  double* scale = reinterpret_cast<double*>(base + o_scale);
  (void)o_flag;
  S.items[0].loc = loc;
  S.items[0].scale = scale;
  Uploader up;
  up.add(D.items, S.items.data(), 1);
  up.add(D.dtiles, S.dtiles.data(), S.dtiles.size());
  up.add(D.stiles, S.stiles.data(), S.stiles.size());
  RTD_TRY(up.flush(ctx));
  hipStream_t st = ctx->stream;
  RTD_HIP(launch_cstep_init(mu0, sigma0, kappa_scale, p, D.A, loc, scale, st));
  RTD_HIP(launch_fill_i32(D.A.status, ACTIVE, 1, st));
  RTD_HIP(launch_fill_i32(D.A.iter, 0, 1, st));
  RTD_HIP(launch_fill_u8(D.A.mask, 0, m, st));
  RTD_TRY(run_csteps(ctx, S, D, bucket_of(p), dtype, 0, 1, o, ctx->flag));
  RTD_HIP(launch_cstep_out(D.A, scale, p, (double)h_sub, mu, sigma, status, iters, logdet, st));
  if (hsubset) RTD_HIP(launch_extract_subset(D.items, D.A, 0, 1, hsubset, h_sub, 0, st));
  return RTDETMCD_OK;
}

int64_t rtdetmcd_sort_reruns(rtdetmcd_handle ctx) { return ctx ? ctx->sort_reruns : -1; }

rtdetmcd_status rtdetmcd_profile(rtdetmcd_handle ctx, int32_t enable) {
  if (!ctx) return RTDETMCD_EINVAL;
  ctx->prof_on = enable != 0;
  if (ctx->prof_on) {
    RTD_HIP(hipSetDevice(ctx->device));
    RTD_HIP(hipStreamSynchronize(ctx->stream));   // every recorded event has completed
    ctx->prof.clear();
    ctx->prof_next = 0;
  }
  return RTDETMCD_OK;
}

rtdetmcd_status rtdetmcd_profile_read(rtdetmcd_handle ctx, int32_t kind, double* ms,
                                      int64_t* launches, double* bytes, double* flops_useful,
                                      double* flops_exec) {
  if (!ctx || kind < 0 || kind >= RTDETMCD_PROF_KINDS) return RTDETMCD_EINVAL;
  RTD_HIP(hipSetDevice(ctx->device));
  RTD_HIP(hipStreamSynchronize(ctx->stream));
  double t = 0.0, b = 0.0, fu = 0.0, fe = 0.0;
  int64_t k = 0;
  for (const auto& r : ctx->prof) {
    if (r.kind != kind || !r.e1) continue;
    float x = 0.0f;
    RTD_HIP(hipEventElapsedTime(&x, r.e0, r.e1));
    t += x;
    b += r.bytes;
    fu += r.flops_useful;
    fe += r.flops_exec;
    ++k;
  }
  if (ms) *ms = t;
  if (launches) *launches = k;
  if (bytes) *bytes = b;
  if (flops_useful) *flops_useful = fu;
  if (flops_exec) *flops_exec = fe;
  return RTDETMCD_OK;
}

}  // extern "C"
