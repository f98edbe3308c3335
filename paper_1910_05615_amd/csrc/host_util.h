// Host-side helpers of librtdetmcd: chi-square distribution, consistency
// factor, the block-count and subset-size rules, and the handle/workspace.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "common.h"

namespace rtd {

// Regularised lower incomplete gamma P(a, x): power series for x < a + 1,
// otherwise 1 - Q with Q from the Legendre continued fraction evaluated by the
// modified Lentz method (the classical series / continued-fraction pair).
inline double gamma_p(double a, double x) {
  if (x <= 0.0) return 0.0;
  const double lg = std::lgamma(a);
  if (x < a + 1.0) {
    double ap = a, sum = 1.0 / a, del = sum;
    for (int n = 0; n < 10000; ++n) {
      ap += 1.0;
      del *= x / ap;
      sum += del;
      if (std::fabs(del) < std::fabs(sum) * 1e-17) break;
    }
    return sum * std::exp(-x + a * std::log(x) - lg);
  }
  const double tiny = 1e-300;
  double b = x + 1.0 - a, c = 1.0 / tiny, d = 1.0 / b, hh = d;
  for (int i = 1; i < 10000; ++i) {
    const double an = -i * (i - a);
    b += 2.0;
    d = an * d + b;
    if (std::fabs(d) < tiny) d = tiny;
    c = b + an / c;
    if (std::fabs(c) < tiny) c = tiny;
    d = 1.0 / d;
    const double del = d * c;
    hh *= del;
    if (std::fabs(del - 1.0) < 1e-17) break;
  }
  return 1.0 - std::exp(-x + a * std::log(x) - lg) * hh;
}

inline double chi2_cdf(double x, double df) { return gamma_p(0.5 * df, 0.5 * x); }

// Quantile by bracketing and bisection to the last bit.
inline double chi2_quantile(double q, double df) {
  if (q <= 0.0) return 0.0;
  double lo = 0.0, hi = df + 10.0;
  while (chi2_cdf(hi, df) < q) hi *= 2.0;
  for (int i = 0; i < 2000; ++i) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (chi2_cdf(mid, df) < q) lo = mid;
    else hi = mid;
  }
  return 0.5 * (lo + hi);
}

// Gaussian consistency factor of the raw MCD scatter at coverage alpha
// (Sec. 2.1): alpha / F_{chi2_{p+2}}(chi2_{p,alpha}).
inline double consistency(double alpha, int p) {
  if (alpha >= 1.0) return 1.0;
  return alpha / chi2_cdf(chi2_quantile(alpha, p), p + 2);
}

// The same two functions remembered per thread: a fit asks for the same few
// values (one per block length and p) many times, and each costs a bisection
// over the incomplete gamma function.
inline double memo_lookup(int kind, double x, double df, double (*f)(double, double)) {
  struct Key {
    int kind;
    uint64_t x, df;
    bool operator==(const Key& o) const { return kind == o.kind && x == o.x && df == o.df; }
  };
  struct Hash {
    size_t operator()(const Key& k) const {
      return std::hash<uint64_t>()(k.x * 0x9E3779B97F4A7C15ull ^ k.df) ^ (size_t)k.kind;
    }
  };
  thread_local std::unordered_map<Key, double, Hash> memo;
  uint64_t bx, bd;
  std::memcpy(&bx, &x, 8);
  std::memcpy(&bd, &df, 8);
  const Key k{kind, bx, bd};
  const auto it = memo.find(k);
  if (it != memo.end()) return it->second;
  const double v = f(x, df);
  if (memo.size() > 65536) memo.clear();
  memo.emplace(k, v);
  return v;
}
inline double chi2_quantile_memo(double q, double df) {
  return memo_lookup(0, q, df, [](double a, double b) { return chi2_quantile(a, b); });
}
inline double consistency_memo(double alpha, int p) {
  return memo_lookup(1, alpha, (double)p,
                     [](double a, double b) { return consistency(a, (int)b); });
}

}  // namespace rtd

// A captured round of C-steps and every kernel argument it was captured
// with (pointers, grid sizes, options): a replay is valid only when all of
// them are the same again.
struct rtd_graph {
  std::vector<int64_t> key;
  hipGraphExec_t exec = nullptr;
};

struct rtdetmcd_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  void* ws = nullptr;          // device workspace (grow only)
  size_t ws_size = 0;
  void* pin = nullptr;         // pinned host staging (grow only)
  size_t pin_size = 0;
  hipEvent_t pin_ev = nullptr; // last upload out of the staging buffer
  void* stage = nullptr;       // device copy of the pinned staging buffer (grow only)
  size_t stage_size = 0;
  bool pin_pending = false;
  int32_t* flag = nullptr;     // pinned readback word
  int sort_safe = 0;           // 1: global sorts rank with ballots (no order check)
  int64_t sort_reruns = 0;     // fits run again with ballot ranking (an order check failed)
  hipStream_t gstream = nullptr;          // capture / replay stream (created on first use)
  hipEvent_t gev[2] = {nullptr, nullptr}; // ordering with `stream`
  std::vector<rtd_graph> graphs;          // captured C-step rounds, most recent last
  void* scratch = nullptr;     // this device's allocation-free scratch array (device address)
  size_t scratch_bytes = 0;
  // kernel timing (rtdetmcd_profile): HIP events around chosen launches
  struct ProfRec {
    int kind;
    hipEvent_t e0, e1;
    double bytes, flops_useful, flops_exec;
  };
  bool prof_on = false;
  std::vector<ProfRec> prof;
  std::vector<hipEvent_t> prof_events;   // every event created for profiling (reused)
  size_t prof_next = 0;                  // next free event of prof_events
  // autotuned C-step plans (opts.tune): shape key -> distance tiling (with
  // its device tile table) and the C-step count of the last fit
  struct TunePlan {
    std::vector<int64_t> key;
    int bucket = 0, tile_rows = 0, mode = 1, iters = 0;
    rtd::Tile* tiles = nullptr;            // device table of the kept tiling
    int ntiles = 0;
  };
  std::vector<TunePlan> tune;
};
