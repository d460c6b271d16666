// Host side of drtopk: planner, per-stream workspace, kernel sequence, C-ABI.
//
// One call enqueues, on the caller's stream and with no host synchronisation:
//   k_init -> delegate pass (+ first digit of the delegate select) -> five more
//   digit passes over the delegates (threshold t, Rule 2) -> qualify (Rule 3)
//   -> scan of the qualifying subranges -> survivor select -> sorted output.
// Small survivor counts finish in one LDS-resident workgroup; large ones take
// the multi-workgroup radix select, an exact compaction and a merge sort.  The
// host cannot see the survivor count, so both routes are enqueued and each
// kernel checks a device-side gate and returns at once when not needed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "drtopk.h"
#include "host.h"
#include "batched.h"
#include "wide_host.h"

namespace drtopk {

thread_local hipError_t tl_launch_err = hipSuccess;
Timing g_timing;

namespace {

constexpr double kAlphaConst = 3.0;  // Rule 4's const; the paper tuned it to 3


size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }


int rule_alpha(uint64_t n, uint32_t k) {
  const double a = 0.5 * (std::log2((double)n) - std::log2((double)k) + kAlphaConst);
  int al = (int)std::floor(a);
  if (al < 2) al = 2;
  if (al > 24) al = 24;
  return al;
}

// Rule 4's alpha, adjusted by measurement on MI355X: beta = 2 adds 2 (its
// lane merges want longer subranges); beta = 1 on large inputs adds 1, at
// most 13 (the delegate pass streams fastest with 2^12..2^14-key subranges:
// n = 2^30, k = 1: 652 us at alpha 13 against 693 us at Rule 4's 16; k = 1024:
// 707 us per call at alpha 12 against 722 us at 11).
int planned_alpha(uint64_t n, uint32_t k, int beta) {
  int a = rule_alpha(n, k);
  if (beta >= 2) return a + 2;
  if (n >= (1ull << 24)) a = a + 1 < 13 ? a + 1 : (a > 13 ? 13 : a);
  return a;
}

// Two delegates per subrange pay off for large k on large inputs only
// (measured on MI355X: at n <= 2^24 and k = 2^13..2^17, beta = 1 at Rule 4's
// alpha is 15-29% faster than beta = 2).
int default_beta(uint64_t n, uint32_t k) {
  return (k <= 4096 || n < (1ull << 25)) ? 1 : 2;
}

bool valid_beta(int b) { return b == 1 || b == 2 || b == 4 || b == 8; }

// Testing hook: survivor-buffer capacity of the delegate method (0 = the
// planner's bound).  A smaller cap makes the kernels drop writes and flag it.
std::atomic<uint64_t> g_cap_override{0};

int floor_log2(uint64_t x) { return 63 - __builtin_clzll(x); }

// Autotuner table: measured (alpha, beta) per (form, floor log2 n, floor log2 k).
std::mutex g_tune_mu;
std::vector<drtopk_tune_t> g_tune;

bool tune_lookup(int form, uint64_t n, uint32_t k, int* alpha, int* beta) {
  const int ln = floor_log2(n), lk = floor_log2(k);
  std::lock_guard<std::mutex> g(g_tune_mu);
  for (const auto& e : g_tune)
    if (e.form == form && e.lg_n == ln && e.lg_k == lk) {
      *alpha = e.alpha;
      *beta = e.beta;
      return true;
    }
  return false;
}

int batched_alpha(uint64_t n, uint32_t k, int* beta = nullptr);
bool batched_eligible(uint64_t n, uint32_t k);

// Problems up to this size (and k <= kBMaxK) finish faster in one workgroup
// than across the device: one launch, no workspace.
constexpr uint64_t kOneWgMaxN = 1ull << 16;

int make_plan(const void* keys, uint64_t n, uint32_t k, int dt, const drtopk_options_t* opt, Plan* P,
              bool pos_in_ws = false) {
  Plan p;
  p.n = n;
  p.k = k;
  p.dt = dt;
  p.vec = (reinterpret_cast<uintptr_t>(keys) & 15u) == 0;
  int mode = opt ? opt->mode : 0;
  if (mode < 0 || mode > 3) return DRTOPK_EINVAL;
  if (mode == 3 && !batched_eligible(n, k)) return DRTOPK_EINVAL;
  if (mode == 0) {
    // k = 1 above 2^14 keys: the delegate pass alone answers it device-wide
    if (n <= kOneWgMaxN && batched_eligible(n, k) && !(k == 1 && n > (1u << 14))) mode = 3;
    else mode = (n <= (uint64_t)kSmallCap || (uint64_t)k * 16 > n) ? 2 : 1;
  }
  if (mode == 3) p.alpha = batched_alpha(n, k, &p.beta);
  p.mode = mode;
  p.variant = opt ? opt->variant : 0;
  if (p.variant < 0 || p.variant > 3) return DRTOPK_EINVAL;
  if (p.variant == 2 && k > kBtMaxK) return DRTOPK_EINVAL;  // the bitonic top-k holds k <= 256
  if (mode == 1) {
    int ta = -1, tb = 0;
    if (!tune_lookup(DRTOPK_FORM_SINGLE, n, k, &ta, &tb)) ta = -1, tb = 0;
    p.beta = (opt && opt->beta > 0) ? opt->beta : tb > 0 ? tb : default_beta(n, k);
    if (!valid_beta(p.beta)) return DRTOPK_EINVAL;
    if (opt && opt->alpha > 24) return DRTOPK_EINVAL;
    p.alpha = (opt && opt->alpha >= 0) ? opt->alpha
              : ta >= 0                ? ta
                                       : planned_alpha(n, k, p.beta);
    if (p.alpha > 24) p.alpha = 24;
    const uint64_t L = 1ull << p.alpha;
    p.S = (n + L - 1) >> p.alpha;
    p.nd = p.S * (uint64_t)p.beta;
    if (p.nd >= (1ull << 32)) return DRTOPK_EINVAL;  // delegate vector must be indexable by 32 bits
    const uint64_t full = n >> p.alpha, last = n & (L - 1);
    const uint64_t per_full = L < (uint64_t)p.beta ? L : (uint64_t)p.beta;
    const uint64_t nd_valid = full * per_full + (last < (uint64_t)p.beta ? last : (uint64_t)p.beta);
    p.kD = p.nd < (uint64_t)k ? (uint32_t)p.nd : k;
    // survivors: at most floor(m/beta)*L + m when m delegates rank at or above
    // the threshold; the tail keeps m <= kD + slack (exact threshold otherwise)
    p.slack = p.kD / 8 > 64 ? p.kD / 8 : 64;
    if (nd_valid < k) {
      p.cap_c = n;
      p.all = true;
    } else {
      const uint64_t m = (uint64_t)p.kD + p.slack;
      const uint64_t c = (m / p.beta) * L + m;
      p.cap_c = c < n ? c : n;
    }
    const uint64_t cap_hook = g_cap_override.load(std::memory_order_relaxed);
    if (cap_hook && cap_hook < p.cap_c) p.cap_c = cap_hook;
    // one block per chunk, about 1024 blocks: at n = 2^30 that is 4 MiB
    // chunks (one round of blocks), which stream best for beta = 1; beta > 1
    // needs the parallelism of 1 MiB chunks for its merges.  A chunk holds
    // whole subranges (4 per wave) and whole unrolled wave steps.
    const uint64_t cmax = p.beta == 1 ? (1ull << 20) : (1ull << 18);
    const uint64_t cmin = 4 * L > 8192 ? 4 * L : 8192;
    uint64_t c = 1;
    while (c * 2 <= n / 1024) c *= 2;
    if (c > cmax) c = cmax;
    if (c < cmin) c = cmin;
    p.chunk = c;
  }
  if (k > (uint32_t)kSmallCap) {
    uint64_t tiles = ((uint64_t)k + kSortTile - 1) / kSortTile, t2 = 1;
    while (t2 < tiles) t2 <<= 1;
    p.M = t2 * kSortTile;
  }
  size_t off = 0;
  auto seg = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  p.off_ctl = seg(sizeof(Ctl));
  if (mode == 1) {
    p.off_dkey = seg(p.nd * 4);
    p.off_didx = seg(p.nd * 4);
    p.off_q = seg(p.S * 4);
    p.off_ckey = seg(p.cap_c * 4);
    p.off_cidx = seg(p.cap_c * 4);
    if (p.variant == 0) {
      p.off_skey = seg(p.cap_c * 4);  // survivors scattered into output-bucket order
      p.off_sidx = seg(p.cap_c * 4);
    }
  }
  if (mode == 1 && p.variant == 2) {  // partial lists of the bitonic rounds
    p.off_L0 = seg((size_t)kBtRoundBlocks * kBtMaxK * 8);
    p.off_L1 = seg((size_t)kBtRoundBlocks * kBtMaxK * 8);
  }
  if (pos_in_ws) p.off_pos = seg((size_t)k * 4);
  p.off_okey = seg((size_t)k * 4);
  p.off_oidx = seg((size_t)k * 4);
  if (p.M) {
    p.off_A = seg(p.M * 8);
    p.off_B = seg(p.M * 8);
  }
  p.total = off;
  *P = p;
  return DRTOPK_OK;
}

// ---------------------------------------------------------------------------
// workspace: one per (device, stream); a call holds its entry's lock while it
// enqueues, so sequences on one stream never interleave.
struct Workspace {
  std::mutex mu;
  void* ptr = nullptr;
  size_t bytes = 0;
  // batched launches: claim counter + descriptors on the device, staged
  // through a pinned host buffer whose last copy `bev` marks
  void* bdev = nullptr;
  size_t bdev_bytes = 0;
  void* bhost = nullptr;
  size_t bhost_bytes = 0;
  hipEvent_t bev = nullptr;
  bool bev_pending = false;
  // check record of the calls on this stream: kErrWords words in pinned host
  // memory, written by kernels whose internal checks fail, read and cleared
  // by drtopk_check (kept across drtopk_release_workspace)
  uint32_t* rec = nullptr;
};

std::mutex g_mu;
std::map<std::pair<int, void*>, std::unique_ptr<Workspace>> g_ws;

Workspace* workspace_entry(int dev, void* stream) {
  std::lock_guard<std::mutex> g(g_mu);
  auto& slot = g_ws[{dev, stream}];
  if (!slot) slot.reset(new (std::nothrow) Workspace());
  return slot.get();
}

// Existing entry of (dev, stream), or null (never creates one).
Workspace* find_workspace(int dev, void* stream) {
  std::lock_guard<std::mutex> g(g_mu);
  auto it = g_ws.find({dev, stream});
  return it == g_ws.end() ? nullptr : it->second.get();
}

// Called with ws->mu held: the stream's check record exists (zeroed).
int ensure_record(Workspace* ws) {
  if (ws->rec) return DRTOPK_OK;
  void* p = nullptr;
  if (hipHostMalloc(&p, kErrWords * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return DRTOPK_ENOMEM;
  }
  std::memset(p, 0, kErrWords * sizeof(uint32_t));
  ws->rec = static_cast<uint32_t*>(p);
  return DRTOPK_OK;
}

// Flags held by a check record (bit i <=> word i set); clears it when `reset`.
uint32_t read_record(volatile uint32_t* rec, bool reset) {
  uint32_t f = 0;
  for (int i = 0; i < kErrWords; ++i) {
    if (rec[i]) f |= 1u << i;
    if (reset) rec[i] = 0;
  }
  return f;
}

// Called with ws->mu held.
int ensure_bytes(Workspace* ws, size_t need) {
  if (ws->bytes >= need) return DRTOPK_OK;
  if (ws->ptr) {
    if (hipFree(ws->ptr) != hipSuccess) return DRTOPK_EDEVICE;
    ws->ptr = nullptr;
    ws->bytes = 0;
  }
  size_t want = need + need / 8;  // headroom to avoid regrowing on small changes
  void* p = nullptr;
  if (hipMalloc(&p, want) != hipSuccess) {
    (void)hipGetLastError();
    if (hipMalloc(&p, need) != hipSuccess) {
      (void)hipGetLastError();
      return DRTOPK_ENOMEM;
    }
    want = need;
  }
  ws->ptr = p;
  ws->bytes = want;
  return DRTOPK_OK;
}

// Called with ws->mu held: room for `need` bytes of batch descriptors on both
// sides and `dev_need` >= need bytes on the device; the pinned buffer is free
// to overwrite on return.
int ensure_batch_bytes(Workspace* ws, size_t need, size_t dev_need) {
  if (ws->bev_pending) {
    if (hipEventSynchronize(ws->bev) != hipSuccess) return DRTOPK_EDEVICE;
    ws->bev_pending = false;
  }
  if (!ws->bev && hipEventCreateWithFlags(&ws->bev, hipEventDisableTiming) != hipSuccess) {
    ws->bev = nullptr;
    return DRTOPK_EDEVICE;
  }
  if (ws->bdev_bytes < dev_need) {
    if (ws->bdev) {
      if (hipFree(ws->bdev) != hipSuccess) return DRTOPK_EDEVICE;
      ws->bdev = nullptr;
      ws->bdev_bytes = 0;
    }
    if (hipMalloc(&ws->bdev, dev_need) != hipSuccess) {
      (void)hipGetLastError();
      ws->bdev = nullptr;
      return DRTOPK_ENOMEM;
    }
    ws->bdev_bytes = dev_need;
  }
  if (ws->bhost_bytes < need) {
    if (ws->bhost) {
      if (hipHostFree(ws->bhost) != hipSuccess) return DRTOPK_EDEVICE;
      ws->bhost = nullptr;
      ws->bhost_bytes = 0;
    }
    if (hipHostMalloc(&ws->bhost, need, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      ws->bhost = nullptr;
      return DRTOPK_ENOMEM;
    }
    ws->bhost_bytes = need;
  }
  return DRTOPK_OK;
}







// Public dtype (DRTOPK_U32 / F32 / I32, optionally | DRTOPK_SMALLEST) to the
// kernels' codec.
bool dtype_ok(int dtype) {
  const int base = dtype & ~DRTOPK_SMALLEST;
  return base == DRTOPK_U32 || base == DRTOPK_F32 || base == DRTOPK_I32 || wide_dtype(dtype);
}
int dt_code(int dtype) {
  const int base = dtype & ~DRTOPK_SMALLEST;
  const int t = base == DRTOPK_F32 ? DT_F32 : base == DRTOPK_I32 ? DT_I32 : DT_U32;
  return t | ((dtype & DRTOPK_SMALLEST) ? DT_MIN : 0);
}

int check_args(const void* keys, uint64_t n, uint32_t k, int dtype) {
  if (!keys) return DRTOPK_EINVAL;
  if (n == 0 || n >= (1ull << 32)) return DRTOPK_EINVAL;
  if (k == 0 || (uint64_t)k > n) return DRTOPK_EINVAL;
  if (!dtype_ok(dtype)) return DRTOPK_EINVAL;
  if (wide_dtype(dtype) && (reinterpret_cast<uintptr_t>(keys) & 7u) != 0) return DRTOPK_EINVAL;
  return DRTOPK_OK;
}

// Input bit pattern of an encoded key (the inverse of enc<DT>, on the host).
uint32_t host_dec(int code, uint32_t u) {
  if (code & DT_MIN) u = ~u;
  switch (code & 3) {
    case DT_F32: return u ^ (((u >> 31) - 1u) | 0x80000000u);
    case DT_I32: return u ^ 0x80000000u;
    default: return u;
  }
}

// Enqueues the kernels of plan p on stream s over the workspace `ws` (at
// least p.total bytes; p.rec set).
int enqueue_plan(const Plan& p, const void* keys, void* ws, void* out_vals, uint32_t* out_idx, void* out_kth,
                 bool kth_only, bool filter_only, hipStream_t s) {
  const uint32_t* kp = static_cast<const uint32_t*>(keys);
  if (p.mode == 3) {
    if (filter_only) return DRTOPK_EINVAL;
    BatchDesc d{};
    d.keys = kp;
    d.n = p.n;
    d.k = p.k;
    d.dtype = (uint32_t)dt_code(p.dt);
    d.alpha = (uint16_t)p.alpha;
    d.beta = (uint16_t)p.beta;
    d.out_vals = kth_only ? nullptr : static_cast<uint32_t*>(out_vals);
    d.out_idx = kth_only ? nullptr : out_idx;
    d.out_kth = static_cast<uint32_t*>(out_kth);
    hipLaunchKernelGGL(k_one, dim3(1), dim3(kBT), 0, s, d, p.rec);
    return hipGetLastError() == hipSuccess ? (int)DRTOPK_OK : (int)DRTOPK_EDEVICE;
  }
  with_codec(dt_code(p.dt), [&](auto c) {
    run_codec<decltype(c)::value>(p, kp, ws, static_cast<uint32_t*>(out_vals), out_idx,
                                  static_cast<uint32_t*>(out_kth), kth_only, filter_only, s);
  });
  const hipError_t le = tl_launch_err;
  tl_launch_err = hipSuccess;
  if (hipGetLastError() != hipSuccess || le != hipSuccess) return DRTOPK_EDEVICE;
  return DRTOPK_OK;
}

// Runs the whole path; `after` runs under the workspace lock after the
// enqueue, with the plan, the workspace pointer and the stream.  pos_in_ws:
// with out_idx NULL the output positions go to a workspace segment
// (Plan::off_pos) that `after` may read on the stream.
template <typename F>
int run_common(const void* keys, uint64_t n, uint32_t k, int dtype, void* out_vals, uint32_t* out_idx,
               void* out_kth, bool kth_only, const drtopk_options_t* opt, void* stream, F&& after,
               bool filter_only = false, bool pos_in_ws = false) {
  int st = check_args(keys, n, k, dtype);
  if (st) return st;
  Plan p;
  const bool ws_pos = pos_in_ws && !out_idx && !kth_only;
  st = make_plan(keys, n, k, dtype, opt, &p, ws_pos);
  if (st) return st;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DRTOPK_EDEVICE;
  Workspace* ws = workspace_entry(dev, stream);
  if (!ws) return DRTOPK_ENOMEM;
  std::lock_guard<std::mutex> g(ws->mu);
  st = ensure_record(ws);
  if (st) return st;
  st = ensure_bytes(ws, p.total);
  if (st) return st;
  p.rec = ws->rec;
  if (ws_pos) out_idx = at<uint32_t>(ws->ptr, p.off_pos);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  st = enqueue_plan(p, keys, ws->ptr, out_vals, out_idx, out_kth, kth_only, filter_only, s);
  if (st) return st;
  return after(p, ws->ptr, s);
}

// 64-bit keys: plan, workspace and the whole path; `after(const WPlan&, void*
// ws, hipStream_t)` runs under the workspace lock after the enqueue.
template <typename F>
int run_wide(const void* keys, uint64_t n, uint32_t k, int dtype, void* out_vals, uint32_t* out_idx, void* out_kth,
             bool kth_only, const drtopk_options_t* opt, void* stream, F&& after, bool pos_in_ws = false) {
  int st = check_args(keys, n, k, dtype);
  if (st) return st;
  WPlan p;
  const bool ws_pos = pos_in_ws && !out_idx && !kth_only;
  st = wide_plan(n, k, dtype, (reinterpret_cast<uintptr_t>(keys) & 15u) == 0, opt, &p, ws_pos);
  if (st) return st;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DRTOPK_EDEVICE;
  Workspace* ws = workspace_entry(dev, stream);
  if (!ws) return DRTOPK_ENOMEM;
  std::lock_guard<std::mutex> g(ws->mu);
  st = ensure_record(ws);
  if (st) return st;
  st = ensure_bytes(ws, p.total);
  if (st) return st;
  if (ws_pos) out_idx = at<uint32_t>(ws->ptr, p.off_pos);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  st = wide_enqueue(p, keys, ws->ptr, ws->rec, out_vals, out_idx, out_kth, kth_only, s);
  if (st) return st;
  return after(p, ws->ptr, s);
}

int fill_stats_wide(const WPlan& p, void* ws, hipStream_t s, drtopk_stats_t* stats) {
  if (!stats) return DRTOPK_OK;
  if (hipStreamSynchronize(s) != hipSuccess) return DRTOPK_EDEVICE;
  uint64_t scanned = 0, cand = 0, tkey = 0;
  uint32_t err = 0, tidx = 0;
  if (wide_counters(p, ws, &scanned, &cand, &err, &tkey, &tidx)) return DRTOPK_EDEVICE;
  std::memset(stats, 0, sizeof(*stats));
  stats->mode = p.mode;
  stats->alpha = p.alpha;
  stats->beta = 1;
  stats->subranges = p.S;
  stats->delegates = p.S;
  stats->scanned = scanned;
  stats->candidates = cand;
  stats->t_key_bits = (uint32_t)(tkey >> 32);
  stats->t_idx = tidx;
  stats->err_flags = err;
  return err ? DRTOPK_EDEVICE : DRTOPK_OK;
}

// Subrange exponent of a problem taken by the batched workgroup kernel; 0 =
// sorted outright (n <= kBSmallN) or radix select without delegates.
// *beta (if given): delegates per subrange, 1 unless a table entry asks for 2.
int batched_alpha(uint64_t n, uint32_t k, int* beta) {
  if (beta) *beta = 1;
  if (n <= kBSmallN) return 0;
  int a = -1, b = 0;
  if (tune_lookup(DRTOPK_FORM_BATCHED, n, k, &a, &b) && a == 0) return 0;  // measured: radix select
  const uint64_t bt = b == 2 ? 2 : 1;
  auto entries = [n, bt](int a) { return ((n + (1ull << a) - 1) >> a) * bt; };
  int r = 0;
  if (n > kBSplitMinN) {
    // split across workgroups: the delegate vector lives in global memory, so
    // it may hold up to kBMaxSG entries and Rule 4's shorter subranges apply
    // (at least 16 keys; tiles shrink so a tile's delegates fit its
    // workgroup's LDS); fewer subranges re-read at the same k
    if (a < 0) a = rule_alpha(n, k);
    if (a < 4) a = 4;
    if (a > 24) a = 24;
    while (a < 24 && entries(a) > kBMaxSG) ++a;
    while (entries(a) < 2ull * k && a > 4 && entries(a - 1) <= kBMaxSG) --a;
    r = entries(a) > k ? a : 0;
  } else {
    if (a < 0) {
      a = rule_alpha(n, k);
      if (a < 8) a = 8;  // a wave reads 256 keys per step: shorter subranges idle lanes
    }
    if (a > 24) a = 24;
    if (a < 2) a = 2;
    while (a < 24 && entries(a) > kBMaxS) ++a;  // delegate vector fits the LDS
    // at least 2k delegates where the LDS allows: with t the k-th of S subrange
    // maxima, about -S ln(1 - k/S) <= 0.7 S elements survive, within capacity
    while (entries(a) < 2ull * k && a > 2 && entries(a - 1) <= kBMaxS) --a;
    r = entries(a) > k && entries(a) <= kBMaxS ? a : 0;
  }
  if (beta && r) *beta = (int)bt;
  return r;
}

bool batched_eligible(uint64_t n, uint32_t k) { return n <= kBMaxN && k <= kBMaxK; }
bool batched_eligible(const drtopk_problem_t& q) {
  return batched_eligible(q.n, q.k) && !wide_dtype((int)q.dtype);
}

// Enqueues one k_batched launch over `items` (already validated).
BatchDesc make_desc(const drtopk_problem_t& q) {
  BatchDesc d{};
  d.keys = static_cast<const uint32_t*>(q.keys);
  d.n = q.n;
  d.k = q.k;
  d.dtype = (uint32_t)dt_code((int)q.dtype);
  int beta = 1;
  d.alpha = (uint16_t)batched_alpha(q.n, q.k, &beta);
  d.beta = (uint16_t)beta;
  d.out_vals = static_cast<uint32_t*>(q.out_vals);
  d.out_idx = q.out_idx;
  d.out_kth = static_cast<uint32_t*>(q.out_kth);
  return d;
}

// Tiles of a problem's delegate vector (one workgroup each): problems of
// more than kBSplitMinN keys on the delegate route are split so several
// workgroups stream them (their subranges hold at least 16 keys); one whose
// delegate vector exceeds the LDS (4096 entries) always spans two tiles or
// more, since a tile holds at most 4096 delegates.
uint32_t batched_tiles(const BatchDesc& d) {
  if (d.n <= kBSplitMinN || d.n <= kBSmallN || d.alpha < 4) return 1;
  const uint32_t tlog = tile_log(d.alpha, d.beta);
  return (uint32_t)((d.n + (1ull << tlog) - 1) >> tlog);
}

size_t align64(size_t x) { return (x + 63) & ~(size_t)63; }

// Device layout of a staged launch: claim counter | descriptors | per-problem
// arrival counters | work items | delegate vectors of split problems (device
// only).  Everything before the delegate vectors is copied from the pinned
// buffer, counters zeroed.
int launch_batched(const std::vector<const drtopk_problem_t*>& items, hipStream_t s, Workspace* ws) {
  std::vector<BatchDesc> descs(items.size());
  bool split = false;
  uint64_t dg_entries = 0;
  size_t nwork = 0;
  for (size_t i = 0; i < items.size(); ++i) {
    descs[i] = make_desc(*items[i]);
    descs[i].tiles = batched_tiles(descs[i]);
    if (descs[i].tiles > 1) {
      split = true;
      descs[i].doff = dg_entries;
      dg_entries += ((descs[i].n + (1ull << descs[i].alpha) - 1) >> descs[i].alpha) * descs[i].beta;
    }
    nwork += descs[i].tiles;
  }
  if (items.size() <= kBInline && !split) {  // descriptors as kernel arguments
    BatchInline b{};
    for (size_t i = 0; i < items.size(); ++i) b.d[i] = descs[i];
    hipLaunchKernelGGL(k_batched_inline, dim3((unsigned)items.size()), dim3(kBT), 0, s, b, ws->rec);
    return hipGetLastError() == hipSuccess ? (int)DRTOPK_OK : (int)DRTOPK_EDEVICE;
  }
  const size_t off_desc = 64;
  const size_t off_arrive = align64(off_desc + items.size() * sizeof(BatchDesc));
  const size_t off_items = align64(off_arrive + items.size() * 4);
  const size_t need = align64(off_items + nwork * 4);
  const size_t off_dg = (need + 255) & ~(size_t)255;
  const size_t dev_need = off_dg + (size_t)dg_entries * 8;
  int st = ensure_batch_bytes(ws, need, dev_need);
  if (st) return st;
  char* h = static_cast<char*>(ws->bhost);
  std::memset(h, 0, off_desc);  // claim counter
  std::memcpy(h + off_desc, descs.data(), descs.size() * sizeof(BatchDesc));
  std::memset(h + off_arrive, 0, off_items - off_arrive);
  uint32_t* work = reinterpret_cast<uint32_t*>(h + off_items);
  size_t w = 0;
  for (size_t i = 0; i < descs.size(); ++i)  // longest first; a split problem's tiles adjacent
    for (uint32_t t = 0; t < descs[i].tiles; ++t) work[w++] = ((uint32_t)i << 8) | t;
  if (hipMemcpyAsync(ws->bdev, ws->bhost, need, hipMemcpyHostToDevice, s) != hipSuccess) return DRTOPK_EDEVICE;
  if (hipEventRecord(ws->bev, s) != hipSuccess) return DRTOPK_EDEVICE;
  ws->bev_pending = true;
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const size_t slots = 2 * (size_t)cus;  // two workgroups fit a CU's LDS and registers
  const unsigned grid = (unsigned)(nwork < slots ? nwork : slots);
  char* dv = static_cast<char*>(ws->bdev);
  hipLaunchKernelGGL(k_batched, dim3(grid), dim3(kBT), 0, s, reinterpret_cast<const BatchDesc*>(dv + off_desc),
                     reinterpret_cast<const uint32_t*>(dv + off_items), (uint32_t)nwork,
                     reinterpret_cast<uint32_t*>(dv), reinterpret_cast<uint32_t*>(dv + off_arrive),
                     reinterpret_cast<uint64_t*>(dv + off_dg), ws->rec);
  if (hipGetLastError() != hipSuccess) return DRTOPK_EDEVICE;
  return DRTOPK_OK;
}

// Read-bandwidth probe: the delegate pass's launch geometry (one 256-thread
// workgroup per chunk, each wave a contiguous quarter, eight 16-byte
// non-temporal loads in flight per lane) with only a maximum per lane, so it
// measures what that access pattern can reach on this device.
__global__ __launch_bounds__(256) void k_read_probe(const uint32_t* __restrict__ keys, uint64_t n, uint64_t chunk,
                                                     uint32_t* out) {
  const uint32_t wave = threadIdx.x >> 6, lane = lane_id();
  const uint64_t wlen = chunk >> 2;
  const uint64_t wlo = (uint64_t)blockIdx.x * chunk + wave * wlen;
  uint32_t m = 0;
  if (wlo + wlen <= n) {
    for (uint64_t j = 0; j < wlen; j += 256 * kUnroll) {
      u32x4 v[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u)
        v[u] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(keys + wlo + j + u * 256 + lane * 4));
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) m = max(m, max(max(v[u].x, v[u].y), max(v[u].z, v[u].w)));
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o));
  if (lane == 0) atomicMax(out, m);
}

// Streaming top-k (host input): candidates = running list (r entries) then
// the chunk's list (c entries, positions + off), in that order.
__global__ void k_stream_concat(const uint32_t* rv, const uint32_t* ri, uint32_t r, const uint32_t* cv,
                                const uint32_t* ci, uint32_t c, uint64_t off, uint32_t* kv, uint32_t* ki) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < r + c; i += gridDim.x * blockDim.x) {
    if (i < r) {
      kv[i] = rv[i];
      ki[i] = ri[i];
    } else {
      kv[i] = cv[i - r];
      ki[i] = (uint32_t)(ci[i - r] + off);
    }
  }
}
// Payload of each output slot: out[r] = payload[idx[r]] (T = 4- or 8-byte element).
template <typename T>
__global__ void k_gather_payload(const T* payload, const uint32_t* idx, uint32_t k, T* out) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) out[i] = payload[idx[i]];
}

// New running list: the selected candidates' values and whole-input positions.
__global__ void k_stream_gather(const uint32_t* sv, const uint32_t* si, uint32_t m, const uint32_t* ki,
                                uint32_t* rv, uint32_t* ri) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
    rv[i] = sv[i];
    ri[i] = ki[si[i]];
  }
}

__global__ void k_zero_word(uint32_t* p) {
  if (threadIdx.x == 0) *p = 0;
}
__global__ void k_zero_words(uint32_t* p, uint32_t n) {
  if (threadIdx.x < n) p[threadIdx.x] = 0;
}

// ---------------------------------------------------------------------------
// Fixed workspace of topk_select_noalloc, for callers that cannot allocate
// device memory: one copy of `scratch` per device, held until the process
// ends.  Its first kScratchRec bytes are the check record of the no-alloc
// calls (kErrWords words, set by failing kernel checks, cleared by
// drtopk_check); the rest is the workspace of one call.  In host code the
// array's name is not a device address: the address comes from
// hipGetSymbolAddress, once per device with that device current.
constexpr size_t kScratchBytes = size_t(128) << 20;
constexpr size_t kScratchRec = 256;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::atomic<void*> g_scratch_ptr[kMaxDevices];

// Device address of the current device's scratch (null on failure).
void* scratch_base(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  void* p = g_scratch_ptr[dev].load(std::memory_order_acquire);
  if (p) return p;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  p = g_scratch_ptr[dev].load(std::memory_order_relaxed);
  if (p) return p;
  void* q = nullptr;
  if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || !q) {
    (void)hipGetLastError();
    return nullptr;
  }
  // the record starts clear: the array is zero-initialised at load, and a
  // kernel clears it once more so that nothing depends on that
  hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, nullptr, static_cast<uint32_t*>(q), (uint32_t)kErrWords);
  if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) return nullptr;
  g_scratch_ptr[dev].store(q, std::memory_order_release);
  return q;
}

int fill_stats(const Plan& p, void* ws, hipStream_t s, drtopk_stats_t* stats) {
  if (!stats) return DRTOPK_OK;
  if (hipStreamSynchronize(s) != hipSuccess) return DRTOPK_EDEVICE;
  if (p.mode == 3) {  // no control block: the workgroup keeps its state in LDS
    std::memset(stats, 0, sizeof(*stats));
    stats->mode = 3;
    stats->alpha = p.alpha;
    stats->beta = p.alpha ? p.beta : 1;
    stats->subranges = p.alpha ? (p.n + (1ull << p.alpha) - 1) >> p.alpha : 0;
    stats->delegates = stats->subranges * (uint64_t)stats->beta;
    return DRTOPK_OK;
  }
  Ctl h;
  if (hipMemcpy(&h, at<Ctl>(ws, p.off_ctl), sizeof(Ctl), hipMemcpyDeviceToHost) != hipSuccess) return DRTOPK_EDEVICE;
  std::memset(stats, 0, sizeof(*stats));
  stats->mode = p.mode;
  stats->alpha = p.alpha;
  stats->beta = p.beta;
  stats->subranges = p.S;
  stats->delegates = p.nd;
  stats->scanned = h.nq;
  stats->candidates = p.mode == 1 ? h.nc : p.n;
  stats->t_key_bits = p.mode == 1 ? host_dec(dt_code(p.dt), (uint32_t)(h.selD.prefix >> 32)) : 0;
  stats->t_idx = p.mode == 1 ? ~(uint32_t)h.selD.prefix : 0;
  const uint64_t t0 = h.tstamp[kPhases + 1];
  for (int i = 0; i < kPhases && i < 20; ++i)
    stats->step_ns[i] = (t0 && h.tstamp[i] >= t0) ? (uint32_t)((h.tstamp[i] - t0) * 10) : 0;
  stats->err_flags = h.err;
  if (h.err) return DRTOPK_EDEVICE;
  return DRTOPK_OK;
}

}  // namespace
}  // namespace drtopk

using namespace drtopk;

extern "C" {

int topk_select_ex(const void* keys, uint64_t n, uint32_t k, int dtype, void* out_vals, uint32_t* out_idx,
                   const drtopk_options_t* opt, drtopk_stats_t* stats, void* stream) {
  if (!out_vals) return DRTOPK_EINVAL;
  try {
    if (wide_dtype(dtype))
      return run_wide(keys, n, k, dtype, out_vals, out_idx, nullptr, false, opt, stream,
                      [&](const WPlan& p, void* ws, hipStream_t s) { return fill_stats_wide(p, ws, s, stats); });
    return run_common(keys, n, k, dtype, out_vals, out_idx, nullptr, false, opt, stream,
                      [&](const Plan& p, void* ws, hipStream_t s) { return fill_stats(p, ws, s, stats); });
  } catch (...) {
    return DRTOPK_EDEVICE;
  }
}

int topk_select(const void* keys, uint64_t n, uint32_t k, int dtype, void* out_vals, uint32_t* out_idx,
                void* stream) {
  return topk_select_ex(keys, n, k, dtype, out_vals, out_idx, nullptr, nullptr, stream);
}

int topk_select_noalloc(const void* keys, uint64_t n, uint32_t k, int dtype, void* out_vals, uint32_t* out_idx,
                        void* stream) {
  if (!out_vals) return DRTOPK_EINVAL;
  int st = check_args(keys, n, k, dtype);
  if (st) return st;
  try {
    const bool wide = wide_dtype(dtype);
    Plan p;
    WPlan wp;
    st = wide ? wide_plan(n, k, dtype, (reinterpret_cast<uintptr_t>(keys) & 15u) == 0, nullptr, &wp)
              : make_plan(keys, n, k, dtype, nullptr, &p);
    if (st) return st;
    if ((wide ? wp.total : p.total) > kScratchBytes - kScratchRec) return DRTOPK_ESCRATCH;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return DRTOPK_EDEVICE;
    void* base = scratch_base(dev);
    if (!base) return DRTOPK_EDEVICE;
    void* ws = static_cast<char*>(base) + kScratchRec;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (wide) return wide_enqueue(wp, keys, ws, static_cast<uint32_t*>(base), out_vals, out_idx, nullptr, false, s);
    p.rec = static_cast<uint32_t*>(base);
    p.marks = false;  // no timing events
    return enqueue_plan(p, keys, ws, out_vals, out_idx, nullptr, false, false, s);
  } catch (...) {
    return DRTOPK_EDEVICE;
  }
}

int kth_select(const void* keys, uint64_t n, uint32_t k, int dtype, void* out_kth, void* stream) {
  if (!out_kth) return DRTOPK_EINVAL;
  try {
    if (wide_dtype(dtype))
      return run_wide(keys, n, k, dtype, nullptr, nullptr, out_kth, true, nullptr, stream,
                      [](const WPlan&, void*, hipStream_t) { return (int)DRTOPK_OK; });
    return run_common(keys, n, k, dtype, nullptr, nullptr, out_kth, true, nullptr, stream,
                      [](const Plan&, void*, hipStream_t) { return (int)DRTOPK_OK; });
  } catch (...) {
    return DRTOPK_EDEVICE;
  }
}

int topk_select_batched(const drtopk_problem_t* problems, uint32_t count, void* stream) {
  if (count && !problems) return DRTOPK_EINVAL;
  if (count >= (1u << 24)) return DRTOPK_EINVAL;  // work items carry the problem index in 24 bits
  for (uint32_t i = 0; i < count; ++i) {
    const drtopk_problem_t& q = problems[i];
    if (!q.out_vals && !q.out_kth) return DRTOPK_EINVAL;
    int st = check_args(q.keys, q.n, q.k, (int)q.dtype);
    if (st) return st;
  }
  if (count == 0) return DRTOPK_OK;
  try {
    // problems a workgroup can own go to one persistent launch, largest first
    std::vector<const drtopk_problem_t*> small, large;
    for (uint32_t i = 0; i < count; ++i)
      (batched_eligible(problems[i]) ? small : large).push_back(&problems[i]);
    std::stable_sort(small.begin(), small.end(),
                     [](const drtopk_problem_t* a, const drtopk_problem_t* b) { return a->n > b->n; });
    if (!small.empty()) {
      int dev = 0;
      if (hipGetDevice(&dev) != hipSuccess) return DRTOPK_EDEVICE;
      Workspace* ws = workspace_entry(dev, stream);
      if (!ws) return DRTOPK_ENOMEM;
      std::lock_guard<std::mutex> lock(ws->mu);
      int st = ensure_record(ws);
      if (st) return st;
      st = launch_batched(small, reinterpret_cast<hipStream_t>(stream), ws);
      if (st) return st;
    }
    for (const drtopk_problem_t* q : large) {
      const int st =
          wide_dtype((int)q->dtype)
              ? run_wide(q->keys, q->n, q->k, (int)q->dtype, q->out_vals, q->out_idx, q->out_kth, !q->out_vals,
                         nullptr, stream, [](const WPlan&, void*, hipStream_t) { return (int)DRTOPK_OK; })
              : run_common(q->keys, q->n, q->k, (int)q->dtype, q->out_vals, q->out_idx, q->out_kth, !q->out_vals,
                           nullptr, stream, [](const Plan&, void*, hipStream_t) { return (int)DRTOPK_OK; });
      if (st) return st;
    }
  } catch (...) {
    return DRTOPK_EDEVICE;
  }
  return DRTOPK_OK;
}

int drtopk_footprint(uint64_t n, uint32_t k, int dtype, uint64_t* bytes) {
  if (!bytes) return DRTOPK_EINVAL;
  alignas(16) static const uint32_t dummy[4] = {0, 0, 0, 0};
  int st = check_args(dummy, n, k, dtype);
  if (st) return st;
  if (wide_dtype(dtype)) {
    WPlan wp;
    st = wide_plan(n, k, dtype, true, nullptr, &wp);
    if (st) return st;
    *bytes = 8 * n + 12ull * k + 8 + wp.total;
    return DRTOPK_OK;
  }
  // a batched problem: its descriptor, work items and arrival counter, plus
  // the global delegate vector when it is split across workgroups
  uint64_t ws = sizeof(BatchDesc) + 16;
  if (!batched_eligible(n, k)) {
    Plan p;
    st = make_plan(dummy, n, k, dtype, nullptr, &p);
    if (st) return st;
    ws = p.total;
  } else {
    BatchDesc d{};
    d.n = n;
    d.k = k;
    int beta = 1;
    d.alpha = (uint16_t)batched_alpha(n, k, &beta);
    d.beta = (uint16_t)beta;
    d.tiles = batched_tiles(d);
    if (d.tiles > 1) ws += 4ull * d.tiles + 8ull * beta * ((n + (1ull << d.alpha) - 1) >> d.alpha);
  }
  *bytes = 4 * n + 8ull * k + 4 + ws;
  return DRTOPK_OK;
}

int drtopk_tune_set(const drtopk_tune_t* entries, uint32_t count) {
  if (count && !entries) return DRTOPK_EINVAL;
  std::vector<drtopk_tune_t> t;
  try {
    for (uint32_t i = 0; i < count; ++i) {
      const drtopk_tune_t& e = entries[i];
      if (e.form != DRTOPK_FORM_SINGLE && e.form != DRTOPK_FORM_BATCHED) return DRTOPK_EINVAL;
      if (e.lg_n < 0 || e.lg_n > 31 || e.lg_k < 0 || e.lg_k > 31) return DRTOPK_EINVAL;
      if (e.alpha < 0 || e.alpha > 24 || !valid_beta(e.beta)) return DRTOPK_EINVAL;
      t.push_back(e);
    }
  } catch (...) {
    return DRTOPK_ENOMEM;
  }
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune.swap(t);
  return DRTOPK_OK;
}

int drtopk_tune_get(drtopk_tune_t* out, uint32_t cap, uint32_t* count) {
  if (!count || (cap && !out)) return DRTOPK_EINVAL;
  std::lock_guard<std::mutex> g(g_tune_mu);
  *count = (uint32_t)g_tune.size();
  for (uint32_t i = 0; i < cap && i < g_tune.size(); ++i) out[i] = g_tune[i];
  return DRTOPK_OK;
}

int drtopk_batched_alpha(uint64_t n, uint32_t k, int32_t* route, int32_t* alpha, int32_t* beta) {
  if (!route || !alpha || n == 0 || n >= (1ull << 32) || k == 0 || k > n) return DRTOPK_EINVAL;
  int b = 1;
  if (!batched_eligible(n, k)) {
    *route = 0;
    *alpha = 0;
  } else {
    *alpha = batched_alpha(n, k, &b);
    *route = n <= kBSmallN ? 1 : *alpha ? 2 : 3;
  }
  if (beta) *beta = b;
  return DRTOPK_OK;
}

int drtopk_delegates(const void* keys, uint64_t n, int dtype, int alpha, int beta, void* out_dkeys,
                     uint32_t* out_didx, void* stream) {
  if (!out_dkeys || !out_didx) return DRTOPK_EINVAL;
  int st = check_args(keys, n, 1, dtype);
  if (st) return st;
  if (wide_dtype(dtype)) return DRTOPK_EUNSUPPORTED;
  if (alpha < 0 || alpha > 24 || !valid_beta(beta)) return DRTOPK_EINVAL;
  drtopk_options_t o{alpha, beta, 1, 0};
  Plan p;
  st = make_plan(keys, n, 1, dtype, &o, &p);
  if (st) return st;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DRTOPK_EDEVICE;
  Workspace* ws = workspace_entry(dev, stream);
  if (!ws) return DRTOPK_ENOMEM;
  std::lock_guard<std::mutex> lock(ws->mu);
  st = ensure_record(ws);
  if (st) return st;
  st = ensure_bytes(ws, p.total);
  if (st) return st;
  p.rec = ws->rec;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Ctl* ctl = at<Ctl>(ws->ptr, p.off_ctl);
  const uint32_t* kp = static_cast<const uint32_t*>(keys);
  uint32_t* dk = static_cast<uint32_t*>(out_dkeys);
  with_codec(dt_code(dtype),
             [&](auto c) { delegates_codec<decltype(c)::value>(p, kp, dk, out_didx, ctl, s); });
  if (hipGetLastError() != hipSuccess) return DRTOPK_EDEVICE;
  return DRTOPK_OK;
}

int drtopk_candidates(const void* keys, uint64_t n, uint32_t k, int dtype, int alpha, int beta, int variant,
                      uint32_t* out_pos, uint64_t cap, uint64_t* count, uint32_t* t_out, void* stream) {
  if (!out_pos || !count) return DRTOPK_EINVAL;
  if (alpha < 0 || alpha > 24 || !valid_beta(beta)) return DRTOPK_EINVAL;
  if (wide_dtype(dtype)) return dtype_ok(dtype) ? DRTOPK_EUNSUPPORTED : DRTOPK_EINVAL;
  drtopk_options_t o{alpha, beta, 1, variant};
  try {
    return run_common(keys, n, k, dtype, nullptr, nullptr, nullptr, true, &o, stream,
                      [&](const Plan& p, void* ws, hipStream_t s) {
                        if (hipStreamSynchronize(s) != hipSuccess) return (int)DRTOPK_EDEVICE;
                        uint32_t nc = 0;
                        if (hipMemcpy(&nc, &at<Ctl>(ws, p.off_ctl)->nc, 4, hipMemcpyDeviceToHost) != hipSuccess)
                          return (int)DRTOPK_EDEVICE;
                        if (t_out) {
                          uint64_t t = 0;
                          if (hipMemcpy(&t, &at<Ctl>(ws, p.off_ctl)->selD.prefix, 8, hipMemcpyDeviceToHost) !=
                              hipSuccess)
                            return (int)DRTOPK_EDEVICE;
                          t_out[0] = host_dec(dt_code(p.dt), (uint32_t)(t >> 32));
                          t_out[1] = ~(uint32_t)t;
                        }
                        *count = nc;
                        if (nc > cap) return (int)DRTOPK_EINVAL;
                        if (nc && hipMemcpy(out_pos, at<uint32_t>(ws, p.off_cidx), (size_t)nc * 4,
                                            hipMemcpyDeviceToDevice) != hipSuccess)
                          return (int)DRTOPK_EDEVICE;
                        return (int)DRTOPK_OK;
                      },
                      true);
  } catch (...) {
    return DRTOPK_EDEVICE;
  }
}

int drtopk_plan(uint64_t n, uint32_t k, int dtype, drtopk_options_t* out) {
  if (!out) return DRTOPK_EINVAL;
  static const uint32_t dummy[4] = {0, 0, 0, 0};
  int st = check_args(dummy, n, k, dtype);
  if (st) return st;
  if (wide_dtype(dtype)) {
    WPlan wp;
    st = wide_plan(n, k, dtype, true, nullptr, &wp);
    if (st) return st;
    out->alpha = wp.alpha;
    out->beta = 1;
    out->mode = wp.mode;
    out->variant = 0;
    return DRTOPK_OK;
  }
  Plan p;
  st = make_plan(dummy, n, k, dtype, nullptr, &p);
  if (st) return st;
  out->alpha = p.alpha;
  out->beta = p.beta;
  out->mode = p.mode;
  out->variant = p.variant;
  return DRTOPK_OK;
}

int drtopk_release_workspace(void) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DRTOPK_EDEVICE;
  if (hipDeviceSynchronize() != hipSuccess) return DRTOPK_EDEVICE;
  std::lock_guard<std::mutex> g(g_mu);
  for (auto it = g_ws.begin(); it != g_ws.end();) {
    if (it->first.first == dev) {
      std::lock_guard<std::mutex> g2(it->second->mu);
      Workspace* w = it->second.get();
      if (w->ptr) (void)hipFree(w->ptr);
      w->ptr = nullptr;
      w->bytes = 0;
      if (w->bdev) (void)hipFree(w->bdev);
      w->bdev = nullptr;
      w->bdev_bytes = 0;
      if (w->bhost) (void)hipHostFree(w->bhost);
      w->bhost = nullptr;
      w->bhost_bytes = 0;
      if (w->bev) (void)hipEventDestroy(w->bev);
      w->bev = nullptr;
      w->bev_pending = false;
      ++it;
    } else {
      ++it;
    }
  }
  return DRTOPK_OK;
}

int drtopk_timing_enable(int on) {
  std::lock_guard<std::mutex> g(g_timing.mu);
  g_timing.on = on != 0;
  return DRTOPK_OK;
}

int drtopk_timing_read(double* delegate_ms, double* tail_ms, uint64_t* calls) {
  std::vector<Timing::Rec> recs;
  {
    std::lock_guard<std::mutex> g(g_timing.mu);
    recs.swap(g_timing.pending);
  }
  double d = 0, t = 0;
  int st = DRTOPK_OK;
  for (auto& r : recs) {
    float x = 0, y = 0;
    if (hipEventSynchronize(r.c) != hipSuccess || hipEventElapsedTime(&x, r.a, r.b) != hipSuccess ||
        hipEventElapsedTime(&y, r.b, r.c) != hipSuccess)
      st = DRTOPK_EDEVICE;
    d += x;
    t += y;
  }
  {
    std::lock_guard<std::mutex> g(g_timing.mu);
    for (auto& r : recs) {
      g_timing.pool.push_back(r.a);
      g_timing.pool.push_back(r.b);
      g_timing.pool.push_back(r.c);
    }
  }
  if (delegate_ms) *delegate_ms = d;
  if (tail_ms) *tail_ms = t;
  if (calls) *calls = recs.size();
  return st;
}

int drtopk_read_probe(const void* keys, uint64_t n, uint32_t* out_max, void* stream) {
  if (!keys || !out_max || n < (1u << 20) || n >= (1ull << 32)) return DRTOPK_EINVAL;
  if ((reinterpret_cast<uintptr_t>(keys) & 15u) != 0) return DRTOPK_EINVAL;
  const uint64_t chunk = 1ull << 20;  // the beta = 1 delegate pass's chunk at n = 2^30
  const unsigned g = (unsigned)(n / chunk);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_zero_word, dim3(1), dim3(64), 0, s, out_max);
  hipLaunchKernelGGL(k_read_probe, dim3(g), dim3(256), 0, s, static_cast<const uint32_t*>(keys), n, chunk, out_max);
  return hipGetLastError() == hipSuccess ? (int)DRTOPK_OK : (int)DRTOPK_EDEVICE;
}

int topk_select_payload(const void* keys, uint64_t n, uint32_t k, int dtype, const void* payload,
                        int payload_bytes, void* out_vals, uint32_t* out_idx, void* out_payload, void* stream) {
  if (!payload || !out_payload || (payload_bytes != 4 && payload_bytes != 8)) return DRTOPK_EINVAL;
  int st = check_args(keys, n, k, dtype);
  if (st) return st;
  if (!out_vals) return DRTOPK_EINVAL;
  try {
    // the gather is enqueued under the workspace lock, so with out_idx NULL it
    // reads the positions from the workspace before any later call on the
    // stream can overwrite them
    auto gather = [&](size_t off_pos, void* ws, hipStream_t s) {
      const uint32_t* idx = out_idx ? out_idx : at<uint32_t>(ws, off_pos);
      const unsigned g = grid_for(k, 256, 1024);
      if (payload_bytes == 4)
        hipLaunchKernelGGL(k_gather_payload<uint32_t>, dim3(g), dim3(256), 0, s,
                           static_cast<const uint32_t*>(payload), idx, k, static_cast<uint32_t*>(out_payload));
      else
        hipLaunchKernelGGL(k_gather_payload<uint64_t>, dim3(g), dim3(256), 0, s,
                           static_cast<const uint64_t*>(payload), idx, k, static_cast<uint64_t*>(out_payload));
      return hipGetLastError() == hipSuccess ? (int)DRTOPK_OK : (int)DRTOPK_EDEVICE;
    };
    if (wide_dtype(dtype))
      return run_wide(keys, n, k, dtype, out_vals, out_idx, nullptr, false, nullptr, stream,
                      [&](const WPlan& p, void* ws, hipStream_t s) { return gather(p.off_pos, ws, s); }, true);
    return run_common(keys, n, k, dtype, out_vals, out_idx, nullptr, false, nullptr, stream,
                      [&](const Plan& p, void* ws, hipStream_t s) { return gather(p.off_pos, ws, s); }, false, true);
  } catch (...) {
    return DRTOPK_EDEVICE;
  }
}

int topk_select_host(const void* host_keys, uint64_t n, uint32_t k, int dtype, uint64_t chunk, void* out_vals,
                     uint32_t* out_idx, void* stream) {
  if (!out_vals) return DRTOPK_EINVAL;
  int st = check_args(host_keys, n, k, dtype);
  if (st) return st;
  if (wide_dtype(dtype)) return DRTOPK_EUNSUPPORTED;
  if (chunk == 0) chunk = n < (1ull << 26) ? n : (1ull << 26);
  if (chunk > n) return DRTOPK_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const uint64_t nchunks = (n + chunk - 1) / chunk;
  // device buffers: two chunks, the chunk's top-k, the running list, 2k candidates and the selection
  const uint64_t kk = k;
  const size_t bytes = 2 * chunk * 4 + (2 * kk + 2 * kk + 4 * kk + 2 * kk) * 4;
  void* mem = nullptr;
  if (hipMalloc(&mem, bytes) != hipSuccess) return DRTOPK_ENOMEM;
  uint32_t* buf[2] = {static_cast<uint32_t*>(mem), static_cast<uint32_t*>(mem) + chunk};
  uint32_t* cv = buf[1] + chunk;  // chunk top-k values / positions
  uint32_t* ci = cv + kk;
  uint32_t* rv = ci + kk;  // running list
  uint32_t* ri = rv + kk;
  uint32_t* kv = ri + kk;  // candidates (2k)
  uint32_t* ki = kv + 2 * kk;
  uint32_t* sv = ki + 2 * kk;  // selection over the candidates
  uint32_t* si = sv + kk;
  hipStream_t cs = nullptr;
  hipEvent_t copied[2] = {nullptr, nullptr}, used[2] = {nullptr, nullptr};
  bool ok = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess;
  for (int b = 0; b < 2 && ok; ++b)
    ok = hipEventCreateWithFlags(&copied[b], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&used[b], hipEventDisableTiming) == hipSuccess;
  uint32_t r = 0;  // running list length
  const char* src = static_cast<const char*>(host_keys);
  for (uint64_t c = 0; c < nchunks && ok; ++c) {
    const int b = (int)(c & 1);
    const uint64_t off = c * chunk;
    const uint64_t len = n - off < chunk ? n - off : chunk;
    const uint32_t kc = (uint64_t)k < len ? k : (uint32_t)len;
    // the buffer's previous chunk must be done with before it is overwritten
    if (c >= 2) ok = hipStreamWaitEvent(cs, used[b], 0) == hipSuccess;
    ok = ok && hipMemcpyAsync(buf[b], src + off * 4, len * 4, hipMemcpyHostToDevice, cs) == hipSuccess;
    ok = ok && hipEventRecord(copied[b], cs) == hipSuccess;
    ok = ok && hipStreamWaitEvent(s, copied[b], 0) == hipSuccess;
    if (!ok) break;
    if (r == 0) {
      st = topk_select(buf[b], len, kc, dtype, rv, ri, stream);
      r = kc;
    } else {
      st = topk_select(buf[b], len, kc, dtype, cv, ci, stream);
      if (st == DRTOPK_OK) {
        hipLaunchKernelGGL(k_stream_concat, dim3(grid_for(r + kc, 256, 1024)), dim3(256), 0, s, rv, ri, r, cv, ci, kc,
                           off, kv, ki);
        const uint32_t m = r + kc < k ? r + kc : k;
        st = topk_select(kv, r + kc, m, dtype, sv, si, stream);
        if (st == DRTOPK_OK)
          hipLaunchKernelGGL(k_stream_gather, dim3(grid_for(m, 256, 1024)), dim3(256), 0, s, sv, si, m, ki, rv, ri);
        r = m;
      }
    }
    // positions of the first chunk need no offset: it starts at 0
    if (st != DRTOPK_OK) break;
    ok = hipEventRecord(used[b], s) == hipSuccess;
  }
  if (ok && st == DRTOPK_OK) {
    ok = hipMemcpyAsync(out_vals, rv, kk * 4, hipMemcpyDeviceToDevice, s) == hipSuccess;
    if (ok && out_idx) ok = hipMemcpyAsync(out_idx, ri, kk * 4, hipMemcpyDeviceToDevice, s) == hipSuccess;
  }
  // everything below uses the buffers: wait for both streams before freeing
  if (cs) (void)hipStreamSynchronize(cs);
  (void)hipStreamSynchronize(s);
  for (int b = 0; b < 2; ++b) {
    if (copied[b]) (void)hipEventDestroy(copied[b]);
    if (used[b]) (void)hipEventDestroy(used[b]);
  }
  if (cs) (void)hipStreamDestroy(cs);
  (void)hipFree(mem);
  if (st != DRTOPK_OK) return st;
  if (!ok || hipGetLastError() != hipSuccess) return DRTOPK_EDEVICE;
  // the stream has finished: a failed internal check of its calls is reported
  // here (and stays recorded for drtopk_check)
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DRTOPK_EDEVICE;
  if (Workspace* ws = find_workspace(dev, stream)) {
    std::lock_guard<std::mutex> g(ws->mu);
    if (ws->rec && read_record(ws->rec, false)) return DRTOPK_EDEVICE;
  }
  return DRTOPK_OK;
}

int drtopk_check(void* stream, uint32_t* flags) {
  if (flags) *flags = 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DRTOPK_EDEVICE;
  if (hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)) != hipSuccess) return DRTOPK_EDEVICE;
  uint32_t f = 0;
  if (Workspace* ws = find_workspace(dev, stream)) {
    std::lock_guard<std::mutex> g(ws->mu);
    if (ws->rec) f |= read_record(ws->rec, true);
  }
  // the no-alloc calls' record, in the device's scratch (if it was ever used)
  void* sb = (dev >= 0 && dev < kMaxDevices) ? g_scratch_ptr[dev].load(std::memory_order_acquire) : nullptr;
  if (sb) {
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    uint32_t w[kErrWords] = {};
    if (hipMemcpyAsync(w, sb, sizeof(w), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return DRTOPK_EDEVICE;
    const uint32_t g = read_record(w, false);
    if (g) {
      hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, s, static_cast<uint32_t*>(sb), (uint32_t)kErrWords);
      if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return DRTOPK_EDEVICE;
    }
    f |= g;
  }
  if (flags) *flags = f;
  return f ? DRTOPK_EDEVICE : DRTOPK_OK;
}

int drtopk_set_survivor_cap(uint64_t cap) {
  g_cap_override.store(cap, std::memory_order_relaxed);
  return DRTOPK_OK;
}

const char* drtopk_status_string(int status) {
  switch (status) {
    case DRTOPK_OK: return "ok";
    case DRTOPK_EINVAL: return "invalid argument";
    case DRTOPK_ENOMEM: return "out of device memory";
    case DRTOPK_EDEVICE: return "device error";
    case DRTOPK_EUNSUPPORTED: return "unsupported";
    case DRTOPK_ESCRATCH: return "workspace exceeds the no-allocation scratch buffer";
    default: return "unknown status";
  }
}

const char* drtopk_version(void) { return "drtopk 0.1 (gfx950)"; }

}  // extern "C"
