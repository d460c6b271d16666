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
#include "kernels.h"
#include "tail.h"
#include "batched.h"

namespace drtopk {
namespace {

constexpr double kAlphaConst = 3.0;  // Rule 4's const; the paper tuned it to 3

struct Plan {
  int mode = 0;  // 1 delegate method, 2 plain radix select on V, 3 one workgroup (batched kernel)
  int alpha = 0, beta = 1;
  int dt = 0;
  uint64_t n = 0;
  uint32_t k = 0;
  uint64_t S = 0, nd = 0, cap_c = 0, chunk = 0, M = 0;
  uint32_t kD = 0;   // rank sought among the delegates: min(k, |D|)
  uint32_t slack = 0;
  int variant = 0;   // 0: cooperative tail kernel, 1: one kernel per step
  bool all = false;  // fewer real delegates than k: no threshold, every subrange qualifies
  bool vec = false;
  size_t off_ctl = 0, off_dkey = 0, off_didx = 0, off_q = 0, off_ckey = 0, off_cidx = 0;
  size_t off_okey = 0, off_oidx = 0, off_A = 0, off_B = 0, off_skey = 0, off_sidx = 0, total = 0;
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

thread_local hipError_t tl_launch_err = hipSuccess;  // launches whose API reports errors directly

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

int batched_alpha(uint64_t n, uint32_t k);
bool batched_eligible(uint64_t n, uint32_t k);

// Problems up to this size (and k <= kBMaxK) finish faster in one workgroup
// than across the device: one launch, no workspace.
constexpr uint64_t kOneWgMaxN = 1ull << 16;

int make_plan(const void* keys, uint64_t n, uint32_t k, int dt, const drtopk_options_t* opt, Plan* P) {
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
  if (mode == 3) p.alpha = batched_alpha(n, k);
  p.mode = mode;
  p.variant = opt ? opt->variant : 0;
  if (p.variant < 0 || p.variant > 1) return DRTOPK_EINVAL;
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
};

std::mutex g_mu;
std::map<std::pair<int, void*>, std::unique_ptr<Workspace>> g_ws;

Workspace* workspace_entry(int dev, void* stream) {
  std::lock_guard<std::mutex> g(g_mu);
  auto& slot = g_ws[{dev, stream}];
  if (!slot) slot.reset(new (std::nothrow) Workspace());
  return slot.get();
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

template <typename T>
T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

unsigned grid_for(uint64_t items, uint64_t per_block, unsigned cap) {
  uint64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// ---------------------------------------------------------------------------
// optional phase timing (events on the call's own stream)
struct Timing {
  std::mutex mu;
  bool on = false;
  struct Rec { hipEvent_t a, b, c; };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  hipEvent_t take() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
} g_timing;

struct PhaseMarks {
  hipEvent_t a = nullptr, b = nullptr, c = nullptr;
  bool on = false;
  void begin(hipStream_t st) {
    std::lock_guard<std::mutex> g(g_timing.mu);
    if (!g_timing.on) return;
    a = g_timing.take(); b = g_timing.take(); c = g_timing.take();
    on = a && b && c;
    (void)st;
  }
  void start(hipStream_t st) { if (on) (void)hipEventRecord(a, st); }
  void mid(hipStream_t st) { if (on) (void)hipEventRecord(b, st); }
  void end(hipStream_t st) {
    if (!on) return;
    (void)hipEventRecord(c, st);
    std::lock_guard<std::mutex> g(g_timing.mu);
    g_timing.pending.push_back({a, b, c});
  }
};

// ---------------------------------------------------------------------------
// kernel sequence
template <int DT>
struct Runner {
  static void delegate(const Plan& p, const uint32_t* keys, uint32_t* dkey, uint32_t* didx, Ctl* ctl,
                       hipStream_t st, DirectOut out = DirectOut{nullptr, nullptr, nullptr, 0}) {
    if (p.alpha >= 2) {
      const unsigned g = (unsigned)((p.n + p.chunk - 1) / p.chunk);
#define DRTOPK_DEL(B, V) \
  hipLaunchKernelGGL((k_delegate<DT, B, V>), dim3(g), dim3(256), 0, st, keys, p.n, p.alpha, p.chunk, dkey, didx, ctl, p.kD, \
                     out)
      switch (p.beta * 2 + (p.vec ? 1 : 0)) {
        case 2: DRTOPK_DEL(1, false); break;
        case 3: DRTOPK_DEL(1, true); break;
        case 4: DRTOPK_DEL(2, false); break;
        case 5: DRTOPK_DEL(2, true); break;
        case 8: DRTOPK_DEL(4, false); break;
        case 9: DRTOPK_DEL(4, true); break;
        case 16: DRTOPK_DEL(8, false); break;
        default: DRTOPK_DEL(8, true); break;
      }
#undef DRTOPK_DEL
    } else {
      const unsigned g = grid_for(p.S, 256, 4096);
#define DRTOPK_DELT(B) \
  hipLaunchKernelGGL((k_delegate_thread<DT, B>), dim3(g), dim3(256), 0, st, keys, p.n, p.alpha, p.S, dkey, didx, ctl, \
                     p.kD, out)
      switch (p.beta) {
        case 1: DRTOPK_DELT(1); break;
        case 2: DRTOPK_DELT(2); break;
        case 4: DRTOPK_DELT(4); break;
        default: DRTOPK_DELT(8); break;
      }
#undef DRTOPK_DELT
    }
  }

  template <int B, bool V>
  static void launch_tail_t(TailArgs& ta, hipStream_t st) {
    static int blocks = 0;  // blocks that fit the device at once (phases need no co-residency)
    if (blocks == 0) {
      int dev = 0, cus = 0, per = 0;
      (void)hipGetDevice(&dev);
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(&k_tail<DT, B, V>),
                                                          kTailThreads, 0);
      if (per > 2) per = 2;
      if (per < 1) per = 1;
      blocks = cus * per;
    }
    hipLaunchKernelGGL((k_tail<DT, B, V>), dim3(blocks), dim3(kTailThreads), 0, st, ta);
  }

  static void launch_tail(const Plan& p, TailArgs& ta, hipStream_t st) {
    switch (p.beta * 2 + (p.vec ? 1 : 0)) {
      case 2: launch_tail_t<1, false>(ta, st); break;
      case 3: launch_tail_t<1, true>(ta, st); break;
      case 4: launch_tail_t<2, false>(ta, st); break;
      case 5: launch_tail_t<2, true>(ta, st); break;
      case 8: launch_tail_t<4, false>(ta, st); break;
      case 9: launch_tail_t<4, true>(ta, st); break;
      case 16: launch_tail_t<8, false>(ta, st); break;
      default: launch_tail_t<8, true>(ta, st); break;
    }
  }

  static void qualify(const Plan& p, uint32_t* dkey, uint32_t* didx, Ctl* ctl, uint32_t* Q, uint32_t* ckey,
                      uint32_t* cidx, hipStream_t st) {
    const unsigned g = grid_for(p.S, 256 * 16, 1024);
    switch (p.beta) {
      case 1: hipLaunchKernelGGL((k_qualify<1>), dim3(g), dim3(256), 0, st, dkey, didx, p.S, ctl, Q, ckey, cidx); break;
      case 2: hipLaunchKernelGGL((k_qualify<2>), dim3(g), dim3(256), 0, st, dkey, didx, p.S, ctl, Q, ckey, cidx); break;
      case 4: hipLaunchKernelGGL((k_qualify<4>), dim3(g), dim3(256), 0, st, dkey, didx, p.S, ctl, Q, ckey, cidx); break;
      default: hipLaunchKernelGGL((k_qualify<8>), dim3(g), dim3(256), 0, st, dkey, didx, p.S, ctl, Q, ckey, cidx); break;
    }
  }

  // The k sorted outputs from okey/oidx (exactly k entries), k > kSmallCap.
  // gated: 0 always run, 1 only if the tail kernel set ctl->need_merge
  static void big_sort(const Plan& p, void* ws, uint32_t* out_vals, uint32_t* out_idx, uint32_t* out_kth,
                       int gated, Ctl* ctl, hipStream_t st) {
    uint64_t* A = at<uint64_t>(ws, p.off_A);
    uint64_t* B = at<uint64_t>(ws, p.off_B);
    hipLaunchKernelGGL(k_blocksort, dim3((unsigned)(p.M / kSortTile)), dim3(1024), 0, st,
                       at<uint32_t>(ws, p.off_okey), at<uint32_t>(ws, p.off_oidx), p.k, A, gated, ctl);
    for (uint64_t run = kSortTile; run < p.M; run <<= 1) {
      const int last = (2 * run == p.M) ? 1 : 0;
      hipLaunchKernelGGL((k_merge<DT>), dim3((unsigned)(p.M / 256)), dim3(256), 0, st, A, B, p.M, run, last, p.k,
                         out_vals, out_idx, out_kth, gated, ctl);
      std::swap(A, B);
    }
  }

  // filter_only: stop once the survivors are known (stage checks).
  static void run(const Plan& p, const uint32_t* keys, void* ws, uint32_t* out_vals, uint32_t* out_idx,
                  uint32_t* out_kth, bool kth_only, bool filter_only, hipStream_t st) {
    PhaseMarks pm;
    pm.begin(st);
    run_inner(p, keys, ws, out_vals, out_idx, out_kth, kth_only, filter_only, st, pm);
    pm.end(st);
  }

  static void run_inner(const Plan& p, const uint32_t* keys, void* ws, uint32_t* out_vals, uint32_t* out_idx,
                        uint32_t* out_kth, bool kth_only, bool filter_only, hipStream_t st, PhaseMarks& pm) {
    Ctl* ctl = at<Ctl>(ws, p.off_ctl);
    hipLaunchKernelGGL(k_init, dim3(8), dim3(1024), 0, st, ctl, (uint32_t)p.S, (uint32_t)p.cap_c,
                       p.all ? 1u : 0u);
    pm.start(st);
    uint32_t* okey = at<uint32_t>(ws, p.off_okey);
    uint32_t* oidx = at<uint32_t>(ws, p.off_oidx);
    const uint32_t k = p.k;
    if (p.mode == 1 && p.variant == 0) {
      uint32_t* dkey = at<uint32_t>(ws, p.off_dkey);
      uint32_t* didx = at<uint32_t>(ws, p.off_didx);
      if (k == 1 && !filter_only) {  // the largest delegate is the answer (Rule 1)
        delegate(p, keys, dkey, didx, ctl, st, DirectOut{out_vals, out_idx, out_kth, 1});
        pm.mid(st);
        return;
      }
      delegate(p, keys, dkey, didx, ctl, st);
      pm.mid(st);
      TailArgs ta;
      ta.keys = keys;
      ta.n = p.n;
      ta.alpha = p.alpha;
      ta.S = p.S;
      ta.nd = p.nd;
      ta.k = k;
      ta.kD = p.kD;
      ta.slack = p.slack;
      ta.all = p.all ? 1 : 0;
      ta.kth_only = kth_only ? 1 : 0;
      ta.stop_after_scan = filter_only ? 1 : 0;
      ta.big_sort = (!kth_only && k > (uint32_t)kSmallCap) ? 1 : 0;
      ta.dkey = dkey;
      ta.didx = didx;
      ta.Q = at<uint32_t>(ws, p.off_q);
      ta.ckey = at<uint32_t>(ws, p.off_ckey);
      ta.cidx = at<uint32_t>(ws, p.off_cidx);
      ta.skey = at<uint32_t>(ws, p.off_skey);
      ta.sidx = at<uint32_t>(ws, p.off_sidx);
      ta.okey = okey;
      ta.oidx = oidx;
      ta.cap_s = (uint32_t)p.cap_c;
      ta.out_vals = out_vals;
      ta.out_idx = out_idx;
      ta.out_kth = out_kth;
      ta.ctl = ctl;
      launch_tail(p, ta, st);
      // the merge sort runs only if the tail fell back to its select path
      if (ta.big_sort && !filter_only) big_sort(p, ws, out_vals, out_idx, out_kth, 1, ctl, st);
      return;
    }
    if (p.mode == 1) {
      uint32_t* dkey = at<uint32_t>(ws, p.off_dkey);
      uint32_t* didx = at<uint32_t>(ws, p.off_didx);
      uint32_t* Q = at<uint32_t>(ws, p.off_q);
      uint32_t* ckey = at<uint32_t>(ws, p.off_ckey);
      uint32_t* cidx = at<uint32_t>(ws, p.off_cidx);
      delegate(p, keys, dkey, didx, ctl, st);
      pm.mid(st);
      const unsigned gD = grid_for(p.nd, 256 * 8, 1024);
      for (int pass = 1; pass < kPasses; ++pass)
        hipLaunchKernelGGL((k_pass<SRC_D, DT>), dim3(gD), dim3(256), 0, st, dkey, didx, p.nd, pass, 0, ctl, p.kD);
      qualify(p, dkey, didx, ctl, Q, ckey, cidx, st);
      // expected concatenated length: about k/beta subranges of 2^alpha (grid-stride covers more)
      const unsigned gS = grid_for(((uint64_t)((k - 1) / p.beta) + 1) << p.alpha, 4096, 2048);
      if (p.vec)
        hipLaunchKernelGGL((k_scan<DT, true>), dim3(gS), dim3(256), 0, st, keys, p.n, p.alpha, ctl, Q, ckey, cidx);
      else
        hipLaunchKernelGGL((k_scan<DT, false>), dim3(gS), dim3(256), 0, st, keys, p.n, p.alpha, ctl, Q, ckey, cidx);
      if (filter_only) return;
      const bool may_be_big = p.cap_c > (uint64_t)kSmallCap;
      hipLaunchKernelGGL((k_final_small<SRC_C, DT>), dim3(1), dim3(1024), 0, st, ckey, cidx, (uint64_t)0,
                         may_be_big ? 1 : 0, k, ctl, out_vals, out_idx, out_kth);
      if (!may_be_big) return;
      const unsigned gC = grid_for(p.cap_c, 256 * 8, 1024);
      for (int pass = 0; pass < kPasses; ++pass)
        hipLaunchKernelGGL((k_pass<SRC_C, DT>), dim3(gC), dim3(256), 0, st, ckey, cidx, (uint64_t)0, pass, 2, ctl, k);
      if (kth_only) {
        hipLaunchKernelGGL((k_kth_from_sel<DT>), dim3(1), dim3(64), 0, st, 2, ctl, out_kth);
        return;
      }
      hipLaunchKernelGGL((k_compact<SRC_C, DT>), dim3(gC), dim3(256), 0, st, ckey, cidx, (uint64_t)0, 2, k, ctl, okey,
                         oidx);
      if (k <= (uint32_t)kSmallCap)
        hipLaunchKernelGGL((k_final_small<SRC_OUT, DT>), dim3(1), dim3(1024), 0, st, okey, oidx, (uint64_t)k, 2, k,
                           ctl, out_vals, out_idx, out_kth);
      else
        big_sort(p, ws, out_vals, out_idx, out_kth, 0, ctl, st);
    } else {
      if (p.n <= (uint64_t)kSmallCap) {
        hipLaunchKernelGGL((k_final_small<SRC_V, DT>), dim3(1), dim3(1024), 0, st, keys, (const uint32_t*)nullptr,
                           p.n, 0, k, ctl, out_vals, out_idx, out_kth);
        return;
      }
      const unsigned gV = grid_for(p.n, 256 * 16, 2048);
      for (int pass = 0; pass < kPasses; ++pass) {
        hipLaunchKernelGGL((k_pass<SRC_V, DT>), dim3(gV), dim3(256), 0, st, keys, (const uint32_t*)nullptr, p.n, pass,
                           0, ctl, k);
        if (pass == 0) pm.mid(st);
      }
      if (kth_only) {
        hipLaunchKernelGGL((k_kth_from_sel<DT>), dim3(1), dim3(64), 0, st, 0, ctl, out_kth);
        return;
      }
      hipLaunchKernelGGL((k_compact<SRC_V, DT>), dim3(gV), dim3(256), 0, st, keys, (const uint32_t*)nullptr, p.n, 0,
                         k, ctl, okey, oidx);
      if (k <= (uint32_t)kSmallCap)
        hipLaunchKernelGGL((k_final_small<SRC_OUT, DT>), dim3(1), dim3(1024), 0, st, okey, oidx, (uint64_t)k, 0, k,
                           ctl, out_vals, out_idx, out_kth);
      else
        big_sort(p, ws, out_vals, out_idx, out_kth, 0, ctl, st);
    }
  }
};

template <int DT>
__global__ void k_decode_inplace(uint32_t* v, uint64_t m) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (uint64_t)gridDim.x * blockDim.x)
    v[i] = dec<DT>(v[i]);
}

int check_args(const void* keys, uint64_t n, uint32_t k, int dtype) {
  if (!keys) return DRTOPK_EINVAL;
  if (n == 0 || n >= (1ull << 32)) return DRTOPK_EINVAL;
  if (k == 0 || (uint64_t)k > n) return DRTOPK_EINVAL;
  if (dtype != DRTOPK_U32 && dtype != DRTOPK_F32) return DRTOPK_EINVAL;
  return DRTOPK_OK;
}

uint32_t host_dec(int dt, uint32_t u) { return dt == DT_F32 ? u ^ (((u >> 31) - 1u) | 0x80000000u) : u; }

// Runs the whole path; `fn` (optional) runs under the workspace lock after the
// enqueue, with the plan and workspace pointer.
template <typename F>
int run_common(const void* keys, uint64_t n, uint32_t k, int dtype, void* out_vals, uint32_t* out_idx,
               void* out_kth, bool kth_only, const drtopk_options_t* opt, void* stream, F&& after,
               bool filter_only = false) {
  int st = check_args(keys, n, k, dtype);
  if (st) return st;
  Plan p;
  st = make_plan(keys, n, k, dtype, opt, &p);
  if (st) return st;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DRTOPK_EDEVICE;
  Workspace* ws = workspace_entry(dev, stream);
  if (!ws) return DRTOPK_ENOMEM;
  std::lock_guard<std::mutex> g(ws->mu);
  st = ensure_bytes(ws, p.total);
  if (st) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const uint32_t* kp = static_cast<const uint32_t*>(keys);
  if (p.mode == 3) {
    if (filter_only) return DRTOPK_EINVAL;
    BatchDesc d{};
    d.keys = kp;
    d.n = n;
    d.k = k;
    d.dtype = dtype == DRTOPK_F32 ? DT_F32 : DT_U32;
    d.alpha = (uint32_t)p.alpha;
    d.out_vals = kth_only ? nullptr : static_cast<uint32_t*>(out_vals);
    d.out_idx = kth_only ? nullptr : out_idx;
    d.out_kth = static_cast<uint32_t*>(out_kth);
    hipLaunchKernelGGL(k_one, dim3(1), dim3(kBT), 0, s, d);
    if (hipGetLastError() != hipSuccess) return DRTOPK_EDEVICE;
    return after(p, ws->ptr, s);
  }
  if (dtype == DRTOPK_F32)
    Runner<DT_F32>::run(p, kp, ws->ptr, static_cast<uint32_t*>(out_vals), out_idx, static_cast<uint32_t*>(out_kth),
                        kth_only, filter_only, s);
  else
    Runner<DT_U32>::run(p, kp, ws->ptr, static_cast<uint32_t*>(out_vals), out_idx, static_cast<uint32_t*>(out_kth),
                        kth_only, filter_only, s);
  const hipError_t le = tl_launch_err;
  tl_launch_err = hipSuccess;
  if (hipGetLastError() != hipSuccess || le != hipSuccess) return DRTOPK_EDEVICE;
  return after(p, ws->ptr, s);
}

// Subrange exponent of a problem taken by the batched workgroup kernel; 0 =
// sorted outright (n <= kBSmallN) or radix select without delegates.
int batched_alpha(uint64_t n, uint32_t k) {
  if (n <= kBSmallN) return 0;
  auto subranges = [n](int a) { return (n + (1ull << a) - 1) >> a; };
  int a = -1, b = 0;
  if (tune_lookup(DRTOPK_FORM_BATCHED, n, k, &a, &b) && a == 0) return 0;  // measured: radix select
  if (a < 0) {
    a = rule_alpha(n, k);
    if (a < 8) a = 8;  // a wave reads 256 keys per step: shorter subranges idle lanes
  }
  if (a > 24) a = 24;
  if (a < 2) a = 2;
  while (a < 24 && subranges(a) > kBMaxS) ++a;  // delegate vector fits the LDS
  // at least 2k delegates where the LDS allows: with t the k-th of S subrange
  // maxima, about -S ln(1 - k/S) <= 0.7 S elements survive, within capacity
  while (subranges(a) < 2ull * k && a > 2 && subranges(a - 1) <= kBMaxS) --a;
  return subranges(a) > k && subranges(a) <= kBMaxS ? a : 0;
}

bool batched_eligible(uint64_t n, uint32_t k) { return n <= kBMaxN && k <= kBMaxK; }

// Enqueues one k_batched launch over `items` (already validated).
BatchDesc make_desc(const drtopk_problem_t& q) {
  BatchDesc d{};
  d.keys = static_cast<const uint32_t*>(q.keys);
  d.n = q.n;
  d.k = q.k;
  d.dtype = q.dtype == DRTOPK_F32 ? DT_F32 : DT_U32;
  d.alpha = (uint32_t)batched_alpha(q.n, q.k);
  d.out_vals = static_cast<uint32_t*>(q.out_vals);
  d.out_idx = q.out_idx;
  d.out_kth = static_cast<uint32_t*>(q.out_kth);
  return d;
}

// Tiles of a problem's delegate vector (one workgroup each): problems of
// more than 2^kBTileLog keys on the delegate route with subranges of at
// least 256 keys are split so several workgroups stream them.
uint32_t batched_tiles(const BatchDesc& d) {
  if (d.n <= (1ull << kBTileLog) || d.n <= kBSmallN || d.alpha < 8) return 1;
  const uint32_t tlog = d.alpha > kBTileLog ? d.alpha : kBTileLog;
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
      dg_entries += (descs[i].n + (1ull << descs[i].alpha) - 1) >> descs[i].alpha;
    }
    nwork += descs[i].tiles;
  }
  if (items.size() <= kBInline && !split) {  // descriptors as kernel arguments
    BatchInline b{};
    for (size_t i = 0; i < items.size(); ++i) b.d[i] = descs[i];
    hipLaunchKernelGGL(k_batched_inline, dim3((unsigned)items.size()), dim3(kBT), 0, s, b);
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
                     reinterpret_cast<uint64_t*>(dv + off_dg));
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

__global__ void k_zero_word(uint32_t* p) {
  if (threadIdx.x == 0) *p = 0;
}

int fill_stats(const Plan& p, void* ws, hipStream_t s, drtopk_stats_t* stats) {
  if (!stats) return DRTOPK_OK;
  if (hipStreamSynchronize(s) != hipSuccess) return DRTOPK_EDEVICE;
  if (p.mode == 3) {  // no control block: the workgroup keeps its state in LDS
    std::memset(stats, 0, sizeof(*stats));
    stats->mode = 3;
    stats->alpha = p.alpha;
    stats->beta = 1;
    stats->subranges = p.alpha ? (p.n + (1ull << p.alpha) - 1) >> p.alpha : 0;
    stats->delegates = stats->subranges;
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
  stats->t_key_bits = p.mode == 1 ? host_dec(p.dt, (uint32_t)(h.selD.prefix >> 32)) : 0;
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

int kth_select(const void* keys, uint64_t n, uint32_t k, int dtype, void* out_kth, void* stream) {
  if (!out_kth) return DRTOPK_EINVAL;
  try {
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
      (batched_eligible(problems[i].n, problems[i].k) ? small : large).push_back(&problems[i]);
    std::stable_sort(small.begin(), small.end(),
                     [](const drtopk_problem_t* a, const drtopk_problem_t* b) { return a->n > b->n; });
    if (!small.empty()) {
      int dev = 0;
      if (hipGetDevice(&dev) != hipSuccess) return DRTOPK_EDEVICE;
      Workspace* ws = workspace_entry(dev, stream);
      if (!ws) return DRTOPK_ENOMEM;
      std::lock_guard<std::mutex> lock(ws->mu);
      int st = launch_batched(small, reinterpret_cast<hipStream_t>(stream), ws);
      if (st) return st;
    }
    for (const drtopk_problem_t* q : large) {
      int st = run_common(q->keys, q->n, q->k, (int)q->dtype, q->out_vals, q->out_idx, q->out_kth, !q->out_vals,
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
  uint64_t ws = sizeof(BatchDesc);
  if (!batched_eligible(n, k)) {
    Plan p;
    st = make_plan(dummy, n, k, dtype, nullptr, &p);
    if (st) return st;
    ws = p.total;
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

int drtopk_batched_alpha(uint64_t n, uint32_t k, int32_t* route, int32_t* alpha) {
  if (!route || !alpha || n == 0 || n >= (1ull << 32) || k == 0 || k > n) return DRTOPK_EINVAL;
  if (!batched_eligible(n, k)) {
    *route = 0;
    *alpha = 0;
  } else {
    *alpha = batched_alpha(n, k);
    *route = n <= kBSmallN ? 1 : *alpha ? 2 : 3;
  }
  return DRTOPK_OK;
}

int drtopk_delegates(const void* keys, uint64_t n, int dtype, int alpha, int beta, void* out_dkeys,
                     uint32_t* out_didx, void* stream) {
  if (!out_dkeys || !out_didx) return DRTOPK_EINVAL;
  int st = check_args(keys, n, 1, dtype);
  if (st) return st;
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
  st = ensure_bytes(ws, p.total);
  if (st) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Ctl* ctl = at<Ctl>(ws->ptr, p.off_ctl);
  const uint32_t* kp = static_cast<const uint32_t*>(keys);
  uint32_t* dk = static_cast<uint32_t*>(out_dkeys);
  hipLaunchKernelGGL(k_init, dim3(8), dim3(1024), 0, s, ctl, (uint32_t)p.S, (uint32_t)p.cap_c, 0u);
  const unsigned g = grid_for(p.nd, 256 * 4, 4096);
  if (dtype == DRTOPK_F32) {
    Runner<DT_F32>::delegate(p, kp, dk, out_didx, ctl, s);
    hipLaunchKernelGGL((k_decode_inplace<DT_F32>), dim3(g), dim3(256), 0, s, dk, p.nd);
  } else {
    Runner<DT_U32>::delegate(p, kp, dk, out_didx, ctl, s);
  }
  if (hipGetLastError() != hipSuccess) return DRTOPK_EDEVICE;
  return DRTOPK_OK;
}

int drtopk_candidates(const void* keys, uint64_t n, uint32_t k, int dtype, int alpha, int beta, int variant,
                      uint32_t* out_pos, uint64_t cap, uint64_t* count, uint32_t* t_out, void* stream) {
  if (!out_pos || !count) return DRTOPK_EINVAL;
  if (alpha < 0 || alpha > 24 || !valid_beta(beta)) return DRTOPK_EINVAL;
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
                          t_out[0] = host_dec(p.dt, (uint32_t)(t >> 32));
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

const char* drtopk_status_string(int status) {
  switch (status) {
    case DRTOPK_OK: return "ok";
    case DRTOPK_EINVAL: return "invalid argument";
    case DRTOPK_ENOMEM: return "out of device memory";
    case DRTOPK_EDEVICE: return "device error";
    case DRTOPK_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char* drtopk_version(void) { return "drtopk 0.1 (gfx950)"; }

}  // extern "C"
