// Host-side pieces shared by the library's translation units: the plan of
// one call, launch error tracking, optional phase timing, and the per-codec
// entry points of the single-problem path (one translation unit per codec,
// compiled in parallel).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <mutex>
#include <type_traits>
#include <vector>

#include "drtopk.h"
#include "internal.h"

namespace drtopk {

struct Plan {
  int mode = 0;  // 1 delegate method, 2 plain radix select on V, 3 one workgroup (batched kernel)
  int alpha = 0, beta = 1;
  int dt = 0;
  uint64_t n = 0;
  uint32_t k = 0;
  uint64_t S = 0, nd = 0, cap_c = 0, chunk = 0, M = 0;
  uint32_t kD = 0;   // rank sought among the delegates: min(k, |D|)
  uint32_t slack = 0;
  int variant = 0;   // 0: cooperative tail kernel, 1: one kernel per step (radix selects),
                     // 2: bitonic top-k selects (k <= 256), 3: bucket selects
  bool all = false;  // fewer real delegates than k: no threshold, every subrange qualifies
  bool vec = false;
  size_t off_ctl = 0, off_dkey = 0, off_didx = 0, off_q = 0, off_ckey = 0, off_cidx = 0;
  size_t off_okey = 0, off_oidx = 0, off_A = 0, off_B = 0, off_skey = 0, off_sidx = 0, total = 0;
  size_t off_pos = 0;  // k output positions kept in the workspace (payload gathers without out_idx)
  size_t off_L0 = 0, off_L1 = 0;  // variant 2: partial top-k lists of the bitonic rounds
  uint32_t* rec = nullptr;  // the stream's check record (set by the caller before the enqueue)
  bool marks = true;        // phase timing events may be recorded (drtopk_timing_enable)
};

extern thread_local hipError_t tl_launch_err;  // launches whose API reports errors directly

template <typename T>
inline T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

inline unsigned grid_for(uint64_t items, uint64_t per_block, unsigned cap) {
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
};
extern Timing g_timing;

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

// Calls f(std::integral_constant<int, DT>{}) for a codec (0..2, 4..6): the
// host-side dispatch to the per-codec translation units.
template <typename F>
inline void with_codec(int code, F&& f) {
  switch (code) {
    case DT_F32: f(std::integral_constant<int, DT_F32>{}); break;
    case DT_I32: f(std::integral_constant<int, DT_I32>{}); break;
    case DT_U32 | DT_MIN: f(std::integral_constant<int, DT_U32 | DT_MIN>{}); break;
    case DT_F32 | DT_MIN: f(std::integral_constant<int, DT_F32 | DT_MIN>{}); break;
    case DT_I32 | DT_MIN: f(std::integral_constant<int, DT_I32 | DT_MIN>{}); break;
    default: f(std::integral_constant<int, DT_U32>{}); break;
  }
}

// The whole single-problem path for plan p on codec DT (enqueue only).
template <int DT>
void run_codec(const Plan& p, const uint32_t* keys, void* ws, uint32_t* out_vals, uint32_t* out_idx,
               uint32_t* out_kth, bool kth_only, bool filter_only, hipStream_t st);
// The delegate vector alone, decoded to the input's bit patterns.
template <int DT>
void delegates_codec(const Plan& p, const uint32_t* keys, uint32_t* dkey, uint32_t* didx, Ctl* ctl, hipStream_t st);

}  // namespace drtopk
