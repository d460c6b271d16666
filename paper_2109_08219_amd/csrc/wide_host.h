// Host side of the 64-bit key path: plan and enqueue (implemented in
// wide.hip, its own translation unit).
#pragma once

#include <cstddef>
#include <cstdint>

#include <hip/hip_runtime.h>

#include "drtopk.h"

namespace drtopk {

struct WPlan {
  int mode = 0;  // 1 delegate method, 2 radix select over the whole input
  int alpha = 0;
  int dt = 0;    // public dtype (DRTOPK_U64 / I64 / F64, optionally | DRTOPK_SMALLEST)
  uint64_t n = 0;
  uint32_t k = 0;
  bool vec = false;  // keys 16-byte aligned: 128-bit loads
  uint64_t S = 0, cap_c = 0, chunk = 0, M = 0;
  uint64_t codec_a = 0, codec_c = 0;
  size_t off_ctl = 0, off_dkey = 0, off_didx = 0, off_q = 0, off_ckey = 0, off_cidx = 0;
  size_t off_okey = 0, off_oidx = 0, off_A = 0, off_B = 0, off_pos = 0, total = 0;
};

inline bool wide_dtype(int dtype) {
  const int base = dtype & ~DRTOPK_SMALLEST;
  return base == DRTOPK_U64 || base == DRTOPK_I64 || base == DRTOPK_F64;
}

// Plan of one 64-bit-key call (no device work).  pos_in_ws: reserve k output
// positions in the workspace (WPlan::off_pos).
int wide_plan(uint64_t n, uint32_t k, int dtype, bool vec, const drtopk_options_t* opt, WPlan* out,
              bool pos_in_ws = false);

// Enqueues the whole path on `s` over the workspace `ws` (at least p.total
// bytes).  kth_only: only out_kth is written.
int wide_enqueue(const WPlan& p, const void* keys, void* ws, uint32_t* rec, void* out_vals, uint32_t* out_idx,
                 void* out_kth, bool kth_only, hipStream_t s);

// Counters of a finished call (the stream synchronised): qualifying
// subranges, survivors, check flags, the threshold's key bits and position.
int wide_counters(const WPlan& p, void* ws, uint64_t* scanned, uint64_t* candidates, uint32_t* err,
                  uint64_t* t_key_bits, uint32_t* t_idx);

}  // namespace drtopk
