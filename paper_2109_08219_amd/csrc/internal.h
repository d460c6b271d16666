// Internal definitions shared by the drtopk kernels and their host driver.
//
// Ordering: every key is compared as a 64-bit composite
//     c = (encoded_key << 32) | ~position
// so a larger composite ranks higher: larger key first, and among equal keys
// the lower position first.  The composite of a padding entry (key 0, position
// 0xFFFFFFFF) is 0, below every real element.  With ties broken this way all
// elements are distinct, and the paper's Rules 1-3 hold exactly.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace drtopk {

constexpr uint32_t kInvalid = 0xFFFFFFFFu;
constexpr int kBins = 2048;       // 11-bit radix digits
constexpr int kPasses = 6;        // 64-bit composite = 11+11+10 key bits, 11+11+10 position bits
constexpr int kSmallCap = 8192;   // candidate counts sorted by one workgroup in LDS
constexpr int kSortTile = 4096;   // block-sort tile of the large-k output sort

enum { DT_U32 = 0, DT_F32 = 1 };
enum { SRC_D = 0, SRC_C = 1, SRC_V = 2, SRC_OUT = 3 };

__host__ __device__ constexpr int pass_shift(int p) {
  return p == 0 ? 53 : p == 1 ? 42 : p == 2 ? 32 : p == 3 ? 21 : p == 4 ? 10 : 0;
}
__host__ __device__ constexpr int pass_bits(int p) { return (p == 2 || p == 5) ? 10 : 11; }

// Selection state of an MSD radix select over composites.
struct Sel {
  uint64_t prefix;  // composite bits fixed so far
  uint64_t mask;    // which composite bits are fixed
  uint32_t rank;    // 1-based rank still sought among entries matching `prefix`
  uint32_t found;   // 1 once the bucket search succeeded, 0 on an inconsistency
};

// Per-call control block at the head of the workspace; zeroed by k_init.
struct Ctl {
  uint32_t histD[kPasses][kBins];  // digit histograms of the delegate select
  uint32_t histC[kPasses][kBins];  // digit histograms of the survivor select
  Sel selD;                        // k-th largest delegate (the threshold t)
  Sel selC;                        // k-th largest survivor
  uint32_t ticketD[kPasses + 1];
  uint32_t ticketC[kPasses + 1];
  uint32_t nq;    // subranges to re-read
  uint32_t nc;    // survivors
  uint32_t nout;  // compacted outputs (large-survivor path)
  uint32_t err;   // nonzero: an internal consistency check failed
  uint32_t cap_q; // capacity of the qualifying-subrange list
  uint32_t cap_c; // capacity of the survivor buffer
  uint32_t all;   // 1: fewer delegates than k, every subrange qualifies (t = lowest)
};

// Fill levels clamped to their buffers (a violated bound sets err instead of
// writing past the end).
__device__ __forceinline__ uint32_t clamp_nc(const Ctl* c) { return c->nc < c->cap_c ? c->nc : c->cap_c; }
__device__ __forceinline__ uint32_t clamp_nq(const Ctl* c) { return c->nq < c->cap_q ? c->nq : c->cap_q; }

// Order-preserving uint32 encoding of the input bit patterns.
template <int DT>
__device__ __forceinline__ uint32_t enc(uint32_t b) {
  if constexpr (DT == DT_U32) return b;
  else return b ^ ((uint32_t)((int32_t)b >> 31) | 0x80000000u);
}
template <int DT>
__device__ __forceinline__ uint32_t dec(uint32_t u) {
  if constexpr (DT == DT_U32) return u;
  else return u ^ (((u >> 31) - 1u) | 0x80000000u);
}

__device__ __forceinline__ uint64_t comp(uint32_t key, uint32_t pos) {
  return ((uint64_t)key << 32) | (uint64_t)(~pos);
}
__device__ __forceinline__ uint32_t comp_key(uint64_t c) { return (uint32_t)(c >> 32); }
__device__ __forceinline__ uint32_t comp_pos(uint64_t c) { return ~(uint32_t)c; }

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int m) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  lo = (uint32_t)__shfl_xor((int)lo, m);
  hi = (uint32_t)__shfl_xor((int)hi, m);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t atomic_load_u32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave-wide append: every lane with `pred` gets a distinct slot in a global
// array whose fill level is *counter; one atomic per wave.  Call with the
// whole wave active.
__device__ __forceinline__ uint32_t wave_append(bool pred, uint32_t* counter) {
  uint64_t b = __ballot(pred);
  uint32_t base = 0;
  if (b) {
    int leader = __ffsll((unsigned long long)b) - 1;
    if ((int)lane_id() == leader) base = atomicAdd(counter, (uint32_t)__popcll(b));
    base = (uint32_t)__shfl((int)base, leader);
  }
  return base + mbcnt(b);
}

}  // namespace drtopk
