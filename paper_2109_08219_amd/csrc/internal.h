// Internal definitions shared by the drtopk kernels and their host driver.
//
// Ordering: every key is compared as a 64-bit composite
//     c = (encoded_key << 32) | ~position
// so a larger composite ranks higher: larger key first, and among equal keys
// the lower position first.  The composite of a padding entry (key 0, position
// 0xFFFFFFFF) is 0, below every real element.  With ties broken this way all
// elements are distinct, and the paper's Rules 1-3 hold exactly.
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace drtopk {

constexpr uint32_t kInvalid = 0xFFFFFFFFu;
constexpr int kBins = 2048;       // 11-bit radix digits
constexpr int kPasses = 6;        // 64-bit composite = 11+11+10 key bits, 11+11+10 position bits
constexpr int kSmallCap = 8192;   // candidate counts sorted by one workgroup in LDS
constexpr int kSortTile = 4096;   // block-sort tile of the large-k output sort
constexpr uint32_t kBtMaxK = 256;        // largest k of the bitonic top-k (tail variant 2)
constexpr uint32_t kBtRoundBlocks = 256; // most blocks of one bitonic top-k round

// Key codecs: bits 0-1 the key type, DT_MIN set = the k smallest first.
enum { DT_U32 = 0, DT_F32 = 1, DT_I32 = 2, DT_MIN = 4 };
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

// One phase of the tail kernel: chunk claims, completed chunks, ready flag
// (each on its own 256-byte line).
struct Phase {
  uint32_t claim;
  uint32_t pad0[31];
  uint32_t done;
  uint32_t pad1[31];
  uint32_t ready;
  uint32_t pad2[63];
};
constexpr int kPhases = 48;  // the tail's own phases, then the levels of its large-k merge sort

// Per-call control block at the head of the workspace; zeroed by k_init.
struct Ctl {
  Phase ph[kPhases];
  uint32_t histD[kPasses][kBins];  // digit histograms of the delegate select
  uint32_t histC[kPasses][kBins];  // digit histograms of the survivor select
  uint32_t histL[kBins];           // delegates by log-distance from the top of the key range
  uint32_t histW[kPasses][kBins];  // digit histograms of the select over W (compacted delegates)
  uint32_t histH[kBins];           // refinement of the cut bin (next finer digit)
  uint32_t bcount[kBins];          // survivors per output bucket
  uint32_t bcur[kBins];            // scatter cursors per output bucket
  Sel selD;                        // k-th largest delegate (the threshold t)
  Sel selC;                        // k-th largest survivor
  uint32_t ticketD[kPasses + 1];
  uint32_t ticketC[kPasses + 1];
  Sel selW;
  uint32_t cut_lo, cut_hi;  // key interval of the cut bin
  uint32_t cut_rank;        // rank of the kD-th delegate inside the cut bin
  uint32_t cut_count;       // delegates in the cut bin
  uint32_t bstar;           // output bucket holding slot k-1 (buckets after it are not scattered)
  uint32_t bigbucket;       // an output bucket overflows one workgroup: take the select path
  uint32_t ngroups;         // output sort groups
  uint32_t need_merge;      // the select fallback was taken with k > kSmallCap (merge-sort phases ran)
  uint32_t wmap;  // monotone map used to cut the delegates: 0 top 11 bits, 1 log-distance
  uint32_t wbin;  // delegates with bin >= wbin form W, a superset of those ranked >= t
  uint32_t wsize; // |W|, known from the fused histogram
  uint32_t nw;    // W fill level
  uint32_t selpub[8];  // selection state published between tail phases (W: 0..3, survivors: 4..7)
  uint32_t uniq_idx;  // position of a unique entry found by a tail pass
  uint32_t tpub[4];   // threshold t' and its bin, published by block 0 of the tail (coherent stores)
  uint32_t rkmax;     // refinement: largest delegate key in the cut bin
  uint32_t rknmin;    // refinement: complement of the smallest delegate key in the cut bin
  uint64_t tstamp[kPhases + 2];  // device real-time clock: tail start, each phase's completion
  uint64_t max1;  // largest delegate composite = largest element (the k = 1 answer)
  uint32_t dknmin;  // complement of the smallest delegate key (0 = no delegate)
  // bucket select (tail variant 3), [0] over the delegates, [1] over the survivors
  uint64_t bmax[2];   // largest composite of the source
  uint64_t bnmin[2];  // complement of the smallest
  uint64_t blo[2], bhi[2];  // live range, shrunk to the bucket holding the sought rank
  uint32_t brank[2];  // rank still sought inside it
  uint32_t bdone[2];  // the range is one composite: the selection is done
  uint32_t bticket[2][kPasses];  // its pass tickets (histograms: histW over the delegates, histC)
  uint32_t nq;    // subranges to re-read
  uint32_t nc;    // survivors
  uint32_t nout;  // compacted outputs (large-survivor path)
  uint32_t err;   // nonzero: an internal consistency check failed
  uint32_t cap_q; // capacity of the qualifying-subrange list
  uint32_t cap_c; // capacity of the survivor buffer
  uint32_t all;   // 1: fewer delegates than k, every subrange qualifies (t = lowest)
  uint32_t* rec;  // the stream's sticky check record (kErrWords words, not cleared per call)
  uint32_t boff[kBins + 1];   // first output slot of each bucket
  uint32_t gfirst[kBins + 1]; // first bucket of each sort group
  uint32_t bgrp[kBins];       // sort group of each bucket up to b*
  uint32_t gbase[kBins + 1];  // first output slot of each sort group
};

// Internal consistency checks.  A failed check means a defect of the library
// (or the survivor-capacity testing hook), never bad input; the flags are
// OR-ed into Ctl::err for this call's statistics and recorded in the stream's
// check record, which stays set until the host reads and clears it.
enum : uint32_t {
  ERR_SELECT = 1u,  // a radix-select bucket search found no bucket holding the rank
  ERR_FEW = 2u,     // fewer survivors than k reached the output step
  ERR_CAP = 16u,    // a bounded buffer was full: writes past its end were dropped
  ERR_WAIT = 64u,   // a phase wait gave up after about a second
  ERR_GROUP = 128u, // an output sort group exceeded one workgroup
};
constexpr int kErrWords = 8;  // check record: word i set <=> flag bit i raised

// Records `bit` (one of the ERR_ flags) in the record `rec`: word log2(bit)
// is set by a plain store, so concurrent setters of different flags never
// overwrite each other, and no atomic to host memory is needed.
__device__ __forceinline__ void record_err(uint32_t* rec, uint32_t bit) {
  if (rec) rec[__builtin_ctz(bit)] = 1u;
}
__device__ __forceinline__ void flag_err(Ctl* c, uint32_t bit) {
  atomicOr(&c->err, bit);
  record_err(c->rec, bit);
}

// Fill levels clamped to their buffers (a violated bound sets err instead of
// writing past the end).
__device__ __forceinline__ uint32_t clamp_nc(const Ctl* c) { return c->nc < c->cap_c ? c->nc : c->cap_c; }
__device__ __forceinline__ uint32_t clamp_nq(const Ctl* c) { return c->nq < c->cap_q ? c->nq : c->cap_q; }

// Order-preserving uint32 encoding of the input bit patterns: the larger
// encoding ranks first.  float32 by IEEE totalOrder (negative patterns have
// every bit flipped, non-negative ones the sign bit), int32 with the sign bit
// flipped; for the k smallest the encoding is complemented, so the same
// kernels select them (ties still go to the lower position).
template <int DT>
__device__ __forceinline__ uint32_t enc(uint32_t b) {
  uint32_t e;
  if constexpr ((DT & 3) == DT_U32) e = b;
  else if constexpr ((DT & 3) == DT_F32) e = b ^ ((uint32_t)((int32_t)b >> 31) | 0x80000000u);
  else e = b ^ 0x80000000u;
  if constexpr ((DT & DT_MIN) != 0) e = ~e;
  return e;
}
template <int DT>
__device__ __forceinline__ uint32_t dec(uint32_t u) {
  if constexpr ((DT & DT_MIN) != 0) u = ~u;
  if constexpr ((DT & 3) == DT_U32) return u;
  else if constexpr ((DT & 3) == DT_F32) return u ^ (((u >> 31) - 1u) | 0x80000000u);
  else return u ^ 0x80000000u;
}


__device__ __forceinline__ uint64_t comp(uint32_t key, uint32_t pos) {
  return ((uint64_t)key << 32) | (uint64_t)(~pos);
}
__device__ __forceinline__ uint32_t comp_key(uint64_t c) { return (uint32_t)(c >> 32); }
__device__ __forceinline__ uint32_t comp_pos(uint64_t c) { return ~(uint32_t)c; }

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63; }

// Monotone bin of a key by its distance from the top of the uint32 range,
// with 64 sub-bins per octave: maxima of many keys crowd near the top, where
// equal-width digits put most of them in one bin.  Larger key -> larger or
// equal bin; bins 320..2047 are used.
__device__ __forceinline__ uint32_t log_bin(uint32_t key) {
  const uint32_t x = ~key;
  if (x < 64u) return 2047u - x;
  const uint32_t e = 32u - (uint32_t)__clz((int)x);  // bit length, 7..32
  const uint32_t m = (x >> (e - 7u)) & 63u;
  return 2047u - (64u + (e - 7u) * 64u + m);
}
__device__ __forceinline__ uint32_t top_bin(uint32_t key) { return key >> 21; }

// Key interval [lo, hi] of a bin of either map (inverse of top_bin / log_bin).
__device__ __forceinline__ void bin_interval(uint32_t map, uint32_t bin, uint32_t& lo, uint32_t& hi) {
  if (map == 0) {
    lo = bin << 21;
    hi = lo | 0x1FFFFFu;
    return;
  }
  const uint32_t f = 2047u - bin;
  if (f < 64u) {
    lo = hi = ~f;
    return;
  }
  const uint32_t e = 7u + (f - 64u) / 64u, m = (f - 64u) % 64u;
  const uint64_t xlo = (uint64_t)(64u + m) << (e - 7u);
  const uint64_t xhi = ((uint64_t)(65u + m) << (e - 7u)) - 1u;
  lo = ~(uint32_t)xhi;
  hi = ~(uint32_t)xlo;
}

__device__ __forceinline__ uint32_t bitlen32(uint32_t x) { return x ? 32u - (uint32_t)__clz((int)x) : 0u; }
__device__ __forceinline__ uint32_t bitlen64(uint64_t x) {
  return x ? 64u - (uint32_t)__clzll((long long)x) : 0u;
}

// Coherent (device-scope, sc1) accesses for data exchanged between blocks of
// one kernel: they bypass the per-XCD L2, so no cache writeback is needed.
__device__ __forceinline__ void st_coh(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_coh(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_coh64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coh64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// The value held by a lane in the other M-half of this lane's 2M-lane block
// (M a power of two below 64), by VALU lane operations only: DPP quad
// permutes (M = 1, 2), DPP row half-mirror and mirror (4, 8: lane i of an
// 8- or 16-lane row pairs with 7 - i or 15 - i), and the gfx950 row and half
// swaps (16, 32).  Exact lane ^ M for M = 1, 2, 16, 32; for 4 and 8 it is
// another lane of the other half, which is what a butterfly reduction needs
// once the lanes of each M-block agree (their results then equal lane ^ M's).
template <int M>
__device__ __forceinline__ uint32_t lane_cross32(uint32_t v) {
  if constexpr (M == 1) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);
  else if constexpr (M == 2) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);
  else if constexpr (M == 4) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false);
  else if constexpr (M == 8) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false);
  else if constexpr (M == 16) {
    // both results hold this lane's own value and its partner's (one each)
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return r[0] == v ? r[1] : r[0];
  } else {
    static_assert(M == 32, "lane_cross32: M in {1, 2, 4, 8, 16, 32}");
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return r[0] == v ? r[1] : r[0];
  }
}
template <int M>
__device__ __forceinline__ uint64_t lane_cross64(uint64_t v) {
  return ((uint64_t)lane_cross32<M>((uint32_t)(v >> 32)) << 32) | lane_cross32<M>((uint32_t)v);
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
