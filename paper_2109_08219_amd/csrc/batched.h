// Many independent top-k problems in one persistent launch.
//
// Each workgroup (kBT threads) takes whole problems from an atomic counter,
// largest first (the host orders them), and runs the delegate method for one
// problem entirely in its LDS:
//   delegate vector (Rule 1, beta = 1): one wave per subrange of 2^alpha keys;
//   t = the k-th largest delegate: the delegate vector sorted in registers;
//   survivors (Rule 2): t itself plus every element ranked >= t in the k-1
//     subranges whose delegate ranks above t (an element >= t lies either in
//     such a subrange or is t), read as one virtual concatenated vector;
//   output: survivors sorted in registers, the first k written.
// Problems of at most kBSmallN keys are sorted outright.  A problem whose
// survivors overflow the LDS (adversarial inputs), or whose delegate vector
// would not exceed k, takes a block-level MSD radix select over its keys.
// No workgroup ever waits for another: the only shared state is the claim
// counter.
#pragma once

#include "tail.h"

namespace drtopk {

constexpr int kBT = 1024;              // threads per workgroup
constexpr uint32_t kBSmallN = 8192;    // problems this small are sorted outright
constexpr uint32_t kBMaxS = 4096;      // delegate vector capacity (LDS)
constexpr uint32_t kBSurv = 8192;      // survivor capacity (LDS)
constexpr uint32_t kBMaxK = 2048;      // largest k handled in a workgroup
constexpr uint64_t kBMaxN = 1ull << 22;  // largest n handled in a workgroup

// One problem as the kernel sees it (64 bytes).
struct BatchDesc {
  const uint32_t* keys;
  uint64_t n;
  uint32_t k;
  uint32_t dtype;
  uint32_t alpha;  // subrange exponent, >= 2; 0 = radix select without delegates
  uint32_t pad;
  uint32_t* out_vals;
  uint32_t* out_idx;
  uint32_t* out_kth;
  uint64_t pad2;
};
static_assert(sizeof(BatchDesc) == 64, "BatchDesc layout");

struct BatchSmem {
  uint64_t D[kBMaxS];     // delegate composites, then sorted
  uint64_t surv[kBSurv];  // survivors, also the exchange buffer of their sort
  uint32_t hist[kBins];
  uint32_t scan[kBT];
  uint32_t nsurv;
  uint32_t item;
  uint32_t out[4];
};

// Bin holding the rank-th largest entry of an LDS histogram (kBT threads, two
// bins each): sm.out = {bin, rank within the bin, found, count of the bin}.
__device__ inline void bb_bucket(const uint32_t* h, uint32_t rank, BatchSmem& sm) {
  const int t = threadIdx.x;
  const uint32_t c0 = h[kBins - 1 - 2 * t], c1 = h[kBins - 2 - 2 * t];
  const uint32_t sum = c0 + c1;
  sm.scan[t] = sum;
  if (t == 0) { sm.out[0] = 0; sm.out[1] = 0; sm.out[2] = 0; sm.out[3] = 0; }
  __syncthreads();
  for (int off = 1; off < kBT; off <<= 1) {
    const uint32_t x = t >= off ? sm.scan[t - off] : 0u;
    __syncthreads();
    sm.scan[t] += x;
    __syncthreads();
  }
  const uint32_t incl = sm.scan[t], excl = incl - sum;
  if (excl < rank && rank <= incl) {
    if (excl + c0 >= rank) {
      sm.out[0] = kBins - 1 - 2 * t; sm.out[1] = rank - excl; sm.out[3] = c0;
    } else {
      sm.out[0] = kBins - 2 - 2 * t; sm.out[1] = rank - excl - c0; sm.out[3] = c1;
    }
    sm.out[2] = 1;
  }
  __syncthreads();
}

// Sorts `cnt` composites from LDS array `src` and writes the first `k` as
// outputs 0..k-1.  `src` holds at least E * kBT entries and serves as the
// exchange buffer of the sort once every thread has loaded its elements.
template <int DT, int E>
__device__ __noinline__ void b_sort_write_e(uint64_t* src, uint32_t cnt, uint32_t k, uint32_t* out_vals,
                                            uint32_t* out_idx, uint32_t* out_kth) {
  uint64_t v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint32_t g = threadIdx.x * E + e;
    v[e] = g < cnt ? src[g] : 0ull;
  }
  block_bitonic<E, kBT>(v, src);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint32_t g = threadIdx.x * E + e;
    if (g < k) write_out<DT>(v[e], g, k, out_vals, out_idx, out_kth);
  }
}

// cnt <= kBSurv, k <= cnt.
template <int DT>
__device__ inline void b_sort_write(uint64_t* src, uint32_t cnt, uint32_t k, uint32_t* out_vals, uint32_t* out_idx,
                                    uint32_t* out_kth) {
  if (cnt <= 1u * kBT) b_sort_write_e<DT, 1>(src, cnt, k, out_vals, out_idx, out_kth);
  else if (cnt <= 2u * kBT) b_sort_write_e<DT, 2>(src, cnt, k, out_vals, out_idx, out_kth);
  else if (cnt <= 4u * kBT) b_sort_write_e<DT, 4>(src, cnt, k, out_vals, out_idx, out_kth);
  else b_sort_write_e<DT, 8>(src, cnt, k, out_vals, out_idx, out_kth);
}

// Problems of at most kBSmallN keys: load all composites, sort, write.
template <int DT>
__device__ inline void b_small(const BatchDesc& d, BatchSmem& sm) {
  const uint32_t n = (uint32_t)d.n;
  for (uint32_t i = threadIdx.x; i < n; i += kBT) sm.surv[i] = comp(enc<DT>(d.keys[i]), i);
  __syncthreads();
  b_sort_write<DT>(sm.surv, n, d.k, d.out_vals, d.out_idx, d.out_kth);
}

// Block-level MSD radix select of the k-th composite over the problem's keys,
// exact compaction of the k entries ranked at or above it, sort, write.
template <int DT>
__device__ inline void b_radix(const BatchDesc& d, BatchSmem& sm) {
  const uint32_t n = (uint32_t)d.n, k = d.k;
  uint64_t prefix = 0, mask = 0;
  uint32_t r = k;
  bool key_only = false;
  for (int p = 0; p < kPasses; ++p) {
    for (int i = threadIdx.x; i < kBins; i += kBT) sm.hist[i] = 0;
    __syncthreads();
    const int sh = pass_shift(p);
    const uint32_t dm = (1u << pass_bits(p)) - 1;
    const uint32_t kmask = (uint32_t)(mask >> 32), kpref = (uint32_t)(prefix >> 32);
    const uint32_t imask = (uint32_t)mask, ipref = (uint32_t)prefix;
    for (uint32_t i = threadIdx.x; i < n; i += kBT) {
      const uint32_t kk = enc<DT>(d.keys[i]);
      if ((kk & kmask) != kpref) continue;
      uint64_t x = (uint64_t)kk << 32;
      if (p >= 3) {
        const uint32_t ip = ~i;
        if ((ip & imask) != ipref) continue;
        x |= ip;
      }
      atomicAdd(&sm.hist[(uint32_t)(x >> sh) & dm], 1u);
    }
    __syncthreads();
    bb_bucket(sm.hist, r, sm);
    prefix |= (uint64_t)sm.out[0] << sh;
    mask |= (uint64_t)dm << sh;
    r = sm.out[1];
    if (p == 2 && sm.out[3] == 1u) {  // the k-th key is unique: every key >= it is in the answer
      key_only = true;
      break;
    }
  }
  const uint64_t T = key_only ? (prefix & 0xFFFFFFFF00000000ull) : prefix;
  if (threadIdx.x == 0) sm.nsurv = 0;
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < n; i += kBT) {
    const uint64_t x = comp(enc<DT>(d.keys[i]), i);
    if (x >= T) {
      const uint32_t s = atomicAdd(&sm.nsurv, 1u);
      if (s < kBSurv) sm.surv[s] = x;
    }
  }
  __syncthreads();
  const uint32_t ns = sm.nsurv < kBSurv ? sm.nsurv : kBSurv;
  b_sort_write<DT>(sm.surv, ns, k, d.out_vals, d.out_idx, d.out_kth);
}

// Loads 4 consecutive keys at p (p a multiple of 4); those at or beyond
// `end` read as 0 and are ignored by the caller.
__device__ __forceinline__ void b_load4(const uint32_t* keys, uint32_t p, uint32_t end, bool vec, uint32_t (&v)[4]) {
  if (vec && p + 4 <= end) {
    const u32x4 x = *reinterpret_cast<const u32x4*>(keys + p);
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = p + c < end ? keys[p + c] : 0u;
  }
}

// The delegate method for one problem; false if the survivors overflow LDS
// (nothing has been written then).
template <int DT>
__device__ inline bool b_delegate(const BatchDesc& d, BatchSmem& sm) {
  const uint32_t n = (uint32_t)d.n, k = d.k, alpha = d.alpha;
  const uint32_t L = 1u << alpha;
  const uint32_t S = (n + L - 1) >> alpha;
  const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
  constexpr uint32_t kWaves = kBT / 64;
  const bool vec = (reinterpret_cast<uintptr_t>(d.keys) & 15u) == 0;
  // delegate vector: one wave per subrange
  for (uint32_t s = wave; s < S; s += kWaves) {
    const uint32_t lo = s << alpha, hi = lo + L < n ? lo + L : n;
    uint64_t m = 0;
    for (uint32_t p = lo + lane * 4; p < hi; p += 256) {
      uint32_t v[4];
      b_load4(d.keys, p, hi, vec, v);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const uint64_t x = comp(enc<DT>(v[c]), p + c);
        if (p + c < hi && x > m) m = x;
      }
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint64_t y = shfl_xor64(m, o);
      m = y > m ? y : m;
    }
    if (lane == 0) sm.D[s] = m;
  }
  __syncthreads();
  // t: the delegate vector sorted (descending) in registers and kept in LDS
  {
    uint64_t v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint32_t g = threadIdx.x * 4 + e;
      v[e] = g < S ? sm.D[g] : 0ull;
    }
    block_bitonic<4, kBT>(v, sm.D);
#pragma unroll
    for (int e = 0; e < 4; ++e) sm.D[threadIdx.x * 4 + e] = v[e];
  }
  if (threadIdx.x == 0) sm.nsurv = 0;
  __syncthreads();
  const uint64_t t = sm.D[k - 1];
  // survivors: elements >= t in the subranges of the k-1 delegates above t
  const uint32_t total = (k - 1) << alpha;
  for (uint32_t e = threadIdx.x * 4; e < total; e += kBT * 4) {
    const uint32_t s = comp_pos(sm.D[e >> alpha]) >> alpha;
    const uint32_t p = (s << alpha) + (e & (L - 1));
    uint32_t v[4];
    b_load4(d.keys, p, n, vec, v);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const uint64_t x = comp(enc<DT>(v[c]), p + c);
      if (p + c < n && x >= t) {
        const uint32_t slot = atomicAdd(&sm.nsurv, 1u);
        if (slot < kBSurv) sm.surv[slot] = x;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t slot = atomicAdd(&sm.nsurv, 1u);  // t itself: its subrange is not re-read
    if (slot < kBSurv) sm.surv[slot] = t;
  }
  __syncthreads();
  const uint32_t ns = sm.nsurv;
  if (ns > kBSurv) return false;
  b_sort_write<DT>(sm.surv, ns, k, d.out_vals, d.out_idx, d.out_kth);
  return true;
}

template <int DT>
__device__ inline void b_problem(const BatchDesc& d, BatchSmem& sm) {
  if (d.n <= kBSmallN) {
    b_small<DT>(d, sm);
    return;
  }
  if (d.alpha >= 2) {
    const uint64_t S = (d.n + (1ull << d.alpha) - 1) >> d.alpha;
    if (S <= kBMaxS && S > d.k && b_delegate<DT>(d, sm)) return;
    __syncthreads();
  }
  b_radix<DT>(d, sm);
}

// Grid: any number of workgroups of kBT threads; *counter starts at 0.
__global__ __launch_bounds__(kBT) void k_batched(const BatchDesc* __restrict__ descs, uint32_t count,
                                                 uint32_t* counter) {
  __shared__ BatchSmem sm;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) sm.item = atomicAdd(counter, 1u);
    __syncthreads();
    const uint32_t i = sm.item;
    if (i >= count) break;
    const BatchDesc d = descs[i];
    if (d.dtype == DT_F32) b_problem<DT_F32>(d, sm);
    else b_problem<DT_U32>(d, sm);
  }
}

}  // namespace drtopk
