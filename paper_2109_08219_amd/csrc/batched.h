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
// Two workgroups share a CU, so one streams keys while the other sorts.
// No workgroup ever waits for another: the only shared state is the claim
// counter.
#pragma once

#include "tail.h"

namespace drtopk {

constexpr int kBT = 512;                  // threads per workgroup (two workgroups per CU)
constexpr int kBWaves = kBT / 64;
constexpr uint32_t kBSmallN = 4096;       // problems this small are sorted outright
constexpr uint32_t kBMaxS = 4096;         // delegate vector capacity (LDS)
constexpr uint32_t kBSurv = 4096;         // survivor capacity (LDS)
constexpr uint32_t kBMaxK = 2048;         // largest k handled in a workgroup
constexpr uint64_t kBMaxN = 1ull << 22;   // largest n handled in a workgroup
constexpr int kBU = 8;                    // 1 KiB wave loads in flight per wave step
constexpr uint32_t kBStep = 256 * kBU;    // keys per wave step

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

__device__ __forceinline__ uint64_t wave_max64(uint64_t m) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t y = shfl_xor64(m, o);
    m = y > m ? y : m;
  }
  return m;
}

// Bin holding the rank-th largest entry of an LDS histogram (each thread owns
// kBins / kBT consecutive bins, highest first): sm.out = {bin, rank within the
// bin, found, count of the bin}.
__device__ inline void bb_bucket(const uint32_t* h, uint32_t rank, BatchSmem& sm) {
  constexpr int PER = kBins / kBT;
  const int t = threadIdx.x;
  uint32_t c[PER], sum = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    c[j] = h[kBins - 1 - PER * t - j];
    sum += c[j];
  }
  sm.scan[t] = sum;
  if (t == 0) { sm.out[0] = 0; sm.out[1] = 0; sm.out[2] = 0; sm.out[3] = 0; }
  __syncthreads();
  for (int off = 1; off < kBT; off <<= 1) {
    const uint32_t x = t >= off ? sm.scan[t - off] : 0u;
    __syncthreads();
    sm.scan[t] += x;
    __syncthreads();
  }
  uint32_t excl = sm.scan[t] - sum;
  if (excl < rank && rank <= excl + sum) {
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      if (excl < rank && rank <= excl + c[j]) {
        sm.out[0] = kBins - 1 - PER * t - j;
        sm.out[1] = rank - excl;
        sm.out[3] = c[j];
        sm.out[2] = 1;
      }
      excl += c[j];
    }
  }
  __syncthreads();
}

// Sorts `cnt` composites of LDS array `src` (descending) and leaves them
// there; `src` holds at least E * kBT entries.
template <int E>
__device__ __noinline__ void b_sort_lds_e(uint64_t* src, uint32_t cnt) {
  uint64_t v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint32_t g = threadIdx.x * E + e;
    v[e] = g < cnt ? src[g] : 0ull;
  }
  block_bitonic<E, kBT>(v, src);
#pragma unroll
  for (int e = 0; e < E; ++e) src[threadIdx.x * E + e] = v[e];
  __syncthreads();
}

__device__ inline void b_sort_lds(uint64_t* src, uint32_t cnt) {
  if (cnt <= 1u * kBT) b_sort_lds_e<1>(src, cnt);
  else if (cnt <= 2u * kBT) b_sort_lds_e<2>(src, cnt);
  else if (cnt <= 4u * kBT) b_sort_lds_e<4>(src, cnt);
  else b_sort_lds_e<8>(src, cnt);
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

// Problems of at most kBSmallN keys: load all composites, sort, write.
template <int DT>
__device__ inline void b_small(const BatchDesc& d, BatchSmem& sm) {
  const uint32_t n = (uint32_t)d.n;
  const bool vec = (reinterpret_cast<uintptr_t>(d.keys) & 15u) == 0;
  for (uint32_t i = threadIdx.x * 4; i < n; i += kBT * 4) {
    uint32_t v[4];
    b_load4(d.keys, i, n, vec, v);
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (i + c < n) sm.surv[i + c] = comp(enc<DT>(v[c]), i + c);
  }
  __syncthreads();
  b_sort_write<DT>(sm.surv, n, d.k, d.out_vals, d.out_idx, d.out_kth);
}

// Block-level MSD radix select over the problem's 64-bit composites: each
// pass histograms one digit of the elements in the current class (those
// matching the digits chosen so far) and picks the bin holding rank r.  As
// soon as the elements ranked above the class plus the class itself fit the
// LDS, they are compacted, sorted and the first k written: two passes over
// the keys for typical inputs, at most seven for massive ties.
template <int DT>
__device__ inline void b_radix(const BatchDesc& d, BatchSmem& sm) {
  const uint32_t n = (uint32_t)d.n, k = d.k;
  const bool vec = (reinterpret_cast<uintptr_t>(d.keys) & 15u) == 0;
  const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
  uint64_t prefix = 0, mask = 0;
  uint32_t r = k, above = 0;
  for (int p = 0; p < kPasses; ++p) {
    for (int i = threadIdx.x; i < kBins; i += kBT) sm.hist[i] = 0;
    __syncthreads();
    const int sh = pass_shift(p);
    const uint32_t dm = (1u << pass_bits(p)) - 1;
    for (uint32_t base = wave * kBStep; base < n; base += kBWaves * kBStep) {
      uint32_t v[kBU][4];
#pragma unroll
      for (int j = 0; j < kBU; ++j) b_load4(d.keys, base + j * 256 + lane * 4, n, vec, v[j]);
#pragma unroll
      for (int j = 0; j < kBU; ++j)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const uint32_t i = base + j * 256 + lane * 4 + c;
          const uint64_t x = comp(enc<DT>(v[j][c]), i);
          if (i < n && (x & mask) == prefix) atomicAdd(&sm.hist[(uint32_t)(x >> sh) & dm], 1u);
        }
    }
    __syncthreads();
    bb_bucket(sm.hist, r, sm);
    prefix |= (uint64_t)sm.out[0] << sh;
    mask |= (uint64_t)dm << sh;
    above += r - sm.out[1];
    r = sm.out[1];
    if (above + sm.out[3] <= kBSurv) break;  // always true after the last pass (class of one)
  }
  // every element ranked above the class, and the class: (x & mask) >= prefix
  if (threadIdx.x == 0) sm.nsurv = 0;
  __syncthreads();
  for (uint32_t base = wave * kBStep; base < n; base += kBWaves * kBStep) {
    uint32_t v[kBU][4];
#pragma unroll
    for (int j = 0; j < kBU; ++j) b_load4(d.keys, base + j * 256 + lane * 4, n, vec, v[j]);
#pragma unroll
    for (int j = 0; j < kBU; ++j)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const uint32_t i = base + j * 256 + lane * 4 + c;
        const uint64_t x = comp(enc<DT>(v[j][c]), i);
        if (i < n && (x & mask) >= prefix) {
          const uint32_t slot = atomicAdd(&sm.nsurv, 1u);
          if (slot < kBSurv) sm.surv[slot] = x;
        }
      }
  }
  __syncthreads();
  const uint32_t ns = sm.nsurv < kBSurv ? sm.nsurv : kBSurv;
  b_sort_write<DT>(sm.surv, ns, k, d.out_vals, d.out_idx, d.out_kth);
}

// Delegate vector for subranges of at least 256 keys: waves stream the problem
// in steps of kBStep keys with kBU 1 KiB loads in flight; each 256-key block
// lies inside one subrange, whose delegate takes the block's maximum by an LDS
// atomic max (D starts at 0, below every composite of a real element).
template <int DT>
__device__ inline void b_delegates_wide(const BatchDesc& d, BatchSmem& sm, bool vec) {
  const uint32_t n = (uint32_t)d.n, alpha = d.alpha, L = 1u << alpha;
  const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
  for (uint32_t base = wave * kBStep; base < n; base += kBWaves * kBStep) {
    uint32_t v[kBU][4];
#pragma unroll
    for (int j = 0; j < kBU; ++j) b_load4(d.keys, base + j * 256 + lane * 4, n, vec, v[j]);
    if (L >= kBStep) {
      uint64_t m = 0;
#pragma unroll
      for (int j = 0; j < kBU; ++j)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const uint32_t p = base + j * 256 + lane * 4 + c;
          const uint64_t x = comp(enc<DT>(v[j][c]), p);
          if (p < n && x > m) m = x;
        }
      m = wave_max64(m);
      if (lane == 0) atomicMax((unsigned long long*)&sm.D[base >> alpha], (unsigned long long)m);
    } else {
#pragma unroll
      for (int j = 0; j < kBU; ++j) {
        uint64_t m = 0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const uint32_t p = base + j * 256 + lane * 4 + c;
          const uint64_t x = comp(enc<DT>(v[j][c]), p);
          if (p < n && x > m) m = x;
        }
        m = wave_max64(m);
        if (lane == 0 && base + j * 256 < n)
          atomicMax((unsigned long long*)&sm.D[(base + j * 256) >> alpha], (unsigned long long)m);
      }
    }
  }
}

// Delegate vector for subranges of 4..128 keys: each 256-key wave-load holds
// whole subranges, 2^(alpha-2) lanes each; a segmented butterfly gives each
// subrange's maximum to its first lane.
template <int DT>
__device__ inline void b_delegates_narrow(const BatchDesc& d, BatchSmem& sm, bool vec) {
  const uint32_t n = (uint32_t)d.n, alpha = d.alpha;
  const uint32_t G = 1u << (alpha - 2);  // lanes per subrange
  const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
  for (uint32_t base = wave * kBStep; base < n; base += kBWaves * kBStep) {
    uint32_t v[kBU][4];
#pragma unroll
    for (int j = 0; j < kBU; ++j) b_load4(d.keys, base + j * 256 + lane * 4, n, vec, v[j]);
#pragma unroll
    for (int j = 0; j < kBU; ++j) {
      const uint32_t p = base + j * 256 + lane * 4;
      uint64_t m = 0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const uint64_t x = comp(enc<DT>(v[j][c]), p + c);
        if (p + c < n && x > m) m = x;
      }
      for (uint32_t o = 1; o < G; o <<= 1) {
        const uint64_t y = shfl_xor64(m, (int)o);
        m = y > m ? y : m;
      }
      if ((lane & (G - 1)) == 0 && p < n) sm.D[p >> alpha] = m;
    }
  }
}

// Survivors: every element ranked >= t in the subranges of the k-1 delegates
// above t (sm.D[0..k-2], sorted), read as one virtual vector of
// (k-1) * 2^alpha keys in 16-byte pieces (a piece never crosses a subrange).
template <int DT>
__device__ inline void b_survivors(const BatchDesc& d, BatchSmem& sm, bool vec, uint64_t t) {
  const uint32_t n = (uint32_t)d.n, k = d.k, alpha = d.alpha, L = 1u << alpha;
  const uint32_t total = (k - 1) << alpha;
  const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
  for (uint32_t base = wave * kBStep; base < total; base += kBWaves * kBStep) {
    uint32_t v[kBU][4], pb[kBU];
#pragma unroll
    for (int j = 0; j < kBU; ++j) {
      const uint32_t e = base + j * 256 + lane * 4;
      pb[j] = 0xFFFFFFFFu;
      if (e < total) {
        const uint32_t s = comp_pos(sm.D[e >> alpha]) >> alpha;
        pb[j] = (s << alpha) + (e & (L - 1));
        b_load4(d.keys, pb[j], n, vec, v[j]);
      }
    }
#pragma unroll
    for (int j = 0; j < kBU; ++j) {
      if (pb[j] == 0xFFFFFFFFu) continue;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const uint32_t p = pb[j] + c;
        const uint64_t x = comp(enc<DT>(v[j][c]), p);
        if (p < n && x >= t) {
          const uint32_t slot = atomicAdd(&sm.nsurv, 1u);
          if (slot < kBSurv) sm.surv[slot] = x;
        }
      }
    }
  }
}

// The delegate method for one problem; false if the survivors overflow LDS
// (nothing has been written then).
template <int DT>
__device__ inline bool b_delegate(const BatchDesc& d, BatchSmem& sm) {
  const uint32_t n = (uint32_t)d.n, k = d.k, alpha = d.alpha;
  const uint32_t S = (n + (1u << alpha) - 1) >> alpha;
  const bool vec = (reinterpret_cast<uintptr_t>(d.keys) & 15u) == 0;
  if (alpha >= 8) {
    for (uint32_t i = threadIdx.x; i < S; i += kBT) sm.D[i] = 0;
    __syncthreads();
    b_delegates_wide<DT>(d, sm, vec);
  } else {
    b_delegates_narrow<DT>(d, sm, vec);
  }
  __syncthreads();
  b_sort_lds(sm.D, S);  // descending: D[k-1] is t, D[0..k-2] the delegates above it
  if (threadIdx.x == 0) sm.nsurv = 1;
  const uint64_t t = sm.D[k - 1];
  if (threadIdx.x == 0) sm.surv[0] = t;  // t itself: its subrange is not re-read
  __syncthreads();
  b_survivors<DT>(d, sm, vec, t);
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
__global__ __launch_bounds__(kBT) __attribute__((amdgpu_waves_per_eu(4))) void k_batched(
    const BatchDesc* __restrict__ descs, uint32_t count, uint32_t* counter) {
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

// One problem, descriptor by value: the single-problem path for small inputs.
__global__ __launch_bounds__(kBT) __attribute__((amdgpu_waves_per_eu(4))) void k_one(BatchDesc d) {
  __shared__ BatchSmem sm;
  if (d.dtype == DT_F32) b_problem<DT_F32>(d, sm);
  else b_problem<DT_U32>(d, sm);
}

}  // namespace drtopk
