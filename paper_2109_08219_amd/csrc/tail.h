// Everything after the delegate pass, in one launch.
//
// Phases:
//   W   compact the delegates at or above the cut found by the delegate pass
//       (a superset of those ranked >= t, Rule 2's threshold);
//   T   t = the kD-th largest of W: one block sorts W in LDS when W is small,
//       else a multi-block MSD radix select (one phase per digit) followed by
//       Rule 3 over W;
//   S   re-read the qualifying subranges as one virtual concatenated vector,
//       keeping elements ranked >= t;
//   F   the k-th survivor and the output: one block sorts the survivors in
//       LDS when they are few, else radix select + exact compaction (the sort
//       of a large k follows as separate kernels).
// Work inside a phase is claimed chunk by chunk from an atomic counter; a
// phase is complete when the chunks claimed have been reported done, and the
// block that reports the last chunk finalises it and raises the phase's ready
// flag.  A waiting block therefore only ever waits for chunks that running
// blocks hold, so the kernel needs no co-residency guarantee (plain launch,
// safe beside kernels on other streams).  Waits are bounded and flag
// ctl->err if exceeded.  Data crossing blocks goes through atomics and
// coherent (sc1) stores/loads only.
#pragma once

#include <type_traits>

#include "kernels.h"

namespace drtopk {

constexpr int kTailThreads = 512;
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
constexpr uint32_t kSpinLimit = 1u << 20;  // ~1 s of polling, then give up and flag

struct TailArgs {
  const uint32_t* keys;
  uint64_t n;
  int alpha;
  uint64_t S;
  uint64_t nd;
  uint32_t k, kD;
  uint32_t slack;  // survivor buffers hold floor((kD+slack)/beta)*2^alpha + kD + slack entries
  int all, kth_only, stop_after_scan, big_sort;
  const uint32_t* dkey;
  const uint32_t* didx;
  uint32_t *Q, *ckey, *cidx, *skey, *sidx, *okey, *oidx;
  uint32_t cap_s;
  uint32_t *out_vals, *out_idx, *out_kth;
  uint64_t *A, *B;  // big_sort: the merge sort's two buffers of M composites
  uint64_t M;       // k rounded up to a power-of-two multiple of kSortTile
  Ctl* ctl;
};

// Bin holding the rank-th largest in a 2048-bin global histogram (coherent
// loads), blockDim.x == kTailThreads: s_out = {bin, rank in bin, found, count}.
__device__ inline void tail_bucket(const uint32_t* gh, uint32_t rank, uint32_t* s_scan, uint32_t* s_out) {
  constexpr int PER = kBins / kTailThreads;  // 4
  const int t = threadIdx.x;
  uint32_t c[PER], sum = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    c[j] = ld_coh(&gh[kBins - 1 - PER * t - j]);
    sum += c[j];
  }
  s_scan[t] = sum;
  if (t == 0) { s_out[0] = 0; s_out[1] = 0; s_out[2] = 0; s_out[3] = 0; }
  __syncthreads();
  for (int off = 1; off < kTailThreads; off <<= 1) {
    const uint32_t x = t >= off ? s_scan[t - off] : 0u;
    __syncthreads();
    s_scan[t] += x;
    __syncthreads();
  }
  const uint32_t incl = s_scan[t], excl = incl - sum;
  if (excl < rank && rank <= incl) {
    uint32_t cum = excl;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      if (cum + c[j] >= rank) {
        s_out[0] = kBins - 1 - PER * t - j;
        s_out[1] = rank - cum;
        s_out[2] = 1;
        s_out[3] = c[j];
        break;
      }
      cum += c[j];
    }
  }
  __syncthreads();
}

// LDS bitonic sort, descending, of P (power of two) composites.
__device__ inline void lds_sort_desc(uint64_t* buf, uint32_t P) {
  for (uint32_t size = 2; size <= P; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t i = threadIdx.x; i < (P >> 1); i += blockDim.x) {
        const uint32_t lo = 2 * i - (i & (stride - 1));
        const uint32_t hi = lo + stride;
        const bool desc = (lo & size) == 0;
        const uint64_t a = buf[lo], b = buf[hi];
        if ((a < b) == desc) { buf[lo] = b; buf[hi] = a; }
      }
      __syncthreads();
    }
  }
}

// Whole wave active.  Each lane appends the elements c with pred[c]: one
// LDS reservation for the wave's four element slots.
template <int CAP>
__device__ __forceinline__ void stage_push4(Stage<CAP>& S, const bool (&pred)[4], const uint32_t (&key)[4],
                                            const uint32_t (&idx)[4]) {
  uint64_t m[4];
  uint32_t pre[4], tot = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    m[c] = __ballot(pred[c]);
    pre[c] = tot;
    tot += (uint32_t)__popcll(m[c]);
  }
  if (!tot) return;
  uint32_t base = 0;
  if (lane_id() == 0) base = atomicAdd(&S.n, tot);
  base = (uint32_t)__shfl((int)base, 0);
#pragma unroll
  for (int c = 0; c < 4; ++c)
    if (pred[c]) {
      const uint32_t off = base + pre[c] + mbcnt(m[c]);
      S.key[off] = key[c];
      S.idx[off] = idx[c];
    }
}

template <int CAP>
__device__ __forceinline__ void stage_flush_coh(Stage<CAP>& S, uint32_t* gcount, uint32_t gcap, uint32_t* gkey,
                                                uint32_t* gidx, Ctl* ctl, bool force, uint32_t margin) {
  __syncthreads();
  const uint32_t n = S.n;
  const bool doit = n != 0 && (force || n + margin > (uint32_t)CAP);
  __syncthreads();
  if (!doit) return;
  if (threadIdx.x == 0) S.base = atomicAdd(gcount, n);
  __syncthreads();
  const uint32_t base = S.base;
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
    if (base + i < gcap) {
      st_coh(&gkey[base + i], S.key[i]);
      if (gidx) st_coh(&gidx[base + i], S.idx[i]);
    } else {
      flag_err(ctl, ERR_CAP);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) S.n = 0;
  __syncthreads();
}

// Two stages checked behind one barrier pair; each is flushed only when
// fewer than its margin of slots are left.  Block-uniform.
template <int CA, int CB>
__device__ __forceinline__ void stage_flush2_coh(Stage<CA>& A, uint32_t* acount, uint32_t acap, uint32_t* akey,
                                                 uint32_t amargin, Stage<CB>& B, uint32_t* bcount, uint32_t bcap,
                                                 uint32_t* bkey, uint32_t* bidx, uint32_t bmargin, Ctl* ctl) {
  __syncthreads();
  const uint32_t na = A.n, nb = B.n;
  __syncthreads();
  if (na + amargin > (uint32_t)CA) stage_flush_coh(A, acount, acap, akey, nullptr, ctl, true, 0);
  if (nb + bmargin > (uint32_t)CB) stage_flush_coh(B, bcount, bcap, bkey, bidx, ctl, true, 0);
}

// Bins of the bucket-rank sort (top 12 bits of x - min) and the fullest bin
// it takes before it leaves the sort to the bitonic network.
constexpr int kRankBins = 4096;
constexpr uint32_t kRankMaxBin = 64;

// Shared memory of the tail kernel, reused phase by phase.
struct TailSmem {
  union {
    uint64_t sortbuf[kSmallCap];  // 64 KiB: the one-block LDS sorts
    struct {
      uint32_t hist[kBins];
      Stage<8 * kTailThreads> sq;   // a whole Q claim's queued subranges
      Stage<16 * kTailThreads> sc;  // a whole Q claim's delegates at beta <= 2
    } st;
  } u;
  uint32_t scan[kTailThreads];
  uint32_t rbins[kRankBins + 1];  // bucket-rank sort: bin counts, then bin starts
  uint64_t rred[2 * (kTailThreads / 64)];
  uint32_t rwave[2 * (kTailThreads / 64)];
  uint32_t out[4];
  uint32_t item;
  int last;
};

// ---- phase protocol -------------------------------------------------------

// Next chunk of phase `ph` for this block (block-uniform result); >= limit
// when the phase has no chunk left.  A coherent read first keeps blocks that
// arrive after the chunks are gone off the contended counter.
__device__ __forceinline__ uint32_t claim(Phase* ph, uint32_t limit, TailSmem& sm) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t cur = ld_coh(&ph->claim);
    sm.item = cur < limit ? atomicAdd(&ph->claim, 1u) : cur;
  }
  __syncthreads();
  return sm.item;
}

// Reports the `mine` chunks this block completed; true in exactly one block,
// the one whose report completes the phase.  All of this block's global
// writes and atomics for those chunks have completed before the report.
__device__ __forceinline__ bool report(Phase* ph, uint32_t mine, uint32_t nchunks, TailSmem& sm) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) sm.last = mine ? (atomicAdd(&ph->done, mine) + mine == nchunks) : 0;
  __syncthreads();
  return sm.last != 0;
}

__device__ __forceinline__ void raise_ready(Phase* ph) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) st_coh(&ph->ready, 1u);
}

// Completion time of phase i (device real-time clock, 100 MHz), for profiling.
__device__ __forceinline__ void stamp(Ctl* ctl, int i) {
  if (threadIdx.x == 0) ctl->tstamp[i] = __builtin_amdgcn_s_memrealtime();
}

__device__ __forceinline__ void wait_ready(Phase* ph, Ctl* ctl) {
  if (threadIdx.x == 0) {
    uint32_t spins = 0;
    while (ld_coh(&ph->ready) == 0u) {
      __builtin_amdgcn_s_sleep(2);
      if (++spins > kSpinLimit) {
        flag_err(ctl, ERR_WAIT);
        break;
      }
    }
  }
  __syncthreads();
}

__device__ __forceinline__ void pub64(uint32_t* p, uint64_t v) {
  st_coh(p, (uint32_t)v);
  st_coh(p + 1, (uint32_t)(v >> 32));
}
__device__ __forceinline__ uint64_t get64(const uint32_t* p) {
  return ((uint64_t)ld_coh(p + 1) << 32) | ld_coh(p);
}

// ---- multi-block radix select over a buffer written earlier in this kernel --
// Phases ph[0..kPasses): one per digit.  Returns the rank-th largest composite
// of (key[i], idx[i]), i < count, identically in every block.
//   key_known: the sought entry's key is key0 and `rank` counts from the
//     largest entry with that key; the three key digits are skipped.
//   bound: a lower bound suffices: once the class holding the rank has at
//     most kBoundTol members below the sought entry, its prefix with the
//     remaining bits zero is returned; the entries ranked at or above it are
//     those at or above the sought entry plus at most kBoundTol more.
constexpr uint32_t kSelChunk = kTailThreads * 8;
constexpr uint32_t kBoundTol = 64;

__device__ inline uint64_t tail_select(const uint32_t* key, const uint32_t* idx, uint32_t count, uint32_t rank,
                                       uint32_t (*hist)[kBins], Phase* ph, uint32_t* pubsel, Ctl* ctl,
                                       TailSmem& sm, bool key_known = false, uint32_t key0 = 0,
                                       bool bound = false) {
  uint64_t prefix = key_known ? (uint64_t)key0 << 32 : 0ull;
  uint64_t mask = key_known ? 0xFFFFFFFF00000000ull : 0ull;
  uint32_t r = rank;
  const uint32_t nchunks = (count + kSelChunk - 1) / kSelChunk;
  if (nchunks == 0 || rank == 0 || rank > count) {  // inconsistent input: flag, never wait
    if (blockIdx.x == 0 && threadIdx.x == 0) flag_err(ctl, ERR_SELECT);
    return 0;
  }
  for (int p = key_known ? 3 : 0; p < kPasses; ++p) {
    for (int i = threadIdx.x; i < kBins; i += kTailThreads) sm.u.st.hist[i] = 0;
    const int sh = pass_shift(p);
    const uint32_t dm = (1u << pass_bits(p)) - 1;
    const uint32_t kmask = (uint32_t)(mask >> 32), kpref = (uint32_t)(prefix >> 32);
    const uint32_t imask = (uint32_t)mask, ipref = (uint32_t)prefix;
    uint32_t mine = 0;
    for (;;) {
      const uint32_t c = claim(&ph[p], nchunks, sm);
      if (c >= nchunks) break;
      ++mine;
      // every load of the claim first (positions only once they are digits), then the tests
      constexpr int R = kSelChunk / kTailThreads;
      uint32_t kv[R], iv[R];
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const uint32_t i = c * kSelChunk + (uint32_t)j * kTailThreads + threadIdx.x;
        kv[j] = i < count ? ld_coh(&key[i]) : 0u;
        iv[j] = i < count && p >= 3 ? ~ld_coh(&idx[i]) : 0u;
      }
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const uint32_t i = c * kSelChunk + (uint32_t)j * kTailThreads + threadIdx.x;
        if (i >= count || (kv[j] & kmask) != kpref) continue;
        if (p >= 3 && (iv[j] & imask) != ipref) continue;
        const uint64_t x = ((uint64_t)kv[j] << 32) | (p >= 3 ? iv[j] : 0u);
        atomicAdd(&sm.u.st.hist[(uint32_t)(x >> sh) & dm], 1u);
      }
    }
    __syncthreads();
    if (mine)
      for (int i = threadIdx.x; i < kBins; i += kTailThreads) {
        const uint32_t v = sm.u.st.hist[i];
        if (v) atomicAdd(&hist[p][i], v);
      }
    if (report(&ph[p], mine, nchunks, sm)) {
      tail_bucket(hist[p], r, sm.scan, sm.out);
      if (threadIdx.x == 0) {
        if (!sm.out[2]) flag_err(ctl, ERR_SELECT);
        pub64(pubsel, prefix | ((uint64_t)sm.out[0] << sh));
        st_coh(pubsel + 2, sm.out[1]);
        st_coh(pubsel + 3, sm.out[3]);
      }
      if (threadIdx.x == 0) ctl->tstamp[(ph - ctl->ph) + p] = __builtin_amdgcn_s_memrealtime();
      raise_ready(&ph[p]);
    }
    wait_ready(&ph[p], ctl);
    prefix = get64(pubsel);
    mask |= (uint64_t)dm << sh;
    r = ld_coh(pubsel + 2);
    const uint32_t members = ld_coh(pubsel + 3);
    __syncthreads();
    if (bound && members - r <= kBoundTol) break;  // uniform: every block read the same words
  }
  return prefix;
}

// ---- block sort ----------------------------------------------------------------
// Bitonic sort (descending) of P = E * kTailThreads composites held in
// registers, element g = threadIdx.x * E + e.  Compare-exchange partners at
// distance j < E are in the same thread (registers), E <= j < 64 E in another
// lane of the same wave (lane shuffles), and only j >= 64 E go through LDS
// with barriers.  Each element computes its own new value from its partner's.

__device__ __forceinline__ uint64_t ce_pick(uint64_t mine, uint64_t other, bool lower, bool desc_block) {
  // `lower`: this element has the lower index of the pair.  In a descending
  // block the lower index keeps the larger value.
  const bool keep_max = lower == desc_block;
  const bool mine_gt = mine > other;
  return keep_max ? (mine_gt ? mine : other) : (mine_gt ? other : mine);
}

// The value of lane (lane ^ M), M a compile-time power of two below 64:
// DPP quad permutes for 1 and 2, a DPP row rotation by 8 (within 16-lane
// rows that is xor 8), ds_swizzle's bit-mask mode (xor inside 32-lane
// halves, no address operand) for 4 and 16, ds_bpermute for 32.
template <int M>
__device__ __forceinline__ uint32_t lane_xor32(uint32_t v) {
  if constexpr (M == 1) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);
  else if constexpr (M == 2) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);
  else if constexpr (M == 4) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x101F);
  else if constexpr (M == 8) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, false);
  else if constexpr (M == 16) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x401F);
  else return (uint32_t)__shfl_xor((int)v, M);
}
template <int M>
__device__ __forceinline__ uint64_t lane_xor64(uint64_t v) {
  return ((uint64_t)lane_xor32<M>((uint32_t)(v >> 32)) << 32) | lane_xor32<M>((uint32_t)v);
}

// One compare-exchange stage of block size S and partner distance J, all
// compile-time, so the element array stays in registers.
template <int E, uint32_t S, uint32_t J>
__device__ __forceinline__ void bs_stage(uint64_t (&v)[E], uint64_t* lds) {
  if constexpr (J < (uint32_t)E) {
    const uint32_t base = threadIdx.x * E;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if ((e & J) == 0) {
        const bool desc_block = ((base + e) & S) == 0;  // (e, e|J) lie in one block of size S
        const uint64_t a = v[e], b = v[e | J];
        const bool a_gt = a > b;
        const uint64_t hi = a_gt ? a : b, lo = a_gt ? b : a;
        v[e] = desc_block ? hi : lo;
        v[e | J] = desc_block ? lo : hi;
      }
    }
  } else if constexpr (J < 64u * E) {
    constexpr uint32_t m = J / E;  // lane distance
    const bool lower = (lane_id() & m) == 0;
#pragma unroll
    for (int e = 0; e < E; ++e)
      v[e] = ce_pick(v[e], lane_xor64<(int)m>(v[e]), lower, ((threadIdx.x * E + e) & S) == 0);
  } else {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) lds[threadIdx.x * E + e] = v[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const uint32_t g = threadIdx.x * E + e;
      v[e] = ce_pick(v[e], lds[g ^ J], (g & J) == 0, (g & S) == 0);
    }
  }
  if constexpr (J > 1) bs_stage<E, S, J / 2>(v, lds);
}

template <int E, uint32_t S, int NT>
__device__ __forceinline__ void bs_size(uint64_t (&v)[E], uint64_t* lds) {
  bs_stage<E, S, S / 2>(v, lds);
  if constexpr (S < (uint32_t)E * NT) bs_size<E, S * 2, NT>(v, lds);
}

// Sorts the E * NT composites held E per thread by a block of NT threads.
template <int E, int NT = kTailThreads>
__device__ __forceinline__ void block_bitonic(uint64_t (&v)[E], uint64_t* lds) {
  bs_size<E, 2, NT>(v, lds);
  __syncthreads();
}

// Sorts `count` (<= kSmallCap) composites read coherently from (key, idx) and
// writes the first `limit` of them as outputs first_slot, first_slot+1, ...
template <int DT, int E>
__device__ __noinline__ void sort_and_write_e(const uint32_t* key, const uint32_t* idx, uint32_t count, uint32_t first_slot,
                                        uint32_t limit, uint32_t k, uint32_t* out_vals, uint32_t* out_idx,
                                        uint32_t* out_kth, uint64_t* lds) {
  uint64_t v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint32_t g = threadIdx.x * E + e;
    v[e] = g < count ? comp(ld_coh(&key[g]), ld_coh(&idx[g])) : 0ull;
  }
  block_bitonic<E>(v, lds);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint32_t g = threadIdx.x * E + e;
    if (g < limit) write_out<DT>(v[e], first_slot + g, k, out_vals, out_idx, out_kth);
  }
}

// Bucket-rank sort of `count` (<= E * kTailThreads) distinct composites, read
// coherently from (key, idx), writing the first `limit` as outputs
// first_slot, first_slot+1, ...: no sorting network.  The composites are
// binned by the top 12 bits of their distance from the smallest (bin 0 holds
// the largest), counted in LDS, scattered bin by bin into `buf`, and each
// takes the slot (start of its bin) + (number of larger composites in its
// bin).  Work per element is its bin's size, so the sort gives up (false,
// nothing written) when the fullest bin holds more than kRankMaxBin -- keys
// crowded into a narrow range -- and the caller sorts by network instead.
template <int DT, int E>
__device__ __noinline__ bool rank_sort_write_e(const uint32_t* key, const uint32_t* idx, uint32_t count,
                                               uint32_t first_slot, uint32_t limit, uint32_t k, uint32_t* out_vals,
                                               uint32_t* out_idx, uint32_t* out_kth, uint64_t* buf, uint32_t* bins,
                                               uint64_t* red, uint32_t* wred) {
  constexpr int NT = kTailThreads, NW = NT / 64, PER = kRankBins / NT;
  const uint32_t t = threadIdx.x, lane = lane_id(), w = t >> 6;
  uint64_t v[E];
  uint64_t mx = 0, nmn = 0;  // largest composite, and the complement of the smallest
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint32_t g = e * NT + t;
    v[e] = g < count ? comp(ld_coh(&key[g]), ld_coh(&idx[g])) : 0ull;
    if (g < count) {
      mx = v[e] > mx ? v[e] : mx;
      nmn = ~v[e] > nmn ? ~v[e] : nmn;
    }
  }
#define DRTOPK_MAX2(M)                                     \
  {                                                        \
    const uint64_t a_ = lane_xor64<M>(mx), b_ = lane_xor64<M>(nmn); \
    mx = a_ > mx ? a_ : mx;                                \
    nmn = b_ > nmn ? b_ : nmn;                             \
  }
  DRTOPK_MAX2(1) DRTOPK_MAX2(2) DRTOPK_MAX2(4) DRTOPK_MAX2(8) DRTOPK_MAX2(16) DRTOPK_MAX2(32)
#undef DRTOPK_MAX2
  if (lane == 0) {
    red[w] = mx;
    red[NW + w] = nmn;
  }
  for (int i = t; i < kRankBins; i += NT) bins[i] = 0;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    mx = red[i] > mx ? red[i] : mx;
    nmn = red[NW + i] > nmn ? red[NW + i] : nmn;
  }
  const uint64_t lo = ~nmn;
  const uint32_t bits = bitlen64(mx - lo);
  const uint32_t sh = bits > 12u ? bits - 12u : 0u;
  uint32_t b[E], r[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint32_t g = e * NT + t;
    b[e] = (uint32_t)(kRankBins - 1) - (uint32_t)((v[e] - lo) >> sh);
    r[e] = g < count ? atomicAdd(&bins[b[e]], 1u) : 0u;
  }
  __syncthreads();
  // exclusive scan of the bin counts (PER consecutive bins per thread) and the fullest bin
  uint32_t c[PER], sum = 0, big = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    c[j] = bins[t * PER + j];
    sum += c[j];
    big = c[j] > big ? c[j] : big;
  }
  uint32_t inc = sum;
#pragma unroll
  for (uint32_t d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(inc, d);
    if (lane >= d) inc += y;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const uint32_t y = __shfl_xor(big, o);
    big = y > big ? y : big;
  }
  if (lane == 63) wred[w] = inc;
  if (lane == 0) wred[NW + w] = big;
  __syncthreads();
  uint32_t off = inc - sum;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    if ((uint32_t)i < w) off += wred[i];
    big = wred[NW + i] > big ? wred[NW + i] : big;
  }
  if (big > kRankMaxBin) return false;  // block-uniform
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    bins[t * PER + j] = off;
    off += c[j];
  }
  if (t == NT - 1) bins[kRankBins] = off;
  __syncthreads();
#pragma unroll
  for (int e = 0; e < E; ++e)
    if (e * NT + t < count) buf[bins[b[e]] + r[e]] = v[e];
  __syncthreads();
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (e * NT + t >= count) continue;
    const uint32_t st = bins[b[e]], en = bins[b[e] + 1];
    uint32_t slot = st;
    for (uint32_t j = st; j < en; ++j) slot += buf[j] > v[e] ? 1u : 0u;
    if (slot < limit) write_out<DT>(v[e], first_slot + slot, k, out_vals, out_idx, out_kth);
  }
  __syncthreads();  // the caller reuses the LDS
  return true;
}

struct RankLds {
  uint32_t* bins;
  uint64_t* red;
  uint32_t* wred;
};

template <int DT>
__device__ inline void sort_and_write(const uint32_t* key, const uint32_t* idx, uint32_t count, uint32_t first_slot,
                                      uint32_t limit, uint32_t k, uint32_t* out_vals, uint32_t* out_idx,
                                      uint32_t* out_kth, uint64_t* lds, const RankLds& rl) {
  if (count > 1u * kTailThreads) {
    bool done;
    if (count <= 2u * kTailThreads)
      done = rank_sort_write_e<DT, 2>(key, idx, count, first_slot, limit, k, out_vals, out_idx, out_kth, lds, rl.bins,
                                      rl.red, rl.wred);
    else if (count <= 4u * kTailThreads)
      done = rank_sort_write_e<DT, 4>(key, idx, count, first_slot, limit, k, out_vals, out_idx, out_kth, lds, rl.bins,
                                      rl.red, rl.wred);
    else if (count <= 8u * kTailThreads)
      done = rank_sort_write_e<DT, 8>(key, idx, count, first_slot, limit, k, out_vals, out_idx, out_kth, lds, rl.bins,
                                      rl.red, rl.wred);
    else
      done = rank_sort_write_e<DT, 16>(key, idx, count, first_slot, limit, k, out_vals, out_idx, out_kth, lds,
                                       rl.bins, rl.red, rl.wred);
    if (done) return;
  }
  if (count <= 1u * kTailThreads)
    sort_and_write_e<DT, 1>(key, idx, count, first_slot, limit, k, out_vals, out_idx, out_kth, lds);
  else if (count <= 2u * kTailThreads)
    sort_and_write_e<DT, 2>(key, idx, count, first_slot, limit, k, out_vals, out_idx, out_kth, lds);
  else if (count <= 4u * kTailThreads)
    sort_and_write_e<DT, 4>(key, idx, count, first_slot, limit, k, out_vals, out_idx, out_kth, lds);
  else if (count <= 8u * kTailThreads)
    sort_and_write_e<DT, 8>(key, idx, count, first_slot, limit, k, out_vals, out_idx, out_kth, lds);
  else
    sort_and_write_e<DT, 16>(key, idx, count, first_slot, limit, k, out_vals, out_idx, out_kth, lds);
}

// Output buckets of the survivors.  Every survivor ranks at or above the
// threshold T and at or below the largest element, so the map is fixed as
// soon as T is: bucket(x) = 2047 - (top 11 significant bits of x - T over
// the range up to the largest element), bucket 0 holding the largest.  Q and
// S count the survivors they write into it (LDS, flushed per block before
// the block reports its chunks), so no pass over the survivors is needed to
// find the bucket that holds output slot k-1.
struct BucketMap {
  uint64_t lo;
  uint32_t sh;
  __device__ __forceinline__ uint32_t operator()(uint64_t x) const { return 2047u - (uint32_t)((x - lo) >> sh); }
};

// Whole wave active: every lane with `pred` adds one to h[bin].  When all of
// them share one bin (sorted or tied inputs, where per-lane atomics on one
// address would serialise) the wave adds its count with a single atomic.
__device__ __forceinline__ void hist_add_wave(uint32_t* h, bool pred, uint32_t bin) {
  const uint64_t m = __ballot(pred);
  if (!m) return;
  const int leader = __ffsll((unsigned long long)m) - 1;
  const uint32_t b0 = (uint32_t)__shfl((int)bin, leader);
  if (__all(!pred || bin == b0)) {
    if ((int)lane_id() == leader) atomicAdd(&h[b0], (uint32_t)__popcll(m));
  } else if (pred) {
    atomicAdd(&h[bin], 1u);
  }
}

// The four elements of every lane of a wave at once (whole wave active).
// While all survivors of the wave fall into one bucket (sorted or tied
// inputs, and the dense stretches of others) the wave only adds their count
// to a pending (bucket, count) pair, wave-uniform, which goes to h[] in one
// atomic when the bucket changes and at hist_pending_flush; otherwise one
// atomic per survivor.  Same-address LDS atomics from every wave of a block
// otherwise serialise.
__device__ __forceinline__ void hist_add_wave4(uint32_t* h, const bool (&take)[4], const uint32_t (&bin)[4],
                                               uint32_t& pbin, uint32_t& pcnt) {
  uint64_t m[4];
  uint32_t tot = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    m[c] = __ballot(take[c]);
    tot += (uint32_t)__popcll(m[c]);
  }
  if (!tot) return;
  // the bucket of the first survivor (element slots in order, then lanes)
  const int c0 = m[0] ? 0 : m[1] ? 1 : m[2] ? 2 : 3;
  const uint32_t bc = c0 == 0 ? bin[0] : c0 == 1 ? bin[1] : c0 == 2 ? bin[2] : bin[3];
  const uint32_t b0 = (uint32_t)__shfl((int)bc, __ffsll((unsigned long long)m[c0]) - 1);
  bool same = true;
#pragma unroll
  for (int c = 0; c < 4; ++c) same = same && (!take[c] || bin[c] == b0);
  if (__all(same)) {
    if (b0 != pbin) {
      if (pcnt && lane_id() == 0) atomicAdd(&h[pbin], pcnt);
      pbin = b0;
      pcnt = 0;
    }
    pcnt += tot;
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (take[c]) atomicAdd(&h[bin[c]], 1u);
  }
}
__device__ __forceinline__ void hist_pending_flush(uint32_t* h, uint32_t& pbin, uint32_t& pcnt) {
  if (pcnt && lane_id() == 0) atomicAdd(&h[pbin], pcnt);
  pcnt = 0;
}

// Adds the block's LDS bucket counts to the global counts and clears them.
// Block-uniform.
__device__ __forceinline__ void hist_flush(uint32_t* h, uint32_t* g) {
  __syncthreads();
  for (int i = threadIdx.x; i < kBins; i += kTailThreads) {
    const uint32_t v = h[i];
    if (v) {
      atomicAdd(&g[i], v);
      h[i] = 0;
    }
  }
  __syncthreads();
}

// One block: sort survivors (<= kSmallCap) and write the first k.
template <int DT>
__device__ inline void small_output(const TailArgs& a, uint32_t nc, TailSmem& sm) {
  sort_and_write<DT>(a.ckey, a.cidx, nc, 0, a.k, a.k, a.kth_only ? nullptr : a.out_vals,
                     a.kth_only ? nullptr : a.out_idx, a.out_kth, sm.u.sortbuf, RankLds{sm.rbins, sm.rred, sm.rwave});
}

enum { PH_H = 0, PH_Q = 1, PH_S = 2, PH_F1 = 3, PH_B1 = 4, PH_B2 = 5, PH_B3 = 6, PH_FSEL = 7, PH_FC = 13, PH_FS = 14,
       PH_DSEL = 15 };
constexpr uint32_t kWChunk = kTailThreads * 8;
constexpr uint32_t kSChunk = kTailThreads * 4 * 16;
constexpr uint32_t kGroup = 2048;  // output positions per sort group (a group holds < 2 kGroup)

// One S-phase claim of STEPS x (kTailThreads x 4) elements of the virtual
// concatenated vector, 16-byte aligned keys and subranges of at least 4:
// every queue lookup first, then every key load, then the tests.
template <int DT, int STEPS>
__device__ __forceinline__ void s_claim_vec(const TailArgs& a, uint64_t first, uint64_t total, uint64_t T,
                                            TailSmem& sm, const BucketMap& bm, uint32_t* bh, Ctl* ctl) {
  const uint64_t lmask = (1ull << a.alpha) - 1;
  uint64_t pp[STEPS];
#pragma unroll
  for (int jj = 0; jj < STEPS; ++jj) {
    const uint64_t e = first + (uint64_t)jj * kTailThreads * 4 + threadIdx.x * 4;
    pp[jj] = e < total ? ((uint64_t)ld_coh(&a.Q[e >> a.alpha]) << a.alpha) + (e & lmask) : a.n;
  }
  bool full = true;
#pragma unroll
  for (int jj = 0; jj < STEPS; ++jj) full = full && pp[jj] + 4 <= a.n;
  uint32_t vv[STEPS][4];
  if (__all(full)) {
#pragma unroll
    for (int jj = 0; jj < STEPS; ++jj) load4<DT, true>(a.keys, pp[jj], vv[jj]);
  } else {
#pragma unroll
    for (int jj = 0; jj < STEPS; ++jj)
#pragma unroll
      for (int c = 0; c < 4; ++c) vv[jj][c] = pp[jj] + c < a.n ? a.keys[pp[jj] + c] : 0u;
  }
  uint32_t pbin = 0xFFFFFFFFu, pcnt = 0;
#pragma unroll
  for (int jj = 0; jj < STEPS; ++jj) {
    bool take[4];
    uint32_t kk[4], ii[4], bin[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const uint64_t pos = pp[jj] + c;
      kk[c] = enc<DT>(vv[jj][c]);
      ii[c] = (uint32_t)pos;
      const uint64_t cc = comp(kk[c], ii[c]);
      take[c] = pos < a.n && cc >= T;
      bin[c] = take[c] ? bm(cc) : 0u;
    }
    hist_add_wave4(bh, take, bin, pbin, pcnt);
    stage_push4(sm.u.st.sc, take, kk, ii);
    stage_flush_coh(sm.u.st.sc, &ctl->nc, ctl->cap_c, a.ckey, a.cidx, ctl, false, kTailThreads * 4);
  }
  hist_pending_flush(bh, pbin, pcnt);
}

// One B2 claim: the survivors [first, first + R x kTailThreads) (below nc)
// all loaded first, then scattered in batches of 8 per thread into their
// sort groups (group g = gt[bucket], LDS): counts and each element's rank in
// its group from an LDS histogram, one global reservation per nonzero group,
// then the stores (ctl->bcur serves as the groups' cursors).  A group's range
// ends up holding its buckets' elements in no particular order, which its
// sort in B3 does not need.
template <int R>
__device__ __forceinline__ void b2_claim(const TailArgs& a, uint32_t first, uint32_t nc, uint32_t bstar,
                                         const BucketMap& bm, const uint32_t* gt, TailSmem& sm, Ctl* ctl) {
  constexpr int kPer = 8;
  constexpr int PER = kBins / kTailThreads;
  uint32_t* lh = sm.u.st.hist;
  uint32_t kk[R], ii[R];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const uint32_t i = first + j * kTailThreads + threadIdx.x;
    kk[j] = i < nc ? ld_coh(&a.ckey[i]) : 0u;
    ii[j] = i < nc ? ld_coh(&a.cidx[i]) : 0u;
  }
#pragma unroll
  for (int b0 = 0; b0 < R; b0 += kPer) {
    for (int i = threadIdx.x; i < kBins; i += kTailThreads) lh[i] = 0;
    __syncthreads();  // histogram cleared
    uint32_t bb[kPer], rk[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const uint32_t i = first + (b0 + j) * kTailThreads + threadIdx.x;
      const uint32_t b = i < nc ? bm(comp(kk[b0 + j], ii[b0 + j])) : (uint32_t)kBins;
      bb[j] = b <= bstar ? gt[b] : (uint32_t)kBins;  // the group, or kBins: not scattered
      rk[j] = bb[j] < (uint32_t)kBins ? atomicAdd(&lh[bb[j]], 1u) : 0u;
    }
    __syncthreads();
    uint32_t base[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {  // reserve each group's range for this batch
      const uint32_t g = threadIdx.x * PER + j;
      const uint32_t cnt = lh[g];
      base[j] = cnt ? ld_coh(&ctl->gbase[g]) + atomicAdd(&ctl->bcur[g], cnt) : 0u;
    }
    __syncthreads();  // every count read before it is overwritten by the base
#pragma unroll
    for (int j = 0; j < PER; ++j) lh[threadIdx.x * PER + j] = base[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      if (bb[j] < (uint32_t)kBins) {
        const uint32_t slot = lh[bb[j]] + rk[j];
        if (slot < a.cap_s) {
          st_coh(&a.skey[slot], kk[b0 + j]);
          st_coh(&a.sidx[slot], ii[b0 + j]);
        } else {
          flag_err(ctl, ERR_CAP);
        }
      }
    }
    __syncthreads();  // the bases are read before the next batch clears them
  }
}

// ---- large-k sort of the fallback path ---------------------------------------
// The k compacted entries (okey / oidx) sorted without leaving the kernel:
// tiles of kSortTile sorted in LDS into A, then runs merged pairwise, one
// phase per level; an entry's slot in its merged run is its slot in its own
// run plus the entries of the partner run placed before it (strictly greater
// for the left run, greater or equal for the right one, so equal pads stay
// in order).  The last level writes the outputs.
constexpr int PH_MS = 24;           // phase of the tile sorts; the merge levels follow
constexpr uint32_t kMChunk = 4096;  // entries per merge claim
static_assert(PH_MS + 1 + 20 <= kPhases, "merge levels for k < 2^32");

template <int DT>
__device__ inline void tail_merge_sort(const TailArgs& a, Ctl* ctl, TailSmem& sm) {
  Phase* ph = ctl->ph;
  uint64_t* A = a.A;
  uint64_t* B = a.B;
  const uint64_t M = a.M;
  const uint32_t k = a.k;
  {
    const uint32_t ntiles = (uint32_t)(M / kSortTile);
    uint32_t mine = 0;
    uint64_t* buf = sm.u.sortbuf;
    for (;;) {
      const uint32_t c = claim(&ph[PH_MS], ntiles, sm);
      if (c >= ntiles) break;
      ++mine;
      for (uint32_t j = threadIdx.x; j < (uint32_t)kSortTile; j += kTailThreads) {
        const uint64_t i = (uint64_t)c * kSortTile + j;
        buf[j] = i < k ? comp(ld_coh(&a.okey[i]), ld_coh(&a.oidx[i])) : 0ull;
      }
      __syncthreads();
      lds_sort_desc(buf, kSortTile);
      for (uint32_t j = threadIdx.x; j < (uint32_t)kSortTile; j += kTailThreads)
        st_coh64(&A[(uint64_t)c * kSortTile + j], buf[j]);
      __syncthreads();
    }
    if (report(&ph[PH_MS], mine, ntiles, sm)) raise_ready(&ph[PH_MS]);
    wait_ready(&ph[PH_MS], ctl);
  }
  int level = 0;
  for (uint64_t run = kSortTile; run < M; run <<= 1, ++level) {
    const bool last = 2 * run == M;
    Phase* P = &ph[PH_MS + 1 + level];
    const uint32_t nch = (uint32_t)(M / kMChunk);
    uint32_t mine = 0;
    for (;;) {
      const uint32_t c = claim(P, nch, sm);
      if (c >= nch) break;
      ++mine;
      for (uint32_t j = threadIdx.x; j < kMChunk; j += kTailThreads) {
        const uint64_t i = (uint64_t)c * kMChunk + j;
        const uint64_t base = i / (2 * run) * (2 * run);
        const bool left = i - base < run;
        const uint64_t own = left ? i - base : i - base - run;
        const uint64_t* other = A + (left ? base + run : base);
        const uint64_t x = ld_coh64(&A[i]);
        uint64_t lo = 0, hi = run;
        while (lo < hi) {
          const uint64_t mid = (lo + hi) >> 1;
          const uint64_t y = ld_coh64(&other[mid]);
          if (left ? y > x : y >= x) lo = mid + 1;
          else hi = mid;
        }
        const uint64_t slot = own + lo;
        if (last) {
          if (slot < k) write_out<DT>(x, (uint32_t)slot, k, a.out_vals, a.out_idx, a.out_kth);
        } else {
          st_coh64(&B[base + slot], x);
        }
      }
    }
    if (last) break;
    if (report(P, mine, nch, sm)) raise_ready(P);
    wait_ready(P, ctl);
    uint64_t* t = A;
    A = B;
    B = t;
  }
  if (blockIdx.x == 0) stamp(ctl, PH_FS);
}

template <int DT, int BETA, bool VEC>
__global__ __launch_bounds__(kTailThreads) void k_tail(TailArgs a) {
  __shared__ TailSmem sm;
  Ctl* ctl = a.ctl;
  Phase* ph = ctl->ph;
  if (blockIdx.x == 0) stamp(ctl, kPhases + 1);

  // ---- threshold ---------------------------------------------------------------
  // Rule 2 needs only a lower bound of the kD-th delegate t.  The delegate pass
  // left the bin holding it, under the better of two monotone maps; its lowest
  // key t' works (as composite T = t' << 32, below every element with that
  // key), or, when the bin is crowded, the lowest key of the finer sub-bin
  // holding t.  m = the delegates ranked >= T bounds the survivors by
  // floor(m/beta)*2^alpha + m, so T is kept only while m <= kD + slack (the
  // buffers are sized for that); otherwise -- massive ties -- the exact t is
  // found by a radix select over the delegates.
  uint64_t T = 0;
  if (!a.all) {
    // the cut bin's key interval, clipped to the delegate keys present (t's
    // key lies in both; no delegate lies between their ends)
    uint32_t lo = ctl->cut_lo, hi = ctl->cut_hi;
    {
      const uint32_t dmax = comp_key(ctl->max1), dmin = ~ctl->dknmin;
      const uint32_t clo = lo > dmin ? lo : dmin, chi = hi < dmax ? hi : dmax;
      if (ctl->dknmin && clo <= chi) {
        lo = clo;
        hi = chi;
      }
    }
    const uint32_t crowd = (1u << 22) >> (a.alpha < 22 ? a.alpha : 22);
    const uint64_t limit = (uint64_t)a.kD + a.slack;
    uint64_t m = (uint64_t)a.kD - ctl->cut_rank + ctl->cut_count;
    const bool refine = hi > lo && (m > limit || ctl->cut_count > (crowd > 256u ? crowd : 256u));
    uint32_t tkey = lo;
    // the bin (or sub-bin) holding t: its key range and t's rank inside it
    uint32_t bhi = hi, brank = ctl->cut_rank;
    if (refine) {
      const uint32_t fsh = bitlen32(hi - lo) > 11u ? bitlen32(hi - lo) - 11u : 0u;
      for (int i = threadIdx.x; i < kBins; i += kTailThreads) sm.u.st.hist[i] = 0;
      // claims of 16 delegates per thread: 2^21 delegates take one round of
      // claims over the device
      constexpr uint32_t kHChunk = kTailThreads * 16;
      const uint32_t nchunks = (uint32_t)((a.nd + kHChunk - 1) / kHChunk);
      uint32_t mine = 0;
      uint32_t kmx = 0, knm = 0;  // largest key in the bin, complement of the smallest
      for (;;) {
        const uint32_t c = claim(&ph[PH_H], nchunks, sm);
        if (c >= nchunks) break;
        ++mine;
        // every load of the claim first, then the tests; padding entries have
        // key 0, so positions are read only when the bin starts at key 0
        constexpr int R = kHChunk / kTailThreads;
        uint32_t kv[R], iv[R];
#pragma unroll
        for (int j = 0; j < R; ++j) {
          const uint64_t i = (uint64_t)c * kHChunk + (uint64_t)j * kTailThreads + threadIdx.x;
          kv[j] = i < a.nd ? a.dkey[i] : 0u;
          iv[j] = i >= a.nd ? kInvalid : lo == 0u ? a.didx[i] : 0u;
        }
#pragma unroll
        for (int j = 0; j < R; ++j) {
          const uint32_t kk = kv[j];
          if (kk >= lo && kk <= hi && iv[j] != kInvalid) {
            atomicAdd(&sm.u.st.hist[(kk - lo) >> fsh], 1u);
            kmx = kk > kmx ? kk : kmx;
            knm = ~kk > knm ? ~kk : knm;
          }
        }
      }
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const uint32_t x = (uint32_t)__shfl_xor((int)kmx, o), y = (uint32_t)__shfl_xor((int)knm, o);
        kmx = x > kmx ? x : kmx;
        knm = y > knm ? y : knm;
      }
      if (lane_id() == 0) {
        sm.rwave[threadIdx.x >> 6] = kmx;
        sm.rwave[kTailThreads / 64 + (threadIdx.x >> 6)] = knm;
      }
      __syncthreads();
      if (mine) {
        for (int i = threadIdx.x; i < kBins; i += kTailThreads) {
          const uint32_t v = sm.u.st.hist[i];
          if (v) atomicAdd(&ctl->histH[i], v);
        }
        if (threadIdx.x == 0) {
          for (int w = 0; w < kTailThreads / 64; ++w) {
            kmx = sm.rwave[w] > kmx ? sm.rwave[w] : kmx;
            knm = sm.rwave[kTailThreads / 64 + w] > knm ? sm.rwave[kTailThreads / 64 + w] : knm;
          }
          atomicMax(&ctl->rkmax, kmx);
          atomicMax(&ctl->rknmin, knm);
        }
      }
      if (report(&ph[PH_H], mine, nchunks, sm)) {
        tail_bucket(ctl->histH, ctl->cut_rank, sm.scan, sm.out);
        if (threadIdx.x == 0) {
          // padding entries (key 0) were left out of the sub-bins; if that leaves
          // the rank unreached, keep the whole bin.  The key range is then cut
          // to the delegate keys present in the bin: t's key lies in it, and no
          // delegate lies between its ends and the (sub-)bin's
          const bool ok = sm.out[2] != 0;
          const uint32_t sublo = lo + (sm.out[0] << fsh);
          const uint32_t subhi = hi - sublo > (1u << fsh) - 1u ? sublo + ((1u << fsh) - 1u) : hi;
          const uint32_t kmax = ld_coh(&ctl->rkmax), kmin = ~ld_coh(&ctl->rknmin);
          const bool seen = kmax >= kmin;  // always, unless the bin was empty (an internal error)
          const uint32_t elo = ok ? sublo : lo, ehi = ok ? subhi : hi;
          st_coh(&ctl->tpub[0], seen && kmin > elo ? kmin : elo);
          st_coh(&ctl->tpub[1], ok ? a.kD - sm.out[1] + sm.out[3] : (uint32_t)(m < 0xFFFFFFFFull ? m : 0xFFFFFFFFull));
          st_coh(&ctl->tpub[2], seen && kmax < ehi ? kmax : ehi);
          st_coh(&ctl->tpub[3], ok ? sm.out[1] : ctl->cut_rank);
        }
        stamp(ctl, PH_H);
        raise_ready(&ph[PH_H]);
      }
      wait_ready(&ph[PH_H], ctl);
      tkey = ld_coh(&ctl->tpub[0]);
      m = ld_coh(&ctl->tpub[1]);
      bhi = ld_coh(&ctl->tpub[2]);
      brank = ld_coh(&ctl->tpub[3]);
    }
    if (m <= limit) {
      T = (uint64_t)tkey << 32;
    } else {
      // massive ties: a radix select, from the position digits on when the
      // bin holds a single key, stopping once t's class has at most
      // kBoundTol members below t (any T <= t serves Rule 2, and the
      // delegates at or above T stay within kD + slack)
      const bool one_key = tkey == bhi;
      T = tail_select(a.dkey, a.didx, (uint32_t)a.nd, one_key ? brank : a.kD, ctl->histW, &ph[PH_DSEL],
                      ctl->selpub, ctl, sm, one_key, tkey, true);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->selD.prefix = T;  // host statistics

  // survivors' output buckets over [T, largest element]; counted in LDS (the
  // output sort's bins, free until the output step)
  BucketMap bm;
  {
    const uint64_t top = ld_coh64(&ctl->max1);
    const uint32_t rb = bitlen64(top > T ? top - T : 0ull);
    bm.lo = T;
    bm.sh = rb > 11u ? rb - 11u : 0u;
  }
  uint32_t* bh = sm.rbins;
  for (int i = threadIdx.x; i < kBins; i += kTailThreads) bh[i] = 0;

  // ---- Q: Rule 3 against T -----------------------------------------------------
  // Subrange s is re-read iff its beta-th delegate ranks above T; otherwise its
  // delegates ranked >= T are survivors.  (T = 0 when there are fewer real
  // delegates than k: every subrange with beta real delegates is re-read.)
  if (threadIdx.x == 0) { sm.u.st.sq.n = 0; sm.u.st.sc.n = 0; }
  {
    // subranges per thread and claim: 8 at beta <= 2, else 16 / beta (the
    // stages then hold a whole claim's output either way)
    constexpr uint32_t kQR = BETA <= 2 ? 8 : 16 / BETA;
    constexpr uint32_t kQChunk = kTailThreads * kQR;
    const uint32_t nchunks = (uint32_t)((a.S + kQChunk - 1) / kQChunk);
    uint32_t mine = 0;
    if constexpr (BETA <= 2) {
      // every delegate of the claim's 8 x kTailThreads subranges is loaded
      // before any is tested (16 loads in flight per thread)
      using DV = typename std::conditional<BETA == 1, uint32_t, u32x2>::type;
      for (;;) {
        const uint32_t c = claim(&ph[PH_Q], nchunks, sm);
        if (c >= nchunks) break;
        ++mine;
        DV dk[8], di[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const uint64_t s = (uint64_t)c * kQChunk + (uint64_t)i * kTailThreads + threadIdx.x;
          const uint64_t sc = s < a.S ? s : 0;
          dk[i] = reinterpret_cast<const DV*>(a.dkey)[sc];
          di[i] = reinterpret_cast<const DV*>(a.didx)[sc];
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const uint64_t s = (uint64_t)c * kQChunk + (uint64_t)i * kTailThreads + threadIdx.x;
          const bool ok = s < a.S;
          uint32_t kk[BETA], ii[BETA];
          if constexpr (BETA == 1) {
            kk[0] = dk[i];
            ii[0] = di[i];
          } else {
            kk[0] = dk[i].x; kk[1] = dk[i].y;
            ii[0] = di[i].x; ii[1] = di[i].y;
          }
          const bool scan = ok && ii[BETA - 1] != kInvalid && comp(kk[BETA - 1], ii[BETA - 1]) > T;
          stage_push(sm.u.st.sq, scan, (uint32_t)s, 0u);
#pragma unroll
          for (int j = 0; j < BETA; ++j) {
            const bool take = ok && !scan && ii[j] != kInvalid && comp(kk[j], ii[j]) >= T;
            hist_add_wave(bh, take, take ? bm(comp(kk[j], ii[j])) : 0u);
            stage_push(sm.u.st.sc, take, kk[j], ii[j]);
          }
        }
        // the stages hold a whole claim: one capacity check per claim
        stage_flush2_coh(sm.u.st.sq, &ctl->nq, ctl->cap_q, a.Q, 8 * kTailThreads, sm.u.st.sc, &ctl->nc,
                         ctl->cap_c, a.ckey, a.cidx, 8 * kTailThreads * BETA, ctl);
      }
    } else {
      // beta = 4 or 8: each subrange's delegate list is beta / 4 16-byte
      // vectors of keys and as many of positions (the delegate arrays start
      // 256-byte aligned in the workspace), all of the claim's loaded before
      // any is tested
      constexpr int NV = BETA / 4;
      for (;;) {
        const uint32_t c = claim(&ph[PH_Q], nchunks, sm);
        if (c >= nchunks) break;
        ++mine;
        u32x4 dk[kQR][NV], di[kQR][NV];
#pragma unroll
        for (int i = 0; i < (int)kQR; ++i) {
          const uint64_t s = (uint64_t)c * kQChunk + (uint64_t)i * kTailThreads + threadIdx.x;
          const uint64_t sc = s < a.S ? s : 0;
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            dk[i][v] = reinterpret_cast<const u32x4*>(a.dkey)[sc * NV + v];
            di[i][v] = reinterpret_cast<const u32x4*>(a.didx)[sc * NV + v];
          }
        }
#pragma unroll
        for (int i = 0; i < (int)kQR; ++i) {
          const uint64_t s = (uint64_t)c * kQChunk + (uint64_t)i * kTailThreads + threadIdx.x;
          const bool ok = s < a.S;
          const uint32_t kl = dk[i][NV - 1][3], il = di[i][NV - 1][3];  // the beta-th delegate
          const bool scan = ok && il != kInvalid && comp(kl, il) > T;
          stage_push(sm.u.st.sq, scan, (uint32_t)s, 0u);
#pragma unroll
          for (int j = 0; j < BETA; ++j) {
            const uint32_t kk = dk[i][j >> 2][j & 3], ii = di[i][j >> 2][j & 3];
            const bool take = ok && !scan && ii != kInvalid && comp(kk, ii) >= T;
            hist_add_wave(bh, take, take ? bm(comp(kk, ii)) : 0u);
            stage_push(sm.u.st.sc, take, kk, ii);
          }
        }
        stage_flush2_coh(sm.u.st.sq, &ctl->nq, ctl->cap_q, a.Q, kQR * kTailThreads, sm.u.st.sc, &ctl->nc,
                         ctl->cap_c, a.ckey, a.cidx, kQR * kTailThreads * BETA, ctl);
      }
    }
    // everything a block staged is published before it reports its chunks:
    // a phase's completion then implies all of its output is visible
    stage_flush_coh(sm.u.st.sq, &ctl->nq, ctl->cap_q, a.Q, nullptr, ctl, true, 0);
    stage_flush_coh(sm.u.st.sc, &ctl->nc, ctl->cap_c, a.ckey, a.cidx, ctl, true, 0);
    hist_flush(bh, ctl->bcount);
    if (report(&ph[PH_Q], mine, nchunks, sm)) {
      stamp(ctl, PH_Q);
      raise_ready(&ph[PH_Q]);
    }
    wait_ready(&ph[PH_Q], ctl);
  }

  // ---- S: the virtual concatenated vector of the queued subranges -----------
  bool s_final = false;
  {
    const uint32_t nq = ld_coh(&ctl->nq) < ctl->cap_q ? ld_coh(&ctl->nq) : ctl->cap_q;
    const uint64_t total = (uint64_t)nq << a.alpha;
    // claims of 1..16 steps of kTailThreads x 4 elements: the fewest that
    // cover the re-read in at most 1.25 rounds of claims over the device
    // (each claim costs a chain of latencies, so one larger claim per block
    // beats two smaller ones; a few extra claims are taken by the blocks that
    // finish first), 16 when even those take several rounds
    constexpr uint32_t kStep = kTailThreads * 4;
    const uint64_t tsteps = (total + kStep - 1) / kStep;
    uint32_t steps = 1;
    while (steps < kSChunk / kStep && (uint64_t)steps * gridDim.x * 5 < tsteps * 4) steps <<= 1;
    const uint32_t chunk = steps * kStep;
    const uint32_t nchunks = (uint32_t)((total + chunk - 1) / chunk);
    const uint64_t lmask = (1ull << a.alpha) - 1;
    if (threadIdx.x == 0) sm.u.st.sc.n = 0;
    uint32_t mine = 0;
    for (;;) {
      const uint32_t ch = claim(&ph[PH_S], nchunks, sm);
      if (ch >= nchunks) break;
      ++mine;
      if (VEC && a.alpha >= 2) {
        const uint64_t first = (uint64_t)ch * chunk;
        if (steps == 16) s_claim_vec<DT, 16>(a, first, total, T, sm, bm, bh, ctl);
        else if (steps == 8) s_claim_vec<DT, 8>(a, first, total, T, sm, bm, bh, ctl);
        else if (steps == 4) s_claim_vec<DT, 4>(a, first, total, T, sm, bm, bh, ctl);
        else if (steps == 2) s_claim_vec<DT, 2>(a, first, total, T, sm, bm, bh, ctl);
        else s_claim_vec<DT, 1>(a, first, total, T, sm, bm, bh, ctl);
        continue;
      }
      for (uint32_t j = 0; j < chunk; j += kStep) {
        const uint64_t e = (uint64_t)ch * chunk + j + threadIdx.x * 4;
        uint32_t v[4];
        uint64_t pos[4];
        bool in[4];
        if (VEC && a.alpha >= 2) {
          const uint64_t p = e < total ? ((uint64_t)ld_coh(&a.Q[e >> a.alpha]) << a.alpha) + (e & lmask) : a.n;
#pragma unroll
          for (int c = 0; c < 4; ++c) { pos[c] = p + c; in[c] = p + c < a.n; }
          if (p + 4 <= a.n) {
            load4<DT, true>(a.keys, p, v);
          } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) v[c] = in[c] ? a.keys[p + c] : 0u;
          }
        } else {
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const uint64_t ec = e + c;
            pos[c] = ec < total ? ((uint64_t)ld_coh(&a.Q[ec >> a.alpha]) << a.alpha) + (ec & lmask) : a.n;
            in[c] = pos[c] < a.n;
            v[c] = in[c] ? a.keys[pos[c]] : 0u;
          }
        }
        bool take[4];
        uint32_t kk[4], ii[4], bin[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          kk[c] = enc<DT>(v[c]);
          ii[c] = (uint32_t)pos[c];
          const uint64_t cc = comp(kk[c], ii[c]);
          take[c] = in[c] && cc >= T;
          bin[c] = take[c] ? bm(cc) : 0u;
        }
        uint32_t pbin = 0xFFFFFFFFu, pcnt = 0;
        hist_add_wave4(bh, take, bin, pbin, pcnt);
        hist_pending_flush(bh, pbin, pcnt);
        stage_push4(sm.u.st.sc, take, kk, ii);
        stage_flush_coh(sm.u.st.sc, &ctl->nc, ctl->cap_c, a.ckey, a.cidx, ctl, false, kTailThreads * 4);
      }
    }
    stage_flush_coh(sm.u.st.sc, &ctl->nc, ctl->cap_c, a.ckey, a.cidx, ctl, true, 0);
    hist_flush(bh, ctl->bcount);
    if (report(&ph[PH_S], mine, nchunks, sm)) {
      stamp(ctl, PH_S);
      raise_ready(&ph[PH_S]);
      s_final = true;
    }
    if (nchunks) wait_ready(&ph[PH_S], ctl);
  }
  if (a.stop_after_scan) return;

  // ---- F: the output ---------------------------------------------------------
  const uint32_t nc = ld_coh(&ctl->nc) < ctl->cap_c ? ld_coh(&ctl->nc) : ctl->cap_c;
  if (nc < a.k) {
    if (blockIdx.x == 0 && threadIdx.x == 0) flag_err(ctl, ERR_FEW);
    return;
  }
  if (nc <= (uint32_t)kSmallCap) {
    // the block that completed the re-read sorts (or any one block if nothing was re-read)
    const bool had_scan = ld_coh(&ctl->nq) != 0u;
    if (had_scan ? !s_final : claim(&ph[PH_F1], 1, sm) != 0) return;
    small_output<DT>(a, nc, sm);
    stamp(ctl, PH_F1);
    return;
  }

  // Many survivors.  Q and S counted them into output buckets; one block
  // turns the counts into bucket offsets (exclusive scan, bucket 0 first),
  // finds the bucket b* holding output slot k-1, and cuts the buckets up to
  // b* into sort groups: group w holds the buckets whose first slot lies in
  // [w*kGroup, (w+1)*kGroup), so a group holds < 2 kGroup when no bucket up
  // to b* exceeds kGroup.  Buckets after b* hold no output and are neither
  // scattered nor sorted.  An overfull bucket up to b* (massive ties) takes
  // the select path instead.
  if (claim(&ph[PH_B1], 1, sm) == 0) {
    constexpr int PER = kBins / kTailThreads;
    uint32_t* lb = sm.u.st.hist;
    const int t0 = threadIdx.x * PER;
    uint32_t cnt[PER], sum = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      cnt[j] = ld_coh(&ctl->bcount[t0 + j]);
      sum += cnt[j];
    }
    sm.scan[threadIdx.x] = sum;
    if (threadIdx.x == 0) { sm.out[0] = kBins; sm.out[1] = 0; }
    __syncthreads();
    for (int o = 1; o < kTailThreads; o <<= 1) {
      const uint32_t x = threadIdx.x >= (unsigned)o ? sm.scan[threadIdx.x - o] : 0u;
      __syncthreads();
      sm.scan[threadIdx.x] += x;
      __syncthreads();
    }
    uint32_t off = sm.scan[threadIdx.x] - sum;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      lb[t0 + j] = off;
      st_coh(&ctl->boff[t0 + j], off);
      if (off < a.k && a.k <= off + cnt[j]) {  // exactly one bucket holds slot k-1
        sm.out[0] = t0 + j;
        sm.out[1] = off + cnt[j];
      }
      off += cnt[j];
    }
    if (threadIdx.x == kTailThreads - 1) st_coh(&ctl->boff[kBins], off);
    __syncthreads();
    const uint32_t bstar = sm.out[0], lim = sm.out[1], total = sm.scan[kTailThreads - 1];
    uint32_t big = 0;  // fullest bucket up to b*
#pragma unroll
    for (int j = 0; j < PER; ++j)
      if ((uint32_t)(t0 + j) <= bstar) big = cnt[j] > big ? cnt[j] : big;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const uint32_t y = (uint32_t)__shfl_xor((int)big, o);
      big = y > big ? y : big;
    }
    if (lane_id() == 0) sm.rwave[threadIdx.x >> 6] = big;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kTailThreads / 64; ++i) big = sm.rwave[i] > big ? sm.rwave[i] : big;
    // every survivor was counted once: a mismatch is an internal error
    const bool bad = bstar >= (uint32_t)kBins || total != ld_coh(&ctl->nc);
    const uint32_t nwin = (lim + kGroup - 1) / kGroup;
    if (bad || big > kGroup || nwin > (uint32_t)kBins) {
      if (threadIdx.x == 0) {
        atomicOr(&ctl->bigbucket, 1u);
        if (bad) flag_err(ctl, ERR_SELECT);
      }
    } else {
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const uint32_t b = t0 + j;
        if (b > bstar) break;
        const int64_t wb = lb[b] / kGroup;
        const int64_t wp = b == 0 ? -1 : (int64_t)(lb[b - 1] / kGroup);
        st_coh(&ctl->bgrp[b], (uint32_t)wb);
        for (int64_t w = wp + 1; w <= wb; ++w) {
          st_coh(&ctl->gfirst[w], b);
          st_coh(&ctl->gbase[w], lb[b]);
        }
        if (b == bstar)
          for (uint32_t w = (uint32_t)wb + 1; w <= nwin; ++w) {
            st_coh(&ctl->gfirst[w], bstar + 1);
            st_coh(&ctl->gbase[w], lb[b] + cnt[j]);
          }
      }
      if (threadIdx.x == 0) {
        st_coh(&ctl->ngroups, nwin);
        st_coh(&ctl->bstar, bstar);
      }
    }
    stamp(ctl, PH_B1);
    raise_ready(&ph[PH_B1]);
  }
  wait_ready(&ph[PH_B1], ctl);
  if (ld_coh(&ctl->bigbucket) == 0u) {
    // B2: scatter the buckets up to b* into bucket order
    {
      const uint32_t bstar = ld_coh(&ctl->bstar);
      // claims of R x kTailThreads survivors, R = 8, 16 or 32: the largest
      // that still gives every block a claim, so that many survivors (sorted
      // or tied inputs) take fewer claims, each with all of its loads in flight
      uint32_t R = 32;
      while (R > 8 && (nc + R * kTailThreads - 1) / (R * kTailThreads) < gridDim.x) R >>= 1;
      const uint32_t chunk = R * kTailThreads;
      const uint32_t nchunks = (nc + chunk - 1) / chunk;
      uint32_t mine = 0;
      static_assert(kBins <= 8 * kTailThreads, "the bucket-to-group table fits the idle Q stage");
      uint32_t* gt = sm.u.st.sq.key;  // bucket -> sort group, for buckets up to b*
      for (;;) {
        const uint32_t c = claim(&ph[PH_B2], nchunks, sm);
        if (c >= nchunks) break;
        if (mine++ == 0) {
          for (uint32_t b = threadIdx.x; b <= bstar; b += kTailThreads) gt[b] = ld_coh(&ctl->bgrp[b]);
          __syncthreads();
        }
        if (R == 32) b2_claim<32>(a, c * chunk, nc, bstar, bm, gt, sm, ctl);
        else if (R == 16) b2_claim<16>(a, c * chunk, nc, bstar, bm, gt, sm, ctl);
        else b2_claim<8>(a, c * chunk, nc, bstar, bm, gt, sm, ctl);
      }
      if (report(&ph[PH_B2], mine, nchunks, sm)) {
        stamp(ctl, PH_B2);
        raise_ready(&ph[PH_B2]);
      }
      wait_ready(&ph[PH_B2], ctl);
    }
    // B3: sort each group in LDS, write the slots below k
    {
      const uint32_t ng = ld_coh(&ctl->ngroups);
      uint32_t mine = 0;
      for (;;) {
        const uint32_t gi = claim(&ph[PH_B3], ng, sm);
        if (gi >= ng) break;
        ++mine;
        const uint32_t lo = ld_coh(&ctl->boff[ld_coh(&ctl->gfirst[gi])]);
        const uint32_t hi = ld_coh(&ctl->boff[ld_coh(&ctl->gfirst[gi + 1])]);
        if (lo >= a.k || hi <= lo) continue;
        const uint32_t cnt = hi - lo;
        if (cnt > (uint32_t)kSmallCap) {
          if (threadIdx.x == 0) flag_err(ctl, ERR_GROUP);
          continue;
        }
        sort_and_write<DT>(a.skey + lo, a.sidx + lo, cnt, lo, a.k - lo < cnt ? a.k - lo : cnt, a.k,
                           a.kth_only ? nullptr : a.out_vals, a.kth_only ? nullptr : a.out_idx, a.out_kth,
                           sm.u.sortbuf, RankLds{sm.rbins, sm.rred, sm.rwave});
      }
      if (report(&ph[PH_B3], mine, ng, sm)) stamp(ctl, PH_B3);
    }
    return;
  }

  // Fallback for an overfull bucket (massive ties): exact radix select of the
  // k-th survivor, exact compaction, then an LDS sort (k <= kSmallCap) or the
  // merge sort above, all in this kernel.
  if (threadIdx.x == 0 && blockIdx.x == 0) ctl->need_merge = a.big_sort ? 1u : 0u;
  const uint64_t Tk = tail_select(a.ckey, a.cidx, nc, a.k, ctl->histC, &ph[PH_FSEL], ctl->selpub + 4, ctl, sm);
  if (a.kth_only) {
    if (blockIdx.x == 0 && threadIdx.x == 0 && a.out_kth) *a.out_kth = dec<DT>(comp_key(Tk));
    return;
  }
  {
    if (threadIdx.x == 0) sm.u.st.sc.n = 0;
    const uint32_t nch = (nc + kWChunk - 1) / kWChunk;
    uint32_t mine = 0;
    for (;;) {
      const uint32_t c = claim(&ph[PH_FC], nch, sm);
      if (c >= nch) break;
      ++mine;
      for (uint32_t j = 0; j < kWChunk; j += kTailThreads) {
        const uint32_t i = c * kWChunk + j + threadIdx.x;
        uint64_t x = 0;
        if (i < nc) x = comp(ld_coh(&a.ckey[i]), ld_coh(&a.cidx[i]));
        stage_push(sm.u.st.sc, i < nc && x >= Tk, comp_key(x), comp_pos(x));
      }
      stage_flush_coh(sm.u.st.sc, &ctl->nout, a.k, a.okey, a.oidx, ctl, false, kWChunk);
    }
    stage_flush_coh(sm.u.st.sc, &ctl->nout, a.k, a.okey, a.oidx, ctl, true, 0);
    if (report(&ph[PH_FC], mine, nch, sm)) {
      stamp(ctl, PH_FC);
      raise_ready(&ph[PH_FC]);
    }
    wait_ready(&ph[PH_FC], ctl);
    if (a.big_sort) {  // k > kSmallCap
      tail_merge_sort<DT>(a, ctl, sm);
      return;
    }
  }
  if (claim(&ph[PH_FS], 1, sm) != 0) return;
  sort_and_write<DT>(a.okey, a.oidx, a.k, 0, a.k, a.k, a.out_vals, a.out_idx, a.out_kth, sm.u.sortbuf,
                     RankLds{sm.rbins, sm.rred, sm.rwave});
  stamp(ctl, PH_FS);
}

}  // namespace drtopk
