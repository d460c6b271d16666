// HIP kernels of the delegate-centric top-k path (gfx950, wave64).
//
//   k_delegate*   delegate vector (Rules 1 and 3): one streaming pass over V
//                 with 128-bit non-temporal loads, per-subrange top-beta, and
//                 the first radix digit of the delegates' histogram fused in
//   k_pass        one MSD digit of a radix select over composites (8 passes
//                 would do for 32-bit keys; 6 digits of 11/11/10 bits cover the
//                 64-bit key+position composite)
//   k_qualify     Rule 3 as a threshold test per subrange; delegates of the
//                 other subranges at or above the threshold go straight to
//                 the survivors
//   k_scan        re-reads only the qualifying subranges, keeps elements at or
//                 above the threshold (Rule 2), wave-ballot compaction
//   k_final_small survivors sorted in LDS by one workgroup
//   k_compact / k_blocksort / k_merge   large-k output: exact k, then a sort
#pragma once

#include "internal.h"

namespace drtopk {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// top-beta list of composites held by one lane (descending)
template <int BETA>
struct TopB {
  uint64_t c[BETA];
  __device__ __forceinline__ void clear() {
#pragma unroll
    for (int j = 0; j < BETA; ++j) c[j] = 0;
  }
  __device__ __forceinline__ void push(uint64_t x) {
    if constexpr (BETA == 1) {
      c[0] = x > c[0] ? x : c[0];
    } else {
      bool g[BETA];
#pragma unroll
      for (int j = 0; j < BETA; ++j) g[j] = x > c[j];
#pragma unroll
      for (int j = BETA - 1; j >= 1; --j) c[j] = g[j] ? (g[j - 1] ? c[j - 1] : x) : c[j];
      c[0] = g[0] ? x : c[0];
    }
  }
  // Four elements at once (BETA >= 4): a 5-comparator network sorts them,
  // the larger of c[BETA-1-j] and the j-th largest of the four replaces
  // c[BETA-1-j] (the top BETA of both lists, as a bitonic sequence), and
  // half-cleaners sort the list again: 21 compare-exchanges or maxima at
  // BETA = 8 where four single insertions take 32.
  __device__ __forceinline__ void push4(uint64_t x0, uint64_t x1, uint64_t x2, uint64_t x3) {
    static_assert(BETA >= 4, "push4 needs a list of at least four");
    cx(x0, x1); cx(x2, x3); cx(x0, x2); cx(x1, x3); cx(x1, x2);
    c[BETA - 1] = c[BETA - 1] > x0 ? c[BETA - 1] : x0;
    c[BETA - 2] = c[BETA - 2] > x1 ? c[BETA - 2] : x1;
    c[BETA - 3] = c[BETA - 3] > x2 ? c[BETA - 3] : x2;
    c[BETA - 4] = c[BETA - 4] > x3 ? c[BETA - 4] : x3;
    clean();
  }
  // Eight elements at once (BETA = 8): Batcher's 19-comparator network
  // sorts them and they are merged like push4's four, all eight entries
  // against the new ones reversed: 39 compare-exchanges or maxima per eight
  // elements against push4's 42.
  __device__ __forceinline__ void push8(uint64_t (&x)[8]) {
    static_assert(BETA == 8, "push8 needs a list of eight");
    cx(x[0], x[1]); cx(x[2], x[3]); cx(x[4], x[5]); cx(x[6], x[7]);
    cx(x[0], x[2]); cx(x[1], x[3]); cx(x[4], x[6]); cx(x[5], x[7]);
    cx(x[1], x[2]); cx(x[5], x[6]);
    cx(x[0], x[4]); cx(x[1], x[5]); cx(x[2], x[6]); cx(x[3], x[7]);
    cx(x[2], x[4]); cx(x[3], x[5]);
    cx(x[1], x[2]); cx(x[3], x[4]); cx(x[5], x[6]);
#pragma unroll
    for (int j = 0; j < 8; ++j) c[7 - j] = c[7 - j] > x[j] ? c[7 - j] : x[j];
    clean();
  }
  // Replace this list by the top-BETA of (this list, the list of a lane in
  // the other M-half of this lane's 2M-block); after the step both lanes hold
  // the same list, so steps M = 1, 2, 4, ... leave every lane of each block
  // with the block's top-BETA.  Max of one list against the other reversed is
  // bitonic and holds the top BETA; half-cleaners then sort it.
  template <int M>
  __device__ __forceinline__ void merge() {
    uint64_t o[BETA];
#pragma unroll
    for (int j = 0; j < BETA; ++j) o[j] = lane_cross64<M>(c[j]);
#pragma unroll
    for (int j = 0; j < BETA; ++j) c[j] = c[j] > o[BETA - 1 - j] ? c[j] : o[BETA - 1 - j];
    clean();
  }

 private:
  // a >= b afterwards
  static __device__ __forceinline__ void cx(uint64_t& a, uint64_t& b) {
    const uint64_t x = a, y = b;
    a = x > y ? x : y;
    b = x > y ? y : x;
  }
  // a bitonic list sorted descending
  __device__ __forceinline__ void clean() {
#pragma unroll
    for (int s = BETA / 2; s >= 1; s >>= 1) {
#pragma unroll
      for (int j = 0; j < BETA; ++j)
        if ((j & s) == 0) cx(c[j], c[j + s]);
    }
  }
};

// Top-BETA of every block of G consecutive lanes (G a wave-uniform power of
// two, at most 64), held by all of its lanes.
template <int BETA>
__device__ __forceinline__ void merge_lanes(TopB<BETA>& tb, uint32_t G) {
  if (G > 1) tb.template merge<1>();
  if (G > 2) tb.template merge<2>();
  if (G > 4) tb.template merge<4>();
  if (G > 8) tb.template merge<8>();
  if (G > 16) tb.template merge<16>();
  if (G > 32) tb.template merge<32>();
}

// ---------------------------------------------------------------------------
// block helpers (blockDim.x == 256)

// Finds, in a 2048-bin histogram read from global memory, the bin holding the
// rank-th largest entry (bins scanned from the top).  s_out = {bin, rank within
// bin, found}.
__device__ inline void block_select_bucket(const uint32_t* gh, uint32_t rank, uint32_t* s_scan,
                                           uint32_t* s_out) {
  const int t = threadIdx.x;
  uint32_t c[8], sum = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    c[j] = atomic_load_u32(&gh[kBins - 1 - 8 * t - j]);
    sum += c[j];
  }
  s_scan[t] = sum;
  if (t == 0) { s_out[0] = 0; s_out[1] = 0; s_out[2] = 0; }
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    uint32_t x = t >= off ? s_scan[t - off] : 0u;
    __syncthreads();
    s_scan[t] += x;
    __syncthreads();
  }
  uint32_t incl = s_scan[t], excl = incl - sum;
  if (excl < rank && rank <= incl) {
    uint32_t cum = excl;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (cum + c[j] >= rank) {
        s_out[0] = kBins - 1 - 8 * t - j;
        s_out[1] = rank - cum;
        s_out[2] = 1;
        break;
      }
      cum += c[j];
    }
  }
  __syncthreads();
}

__device__ inline void flush_hist(const uint32_t* lh, uint32_t* gh) {
  for (int i = threadIdx.x; i < kBins; i += blockDim.x) {
    uint32_t v = lh[i];
    if (v) atomicAdd(&gh[i], v);
  }
}

// Completes digit pass p: the last block to finish (ticket) derives the new
// selection state from the finished global histogram.
//
// Only atomics carry data between blocks here, so no cache writeback is
// needed: each wave waits until its own histogram atomics have completed
// (s_waitcnt; an agent-scope fence would instead write back the whole L2 of
// the XCD, once per wave), the block then takes a ticket, and the last block
// reads the histogram with coherent (sc1) atomic loads.
__device__ inline void finish_pass(uint32_t* gh, uint32_t* ticket, Sel* sel, int p, uint32_t k,
                                   Ctl* ctl, uint32_t* s_scan, uint32_t* s_out, int* s_last) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) *s_last = (atomicAdd(ticket, 1u) == gridDim.x - 1) ? 1 : 0;
  __syncthreads();
  if (!*s_last) return;
  uint64_t prefix = 0, mask = 0;
  uint32_t rank = k;
  if (p > 0) {
    prefix = sel->prefix;
    mask = sel->mask;
    rank = sel->rank;
  }
  block_select_bucket(gh, rank, s_scan, s_out);
  if (threadIdx.x == 0) {
    const int sh = pass_shift(p);
    const uint64_t dm = (1ull << pass_bits(p)) - 1;
    sel->prefix = prefix | ((uint64_t)s_out[0] << sh);
    sel->mask = mask | (dm << sh);
    sel->rank = s_out[1];
    sel->found = s_out[2];
    if (!s_out[2]) flag_err(ctl, ERR_SELECT);
  }
}

// ---------------------------------------------------------------------------
// LDS-staged appends: waves append into a block buffer with LDS atomics; the
// block reserves global space with one atomic per flush.

template <int CAP>
struct Stage {
  uint32_t key[CAP];
  uint32_t idx[CAP];
  uint32_t n;
  uint32_t base;
};

template <int CAP>
__device__ __forceinline__ void stage_init(Stage<CAP>& S) {
  if (threadIdx.x == 0) S.n = 0;
  __syncthreads();
}

// Whole wave active.  Lanes with `pred` append (key, idx).
template <int CAP>
__device__ __forceinline__ void stage_push(Stage<CAP>& S, bool pred, uint32_t key, uint32_t idx) {
  const uint64_t b = __ballot(pred);
  if (!b) return;
  const int leader = __ffsll((unsigned long long)b) - 1;
  uint32_t off = 0;
  if ((int)lane_id() == leader) off = atomicAdd(&S.n, (uint32_t)__popcll(b));
  off = (uint32_t)__shfl((int)off, leader) + mbcnt(b);
  if (pred) {
    S.key[off] = key;
    S.idx[off] = idx;
  }
}

// Block-uniform.  Flushes when `force` or when fewer than `margin` slots are
// left.  gidx may be null (keys only).  Entries past gcap set ctl->err.
template <int CAP>
__device__ __forceinline__ void stage_flush(Stage<CAP>& S, uint32_t* gcount, uint32_t gcap, uint32_t* gkey,
                                            uint32_t* gidx, Ctl* ctl, bool force, uint32_t margin) {
  __syncthreads();
  const uint32_t n = S.n;
  const bool doit = n != 0 && (force || n + margin > (uint32_t)CAP);
  __syncthreads();  // every wave has read n before anyone appends again
  if (!doit) return;
  if (threadIdx.x == 0) S.base = atomicAdd(gcount, n);
  __syncthreads();
  const uint32_t base = S.base;
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
    if (base + i < gcap) {
      gkey[base + i] = S.key[i];
      if (gidx) gidx[base + i] = S.idx[i];
    } else {
      flag_err(ctl, ERR_CAP);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) S.n = 0;
  __syncthreads();
}

// ---------------------------------------------------------------------------
// delegate vector

// Per-thread summary of the delegates this thread emitted: the largest
// composite, and the complement of the smallest key (0 = none).
struct DelAcc {
  uint64_t mx = 0;
  uint32_t nmn = 0;
};

template <int BETA>
__device__ __forceinline__ void emit_delegates(uint64_t s, const TopB<BETA>& tb, uint32_t* dkey,
                                               uint32_t* didx, uint32_t* lh, DelAcc& acc) {
#pragma unroll
  for (int j = 0; j < BETA; ++j) {
    const uint32_t kk = comp_key(tb.c[j]);
    dkey[s * BETA + j] = kk;
    didx[s * BETA + j] = comp_pos(tb.c[j]);  // padding (composite 0) gives 0xFFFFFFFF
    atomicAdd(&lh[top_bin(kk)], 1u);
    atomicAdd(&lh[kBins + log_bin(kk)], 1u);
    if (tb.c[j]) acc.nmn = ~kk > acc.nmn ? ~kk : acc.nmn;
  }
  acc.mx = tb.c[0] > acc.mx ? tb.c[0] : acc.mx;
}

template <int DT>
__device__ __forceinline__ void write_out(uint64_t c, uint32_t r, uint32_t k, uint32_t* out_vals,
                                          uint32_t* out_idx, uint32_t* out_kth) {
  const uint32_t v = dec<DT>(comp_key(c));
  if (out_vals) out_vals[r] = v;
  if (out_idx) out_idx[r] = comp_pos(c);
  if (out_kth && r == k - 1) *out_kth = v;
}

// Outputs written by the delegate pass itself when k = 1: the largest
// element is the largest delegate (Rule 1), so no later step is needed.
struct DirectOut {
  uint32_t* vals;
  uint32_t* idx;
  uint32_t* kth;
  int on;
};

// End of the delegate pass: the last block finds, under both monotone maps,
// the bin holding the kD-th largest delegate, and keeps the map whose cut
// leaves the smaller set W (all delegates in that bin or above).
__device__ inline void finish_delegates(const uint32_t* lh, Ctl* ctl, uint32_t kD, uint32_t* s_scan,
                                        uint32_t* s_out, int* s_last, DelAcc acc, uint64_t* s_red) {
  for (int i = threadIdx.x; i < kBins; i += blockDim.x) {
    const uint32_t a = lh[i], b = lh[kBins + i];
    if (a) atomicAdd(&ctl->histD[0][i], a);
    if (b) atomicAdd(&ctl->histL[i], b);
  }
  // the block's largest delegate and smallest delegate key, over its waves
  // (s_red: 2 entries per wave)
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const uint64_t m = shfl_xor64(acc.mx, o);
    const uint32_t q = (uint32_t)__shfl_xor((int)acc.nmn, o);
    acc.mx = m > acc.mx ? m : acc.mx;
    acc.nmn = q > acc.nmn ? q : acc.nmn;
  }
  const uint32_t nw = blockDim.x >> 6;
  if (lane_id() == 0) {
    s_red[threadIdx.x >> 6] = acc.mx;
    s_red[nw + (threadIdx.x >> 6)] = acc.nmn;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (uint32_t w = 1; w < nw; ++w) {
      acc.mx = s_red[w] > acc.mx ? s_red[w] : acc.mx;
      acc.nmn = (uint32_t)s_red[nw + w] > acc.nmn ? (uint32_t)s_red[nw + w] : acc.nmn;
    }
    // the largest delegate is the largest element: the k = 1 answer, and the
    // top of the survivors' bucket map in the tail; the smallest delegate key
    // lets the tail clip the cut bin to the keys present
    if (acc.mx) atomicMax((unsigned long long*)&ctl->max1, (unsigned long long)acc.mx);
    if (acc.nmn) atomicMax(&ctl->dknmin, acc.nmn);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) *s_last = (atomicAdd(&ctl->ticketD[0], 1u) == gridDim.x - 1) ? 1 : 0;
  __syncthreads();
  if (!*s_last) return;
  block_select_bucket(ctl->histD[0], kD, s_scan, s_out);
  const uint32_t b0 = s_out[0], r0 = s_out[1], f0 = s_out[2];
  const uint32_t c0 = f0 ? atomic_load_u32(&ctl->histD[0][b0]) : 0xFFFFFFFFu;
  __syncthreads();
  block_select_bucket(ctl->histL, kD, s_scan, s_out);
  const uint32_t b1 = s_out[0], r1 = s_out[1], f1 = s_out[2];
  const uint32_t c1 = f1 ? atomic_load_u32(&ctl->histL[b1]) : 0xFFFFFFFFu;
  if (threadIdx.x == 0) {
    const uint64_t w0 = (uint64_t)(kD - r0) + c0, w1 = (uint64_t)(kD - r1) + c1;
    if (!f0 && !f1) flag_err(ctl, ERR_SELECT);
    const bool use_log = f1 && (!f0 || w1 < w0);
    ctl->wmap = use_log ? 1u : 0u;
    ctl->wbin = use_log ? b1 : b0;
    ctl->wsize = (uint32_t)(use_log ? w1 : w0);
    uint32_t lo = 0, hi = 0;
    bin_interval(ctl->wmap, ctl->wbin, lo, hi);
    ctl->cut_lo = lo;
    ctl->cut_hi = hi;
    ctl->cut_rank = use_log ? r1 : r0;
    ctl->cut_count = (uint32_t)(use_log ? c1 : c0);
    // kept for the multi-pass delegate select (plain-radix fallback path)
    ctl->selD.prefix = (uint64_t)b0 << pass_shift(0);
    ctl->selD.mask = 0x7FFull << pass_shift(0);
    ctl->selD.rank = r0;
    ctl->selD.found = f0;
  }
}

template <int DT, bool VEC>
__device__ __forceinline__ void load4(const uint32_t* __restrict__ keys, uint64_t p, uint32_t v[4]) {
  if constexpr (VEC) {
    u32x4 x = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(keys + p));
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
  } else {
    v[0] = keys[p]; v[1] = keys[p + 1]; v[2] = keys[p + 2]; v[3] = keys[p + 3];
  }
}

constexpr int kUnroll = 8;  // 128-bit loads in flight per lane

// Subranges of >= 256 elements: one wave per subrange, each lane folds its
// elements into a private top-beta, then a butterfly merge across the wave.
// The four waves of a block take the chunk's subranges round-robin (wave w:
// subranges w, w+4, ...), so at any time they stream adjacent memory (a read
// pattern about 3% faster on this device than a contiguous quarter per wave)
// while each subrange stays inside one wave.  The chunk [clo, clo + chunk)
// holds 4 * wlen / 2^alpha subranges; `fast`: all of it lies below n.
template <int DT, int BETA, bool VEC>
__device__ __forceinline__ void delegate_wave(const uint32_t* __restrict__ keys, uint64_t n, int alpha,
                                              uint64_t clo, uint32_t wave, uint64_t wlen, bool fast,
                                              uint32_t* dkey, uint32_t* didx, uint64_t s0, uint32_t* lh,
                                              DelAcc& acc) {
  const uint32_t lane = lane_id();
  const int lw = alpha - 8;
  const uint64_t wps_mask = (1ull << lw) - 1;  // wave-loads per subrange - 1
  const uint64_t nwl = wlen >> 8;
  const uint64_t first = clo + ((uint64_t)wave << alpha);
  TopB<BETA> tb;
  tb.clear();
  for (uint64_t j0 = 0; j0 < nwl; j0 += kUnroll) {
    uint32_t v[kUnroll][4];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const uint64_t j = j0 + u;
      const uint64_t p = first + ((j >> lw) << (alpha + 2)) + ((j & wps_mask) << 8) + lane * 4;
      if (fast) {
        load4<DT, VEC>(keys, p, v[u]);
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) v[u][c] = (j < nwl && p + c < n) ? keys[p + c] : 0u;
      }
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const uint64_t j = j0 + u;
      if (j < nwl) {
        const uint64_t sb = first + ((j >> lw) << (alpha + 2));
        const uint64_t p = sb + ((j & wps_mask) << 8) + lane * 4;
        if constexpr (BETA >= 4) {
          uint64_t x[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) x[c] = (fast || p + c < n) ? comp(enc<DT>(v[u][c]), (uint32_t)(p + c)) : 0ull;
          tb.push4(x[0], x[1], x[2], x[3]);
        } else {
#pragma unroll
          for (int c = 0; c < 4; ++c)
            if (fast || p + c < n) tb.push(comp(enc<DT>(v[u][c]), (uint32_t)(p + c)));
        }
        if (((j + 1) & wps_mask) == 0) {
          merge_lanes<BETA>(tb, 64);
          if (lane == 0 && sb < n) emit_delegates<BETA>((sb >> alpha) - s0, tb, dkey, didx, lh, acc);
          tb.clear();
        }
      }
    }
  }
}

// beta >= 2, subranges of 256..2048 elements: a group of G = 8 lanes owns
// each subrange, so a wave works on 8 subranges at once and each lane folds
// 2^alpha/8 of a subrange's elements before the group's 3-step segmented
// merge.  A load instruction reads 8 segments of 128 contiguous bytes.  (G =
// 2^alpha/64 lanes, i.e. 32 at alpha = 11, took 30 us longer at n = 2^30;
// 16 or 32 at alpha = 10 the same time.)  The chunk's batches of 8
// subranges go to the four waves round-robin (adjacent memory, as in
// delegate_wave); the caller checks that the chunk holds a multiple of 32
// subranges.
template <int DT, int BETA, bool VEC>
__device__ __forceinline__ void grouped_batches(const uint32_t* __restrict__ keys, uint64_t n, int alpha,
                                                uint64_t clo, uint32_t wave, uint64_t chunk, uint32_t* dkey,
                                                uint32_t* didx, uint64_t s0, uint32_t* lh, DelAcc& acc) {
  const uint32_t lane = lane_id();
  const uint32_t L = 1u << alpha;
  const uint32_t G = 8;
  const uint32_t ns = 64 / G;           // subranges per batch of the wave
  const uint32_t g = lane / G, l = lane % G;
  const uint32_t lpl = L / (4 * G);     // 16-byte loads per lane per subrange (2^alpha / 32: 8..64)
  const uint64_t nbatch = (chunk >> alpha) / ns;
  for (uint64_t bi = wave; bi < nbatch; bi += 4) {
    const uint64_t s = (clo >> alpha) + bi * ns + g;
    const uint64_t sbase = s << alpha;
    TopB<BETA> tb;
    tb.clear();
    for (uint32_t i0 = 0; i0 < lpl; i0 += kUnroll) {
      uint32_t v[kUnroll][4];
      const uint64_t p0 = sbase + ((uint64_t)i0 * G + l) * 4;
      if constexpr (BETA == 2) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) load4<DT, VEC>(keys, p0 + (uint64_t)u * G * 4, v[u]);
        // The lane's elements come in increasing position, so a later key
        // equal to a held one ranks below it: the top two of this step's 32
        // keys follow from 32-bit key compares alone, with positions kept as
        // element numbers e (position p0 + (e / 4) * 4G + e % 4), and are
        // folded into the running pair once per step.
        uint32_t a0, a1, r0, r1;
        {
          const uint32_t x0 = enc<DT>(v[0][0]), x1 = enc<DT>(v[0][1]);
          const bool sw = x1 > x0;
          a0 = sw ? x1 : x0;
          r0 = sw ? 1u : 0u;
          a1 = sw ? x0 : x1;
          r1 = sw ? 0u : 1u;
        }
#pragma unroll
        for (int e = 2; e < kUnroll * 4; ++e) {
          const uint32_t x = enc<DT>(v[e >> 2][e & 3]);
          const bool g0 = x > a0, g1 = x > a1;
          r1 = g1 ? (g0 ? r0 : (uint32_t)e) : r1;
          r0 = g0 ? (uint32_t)e : r0;
          // second = median of (a0, a1, x) (one v_med3_u32), first = max
          const uint32_t mn = a0 < a1 ? a0 : a1, mx = a0 > a1 ? a0 : a1;
          const uint32_t hi = mx < x ? mx : x;
          a1 = mn > hi ? mn : hi;
          a0 = a0 > x ? a0 : x;  // a0 >= a1 always
        }
        const uint32_t b0 = (uint32_t)p0, st = 4 * G;
        tb.push(comp(a0, b0 + (r0 >> 2) * st + (r0 & 3)));
        tb.push(comp(a1, b0 + (r1 >> 2) * st + (r1 & 3)));
      } else {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) load4<DT, VEC>(keys, p0 + (uint64_t)u * G * 4, v[u]);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const uint32_t pu = (uint32_t)p0 + (uint32_t)u * G * 4;
          if constexpr (BETA == 8) {
            if (u & 1) continue;  // pairs of loads: u and u + 1
            const uint32_t pv = pu + G * 4;
            uint64_t x[8];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              x[c] = comp(enc<DT>(v[u][c]), pu + c);
              x[4 + c] = comp(enc<DT>(v[u + 1][c]), pv + c);
            }
            tb.push8(x);
          } else if constexpr (BETA >= 4) {
            tb.push4(comp(enc<DT>(v[u][0]), pu), comp(enc<DT>(v[u][1]), pu + 1), comp(enc<DT>(v[u][2]), pu + 2),
                     comp(enc<DT>(v[u][3]), pu + 3));
          } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) tb.push(comp(enc<DT>(v[u][c]), pu + c));
          }
        }
      }
    }
    merge_lanes<BETA>(tb, G);
    if (l == 0) emit_delegates<BETA>(s - s0, tb, dkey, didx, lh, acc);
  }
}


// Subranges of 4..128 elements: 2^(alpha-2) lanes per subrange inside each
// 256-element wave-load; segmented butterfly merge.
template <int DT, int BETA, bool VEC>
__device__ __forceinline__ void delegate_group(const uint32_t* __restrict__ keys, uint64_t n, int alpha,
                                               uint64_t wlo, uint64_t whi, bool fast,
                                               uint32_t* dkey, uint32_t* didx, uint32_t* lh, DelAcc& acc) {
  const uint32_t lane = lane_id();
  const uint32_t gl = 1u << (alpha - 2);  // lanes per subrange
  const uint64_t nwl = (whi + 255 - wlo) >> 8;
  for (uint64_t j0 = 0; j0 < nwl; j0 += kUnroll) {
    uint32_t v[kUnroll][4];
    if (fast) {
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) load4<DT, VEC>(keys, wlo + ((j0 + u) << 8) + lane * 4, v[u]);
    } else {
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const uint64_t p = wlo + ((j0 + u) << 8) + lane * 4;
#pragma unroll
        for (int c = 0; c < 4; ++c) v[u][c] = (j0 + u < nwl && p + c < n) ? keys[p + c] : 0u;
      }
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const uint64_t j = j0 + u;
      if (j < nwl) {
        const uint64_t p = wlo + (j << 8) + lane * 4;
        TopB<BETA> tb;
        tb.clear();
#pragma unroll
        for (int c = 0; c < 4; ++c)
          if (fast || p + c < n) tb.push(comp(enc<DT>(v[u][c]), (uint32_t)(p + c)));
        merge_lanes<BETA>(tb, gl);
        if ((lane & (gl - 1)) == 0 && p < n) emit_delegates<BETA>(p >> alpha, tb, dkey, didx, lh, acc);
      }
    }
  }
}

// Subranges of >= 256 elements of the chunk at clo: grouped lanes (beta >= 2,
// full chunks) or a wave per subrange.  Delegate s goes to entries
// (s - s0) * BETA.. of dkey / didx.
template <int DT, int BETA, bool VEC>
__device__ __forceinline__ void delegate_chunk_wide(const uint32_t* __restrict__ keys, uint64_t n, int alpha,
                                                    uint64_t clo, uint64_t chunk, bool grouped, uint32_t* dkey,
                                                    uint32_t* didx, uint64_t s0, uint32_t* lh, DelAcc& acc) {
  const uint32_t wave = threadIdx.x >> 6;
  // full chunks only: a bounds-checked copy of the unrolled grouped loop
  // would set the register budget of the whole kernel (184 VGPRs against
  // 60: 2 waves per SIMD instead of 8); the last chunk takes delegate_wave
  if (grouped && clo + chunk <= n)
    grouped_batches<DT, BETA, VEC>(keys, n, alpha, clo, wave, chunk, dkey, didx, s0, lh, acc);
  else
    delegate_wave<DT, BETA, VEC>(keys, n, alpha, clo, wave, chunk >> 2, clo + chunk <= n, dkey, didx, s0, lh, acc);
}

constexpr uint32_t kDBuf = 512;  // delegates a block keeps in LDS until its end (occupancy: 7 waves per SIMD)

// One block per chunk of `chunk` elements (a multiple of 4 * 2^alpha and of
// 4 * 256 * kUnroll); each wave streams a contiguous quarter of the chunk.
// With subranges of >= 256 elements and at most kDBuf delegates in the
// chunk, the delegates collect in LDS and leave in one coalesced copy at the
// end: stores issued between the loads would hold up each later wait for
// loads, since one counter tracks both on this GPU.
template <int DT, int BETA, bool VEC>
__global__ __launch_bounds__(256) void k_delegate(const uint32_t* __restrict__ keys, uint64_t n, int alpha,
                                                  uint64_t chunk, uint32_t* __restrict__ dkey,
                                                  uint32_t* __restrict__ didx, Ctl* ctl, uint32_t k, DirectOut out) {
  __shared__ uint32_t lh[2 * kBins];
  __shared__ uint32_t s_scan[256];
  __shared__ uint32_t s_out[4];
  __shared__ int s_last;
  __shared__ uint64_t s_red[8];
  __shared__ uint32_t s_dk[kDBuf], s_di[kDBuf];
  for (int i = threadIdx.x; i < 2 * kBins; i += 256) lh[i] = 0;
  __syncthreads();
  DelAcc acc;
  const uint32_t wave = threadIdx.x >> 6;
  const uint64_t wlen = chunk >> 2;
  const uint64_t clo = (uint64_t)blockIdx.x * chunk;
  const uint64_t wlo = clo + wave * wlen;
  const uint64_t gspan = alpha >= 8 && alpha <= 11 ? 8ull << alpha : 0;  // 64 / G subranges per wave batch
  const bool grouped = BETA >= 2 && gspan && wlen % gspan == 0;
  const uint64_t s0 = clo >> alpha;
  const bool lds_out = alpha >= 8 && clo < n && (chunk >> alpha) * BETA <= kDBuf;  // block-uniform
  if (alpha >= 8) {
    if (lds_out)
      delegate_chunk_wide<DT, BETA, VEC>(keys, n, alpha, clo, chunk, grouped, s_dk, s_di, s0, lh, acc);
    else if (clo < n)
      delegate_chunk_wide<DT, BETA, VEC>(keys, n, alpha, clo, chunk, grouped, dkey, didx, 0, lh, acc);
  } else if (wlo < n) {
    const uint64_t whi = wlo + wlen < n ? wlo + wlen : n;
    const bool fast = (wlo + wlen <= n);
    delegate_group<DT, BETA, VEC>(keys, n, alpha, wlo, whi, fast, dkey, didx, lh, acc);
  }
  __syncthreads();
  if (lds_out) {
    // the chunk's subranges below n: S - s0 of them in the last chunk
    const uint64_t S = (n + (1ull << alpha) - 1) >> alpha;
    const uint64_t ns = (chunk >> alpha) < S - s0 ? (chunk >> alpha) : S - s0;
    for (uint32_t i = threadIdx.x; i < (uint32_t)(ns * BETA); i += 256) {
      dkey[s0 * BETA + i] = s_dk[i];
      didx[s0 * BETA + i] = s_di[i];
    }
  }
  finish_delegates(lh, ctl, k, s_scan, s_out, &s_last, acc, s_red);
  if (out.on && s_last && threadIdx.x == 0) write_out<DT>(ld_coh64(&ctl->max1), 0, 1, out.vals, out.idx, out.kth);
}

// Subranges of 1 or 2 elements, or any alpha when the planner asks for the
// simple form: one thread per subrange.
template <int DT, int BETA>
__global__ __launch_bounds__(256) void k_delegate_thread(const uint32_t* __restrict__ keys, uint64_t n,
                                                         int alpha, uint64_t S, uint32_t* __restrict__ dkey,
                                                         uint32_t* __restrict__ didx, Ctl* ctl, uint32_t k,
                                                         DirectOut out) {
  __shared__ uint32_t lh[2 * kBins];
  __shared__ uint32_t s_scan[256];
  __shared__ uint32_t s_out[4];
  __shared__ int s_last;
  __shared__ uint64_t s_red[8];
  for (int i = threadIdx.x; i < 2 * kBins; i += 256) lh[i] = 0;
  __syncthreads();
  DelAcc acc;
  for (uint64_t s = (uint64_t)blockIdx.x * 256 + threadIdx.x; s < S; s += (uint64_t)gridDim.x * 256) {
    TopB<BETA> tb;
    tb.clear();
    const uint64_t lo = s << alpha;
    const uint64_t hi = (lo + (1ull << alpha)) < n ? lo + (1ull << alpha) : n;
    for (uint64_t p = lo; p < hi; ++p) tb.push(comp(enc<DT>(keys[p]), (uint32_t)p));
    emit_delegates<BETA>(s, tb, dkey, didx, lh, acc);
  }
  __syncthreads();
  finish_delegates(lh, ctl, k, s_scan, s_out, &s_last, acc, s_red);
  if (out.on && s_last && threadIdx.x == 0) write_out<DT>(ld_coh64(&ctl->max1), 0, 1, out.vals, out.idx, out.kth);
}

// ---------------------------------------------------------------------------
// one digit of an MSD radix select over composites

template <int SRC, int DT>
__device__ __forceinline__ uint32_t src_key(const uint32_t* key, uint64_t i) {
  if constexpr (SRC == SRC_V) return enc<DT>(key[i]);
  else return key[i];
}
template <int SRC>
__device__ __forceinline__ uint32_t src_pos(const uint32_t* idx, uint64_t i) {
  if constexpr (SRC == SRC_V) return (uint32_t)i;
  else return idx[i];
}

// gate: 0 always run, 1 run only if survivors <= kSmallCap, 2 only if > kSmallCap
__device__ __forceinline__ bool gated_off(const Ctl* ctl, int gate) {
  if (gate == 0) return false;
  const bool small = clamp_nc(ctl) <= (uint32_t)kSmallCap;
  return gate == 1 ? !small : small;
}

template <int SRC, int DT>
__global__ __launch_bounds__(256) void k_pass(const uint32_t* __restrict__ key, const uint32_t* __restrict__ idx,
                                              uint64_t count_static, int p, int gate, Ctl* ctl, uint32_t k) {
  __shared__ uint32_t lh[kBins];
  __shared__ uint32_t s_scan[256];
  __shared__ uint32_t s_out[4];
  __shared__ int s_last;
  if (gated_off(ctl, gate)) return;
  const bool isD = (SRC == SRC_D);
  Sel* sel = isD ? &ctl->selD : &ctl->selC;
  uint32_t* gh = isD ? ctl->histD[p] : ctl->histC[p];
  uint32_t* ticket = isD ? &ctl->ticketD[p] : &ctl->ticketC[p];
  const uint64_t count = (SRC == SRC_C) ? (uint64_t)clamp_nc(ctl) : count_static;
  uint64_t prefix = 0, mask = 0;
  if (p > 0) { prefix = sel->prefix; mask = sel->mask; }
  for (int i = threadIdx.x; i < kBins; i += 256) lh[i] = 0;
  __syncthreads();
  const int sh = pass_shift(p);
  const uint32_t dm = (1u << pass_bits(p)) - 1;
  const uint32_t kmask = (uint32_t)(mask >> 32), kpref = (uint32_t)(prefix >> 32);
  const uint32_t imask = (uint32_t)mask, ipref = (uint32_t)prefix;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (uint64_t)gridDim.x * 256) {
    const uint32_t kk = src_key<SRC, DT>(key, i);
    if ((kk & kmask) != kpref) continue;
    uint64_t c = (uint64_t)kk << 32;
    if (p >= 3) {
      const uint32_t ip = ~src_pos<SRC>(idx, i);
      if ((ip & imask) != ipref) continue;
      c |= ip;
    }
    atomicAdd(&lh[(uint32_t)(c >> sh) & dm], 1u);
  }
  __syncthreads();
  flush_hist(lh, gh);
  finish_pass(gh, ticket, sel, p, k, ctl, s_scan, s_out, &s_last);
}

// ---------------------------------------------------------------------------
// Rule 3 per subrange: re-read s only if its beta-th delegate ranks strictly
// above the threshold t; otherwise keep its delegates that rank at or above t.

template <int BETA>
__global__ __launch_bounds__(256) void k_qualify(const uint32_t* __restrict__ dkey, const uint32_t* __restrict__ didx,
                                                 uint64_t S, Ctl* ctl, uint32_t* __restrict__ Q,
                                                 uint32_t* __restrict__ ckey, uint32_t* __restrict__ cidx) {
  __shared__ Stage<1024> sq;
  __shared__ Stage<4096> sc;
  stage_init(sq);
  stage_init(sc);
  const uint64_t t = ctl->all ? 0ull : ctl->selD.prefix;
  const uint32_t cap_q = ctl->cap_q, cap_c = ctl->cap_c;
  for (uint64_t s0 = (uint64_t)blockIdx.x * 256; s0 < S; s0 += (uint64_t)gridDim.x * 256) {
    const uint64_t s = s0 + threadIdx.x;
    const bool ok = s < S;
    uint64_t dc = 0;
    if (ok) dc = comp(dkey[s * BETA + BETA - 1], didx[s * BETA + BETA - 1]);
    const bool scan = ok && dc > t;
    stage_push(sq, scan, (uint32_t)s, 0u);
#pragma unroll
    for (int j = 0; j < BETA; ++j) {
      uint64_t c = 0;
      if (ok && !scan) c = comp(dkey[s * BETA + j], didx[s * BETA + j]);
      const bool take = c != 0 && c >= t;
      stage_push(sc, take, comp_key(c), comp_pos(c));
    }
    stage_flush(sq, &ctl->nq, cap_q, Q, nullptr, ctl, false, 256);
    stage_flush(sc, &ctl->nc, cap_c, ckey, cidx, ctl, false, 256 * BETA);
  }
  stage_flush(sq, &ctl->nq, cap_q, Q, nullptr, ctl, true, 0);
  stage_flush(sc, &ctl->nc, cap_c, ckey, cidx, ctl, true, 0);
}

// The paper's concatenated vector, never materialised: element e of the
// concatenation of the qualifying subranges is position
// Q[e >> alpha] * 2^alpha + (e & (2^alpha - 1)).  Each thread takes 4
// consecutive elements (one 128-bit load when alpha >= 2), so work is spread
// evenly whatever the subrange size; elements ranked at or above t survive
// (Rule 2's filter, inclusive).
template <int DT, bool VEC>
__global__ __launch_bounds__(256) void k_scan(const uint32_t* __restrict__ keys, uint64_t n, int alpha, Ctl* ctl,
                                              const uint32_t* __restrict__ Q, uint32_t* __restrict__ ckey,
                                              uint32_t* __restrict__ cidx) {
  __shared__ Stage<4096> sc;
  stage_init(sc);
  const uint64_t total = (uint64_t)clamp_nq(ctl) << alpha;
  const uint32_t cap_c = ctl->cap_c;
  const uint64_t t = ctl->all ? 0ull : ctl->selD.prefix;
  const uint64_t lmask = (1ull << alpha) - 1;
  for (uint64_t e0 = (uint64_t)blockIdx.x * 1024; e0 < total; e0 += (uint64_t)gridDim.x * 1024) {
    const uint64_t e = e0 + threadIdx.x * 4;
    uint32_t v[4];
    uint64_t pos[4];
    bool in[4];
    if (VEC && alpha >= 2) {
      const uint64_t p = e < total ? ((uint64_t)Q[e >> alpha] << alpha) + (e & lmask) : n;
#pragma unroll
      for (int c = 0; c < 4; ++c) { pos[c] = p + c; in[c] = p + c < n; }
      if (p + 4 <= n) {
        load4<DT, true>(keys, p, v);
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) v[c] = in[c] ? keys[p + c] : 0u;
      }
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const uint64_t ec = e + c;
        pos[c] = ec < total ? ((uint64_t)Q[ec >> alpha] << alpha) + (ec & lmask) : n;
        in[c] = pos[c] < n;
        v[c] = in[c] ? keys[pos[c]] : 0u;
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const uint64_t cc = comp(enc<DT>(v[c]), (uint32_t)pos[c]);
      stage_push(sc, in[c] && cc >= t, comp_key(cc), (uint32_t)pos[c]);
    }
    stage_flush(sc, &ctl->nc, cap_c, ckey, cidx, ctl, false, 1024);
  }
  stage_flush(sc, &ctl->nc, cap_c, ckey, cidx, ctl, true, 0);
}

// ---------------------------------------------------------------------------
// outputs

template <int SRC, int DT>
__device__ __forceinline__ uint64_t src_comp(const uint32_t* key, const uint32_t* idx, uint64_t i) {
  return comp(src_key<SRC, DT>(key, i), src_pos<SRC>(idx, i));
}


// One workgroup: all `count` (<= kSmallCap) entries sorted in LDS, first k written.
template <int SRC, int DT>
__global__ __launch_bounds__(1024) void k_final_small(const uint32_t* __restrict__ key,
                                                      const uint32_t* __restrict__ idx, uint64_t count_static,
                                                      int gate, uint32_t k, Ctl* ctl, uint32_t* out_vals,
                                                      uint32_t* out_idx, uint32_t* out_kth) {
  __shared__ uint64_t buf[kSmallCap];
  if (gated_off(ctl, gate)) return;
  const uint64_t count = (SRC == SRC_C) ? (uint64_t)clamp_nc(ctl) : count_static;
  if (count > (uint64_t)kSmallCap || count < k) {
    if (threadIdx.x == 0) flag_err(ctl, ERR_FEW);
    return;
  }
  uint32_t P = 64;
  while (P < count) P <<= 1;
  for (uint32_t i = threadIdx.x; i < P; i += 1024) buf[i] = i < count ? src_comp<SRC, DT>(key, idx, i) : 0ull;
  __syncthreads();
  for (uint32_t size = 2; size <= P; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t i = threadIdx.x; i < (P >> 1); i += 1024) {
        const uint32_t lo = 2 * i - (i & (stride - 1));
        const uint32_t hi = lo + stride;
        const bool desc = (lo & size) == 0;
        const uint64_t a = buf[lo], b = buf[hi];
        if ((a < b) == desc) { buf[lo] = b; buf[hi] = a; }
      }
      __syncthreads();
    }
  }
  for (uint32_t r = threadIdx.x; r < k; r += 1024) write_out<DT>(buf[r], r, k, out_vals, out_idx, out_kth);
}

// Exactly the k entries ranked at or above the k-th (selC) -> okey/oidx.
template <int SRC, int DT>
__global__ __launch_bounds__(256) void k_compact(const uint32_t* __restrict__ key, const uint32_t* __restrict__ idx,
                                                 uint64_t count_static, int gate, uint32_t k, Ctl* ctl,
                                                 uint32_t* __restrict__ okey, uint32_t* __restrict__ oidx) {
  __shared__ Stage<2048> so;
  if (gated_off(ctl, gate)) return;
  stage_init(so);
  const uint64_t count = (SRC == SRC_C) ? (uint64_t)clamp_nc(ctl) : count_static;
  const uint64_t T = ctl->selC.prefix;
  for (uint64_t i0 = (uint64_t)blockIdx.x * 1024; i0 < count; i0 += (uint64_t)gridDim.x * 1024) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const uint64_t i = i0 + c * 256 + threadIdx.x;
      uint64_t x = 0;
      if (i < count) x = src_comp<SRC, DT>(key, idx, i);
      stage_push(so, i < count && x >= T, comp_key(x), comp_pos(x));
    }
    stage_flush(so, &ctl->nout, k, okey, oidx, ctl, false, 1024);
  }
  stage_flush(so, &ctl->nout, k, okey, oidx, ctl, true, 0);
}

// k-th value straight from the survivor select (k-selection needs no sort).
template <int DT>
__global__ void k_kth_from_sel(int gate, Ctl* ctl, uint32_t* out_kth) {
  if (gated_off(ctl, gate) || !out_kth) return;
  if (threadIdx.x == 0 && blockIdx.x == 0) *out_kth = dec<DT>((uint32_t)(ctl->selC.prefix >> 32));
}

// Sort tiles of kSortTile composites in LDS (descending); pads are 0.
static __global__ __launch_bounds__(1024) void k_blocksort(const uint32_t* __restrict__ okey,
                                                    const uint32_t* __restrict__ oidx, uint32_t k,
                                                    uint64_t* __restrict__ A, int gated, const Ctl* ctl) {
  __shared__ uint64_t buf[kSortTile];
  if (gated && !ctl->need_merge) return;
  const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
  for (uint32_t j = threadIdx.x; j < kSortTile; j += 1024) {
    const uint64_t i = base + j;
    buf[j] = i < k ? comp(okey[i], oidx[i]) : 0ull;
  }
  __syncthreads();
  for (uint32_t size = 2; size <= kSortTile; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t i = threadIdx.x; i < kSortTile / 2; i += 1024) {
        const uint32_t lo = 2 * i - (i & (stride - 1));
        const uint32_t hi = lo + stride;
        const bool desc = (lo & size) == 0;
        const uint64_t a = buf[lo], b = buf[hi];
        if ((a < b) == desc) { buf[lo] = b; buf[hi] = a; }
      }
      __syncthreads();
    }
  }
  for (uint32_t j = threadIdx.x; j < kSortTile; j += 1024) A[base + j] = buf[j];
}

// Merge pairs of sorted runs of length `run` by rank: an element's output slot
// is its slot in its own run plus the number of partner-run elements placed
// before it (strictly greater for the left run, greater-or-equal for the right
// run, so equal pads stay stable).  The last merge writes the outputs.
template <int DT>
__global__ __launch_bounds__(256) void k_merge(const uint64_t* __restrict__ A, uint64_t* __restrict__ B, uint64_t M,
                                               uint64_t run, int last, uint32_t k, uint32_t* out_vals,
                                               uint32_t* out_idx, uint32_t* out_kth, int gated, const Ctl* ctl) {
  if (gated && !ctl->need_merge) return;
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= M) return;
  const uint64_t pair = i / (2 * run) * (2 * run);
  const uint64_t within = i - pair;
  const bool left = within < run;
  const uint64_t own = left ? within : within - run;
  const uint64_t* other = A + (left ? pair + run : pair);
  const uint64_t x = A[i];
  uint64_t lo = 0, hi = run;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    const uint64_t y = other[mid];
    const bool before = left ? (y > x) : (y >= x);
    if (before) lo = mid + 1;
    else hi = mid;
  }
  const uint64_t out = pair + own + lo;
  if (last) {
    if (out < k) write_out<DT>(x, (uint32_t)out, k, out_vals, out_idx, out_kth);
  } else {
    B[out] = x;
  }
}

static __global__ void k_init(Ctl* ctl, uint32_t cap_q, uint32_t cap_c, uint32_t all, uint32_t* rec) {
  uint32_t* w = reinterpret_cast<uint32_t*>(ctl);
  const uint32_t nw = offsetof(Ctl, cap_q) / 4;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nw; i += gridDim.x * blockDim.x) w[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->cap_q = cap_q;
    ctl->cap_c = cap_c;
    ctl->all = all;
    ctl->rec = rec;
  }
}

}  // namespace drtopk
