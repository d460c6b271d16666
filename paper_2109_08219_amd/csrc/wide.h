// Kernels of the delegate-centric top-k for 64-bit keys (uint64, int64,
// float64).
//
// The paper's selections run on key-value pairs (Section 5.1); here the key
// itself is 64 bits wide.  Every element is compared as a 96-bit composite
//     c = (encoded_key << 32) | ~position
// held in an unsigned __int128, so the order is key descending, then position
// ascending, exactly as for 32-bit keys, and the composite of padding (key 0,
// position 0xFFFFFFFF) is 0, below every element.
//
//   k_wdelegate  the one streaming pass over V: per subrange of 2^alpha keys
//                (alpha >= 7) its maximum composite (Rule 1), 128-bit loads
//   k_wpass      one 12-bit MSD digit of an exact radix select over 96-bit
//                composites (at most 8 passes; it stops as soon as the sought
//                rank's bucket holds a single composite)
//   k_wfind      the selected composite itself once its bucket is unique
//   k_wqualify   subranges whose delegate ranks at or above t (Rules 1-2)
//   k_wscan      re-reads those subranges as one virtual concatenated vector
//                and keeps the elements ranked at or above t
//   k_wfinal     few survivors: one workgroup sorts them and writes the k first
//   k_wcompact / k_wsort / k_wblocksort / k_wmerge   exact k, then sorted
// Work after the delegate pass is enqueued in full; a kernel that the
// device-side state shows to be unneeded returns at once.
#pragma once

#include "internal.h"

namespace drtopk {

typedef unsigned __int128 u128;
typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

constexpr int kWBins = 4096;       // 12-bit digits
constexpr int kWPasses = 8;        // 8 x 12 bits = the 96-bit composite
constexpr int kWSmall = 4096;      // composites one workgroup sorts in LDS
constexpr int kWThreads = 256;
constexpr int kWSortThreads = 1024;

// Runtime key codec: enc(b) = b ^ (sign(b) & a) ^ c maps the input's bit
// pattern to an unsigned key with the same order (uint64: a = c = 0; int64:
// c = 2^63; float64 by totalOrder: a = 2^63 - 1, c = 2^63; the k smallest
// complement c).
struct Codec64 {
  uint64_t a, c;
};

__device__ __forceinline__ uint64_t enc64(uint64_t b, Codec64 cd) {
  const uint64_t s = (uint64_t)((int64_t)b >> 63);
  return b ^ (s & cd.a) ^ cd.c;
}
__device__ __forceinline__ uint64_t dec64(uint64_t u, Codec64 cd) {
  const uint64_t x = u ^ cd.c;
  const uint64_t s = (uint64_t)((int64_t)x >> 63);
  return x ^ (s & cd.a);
}

__device__ __forceinline__ u128 wcomp(uint64_t key, uint32_t pos) {
  return ((u128)key << 32) | (u128)(uint32_t)~pos;
}
__device__ __forceinline__ uint64_t wkey(u128 c) { return (uint64_t)(c >> 32); }
__device__ __forceinline__ uint32_t wpos(u128 c) { return ~(uint32_t)c; }
__device__ __forceinline__ u128 wmax(u128 a, u128 b) { return a > b ? a : b; }

constexpr int wshift(int pass) { return 84 - 12 * pass; }

// Exact selection state over composites.
struct WSel {
  u128 prefix;    // composite bits fixed so far
  u128 mask;      // which bits are fixed
  u128 t;         // the selected composite (valid once `done`, after k_wfind)
  uint32_t rank;  // 1-based rank still sought among composites matching prefix
  uint32_t done;  // the sought bucket is unique (or every bit is fixed)
  uint32_t pad[2];
};

// Per-call control block at the head of the workspace; zeroed by k_winit.
struct WCtl {
  uint32_t hist[2][kWPasses][kWBins];  // [0] delegate select, [1] survivor (or whole-input) select
  uint32_t ticket[2][kWPasses];
  WSel sel[2];
  uint32_t nq;        // qualifying subranges
  uint32_t nc;        // survivors
  uint32_t no;        // compacted outputs
  uint32_t finished;  // outputs already written (few survivors)
  uint32_t err;
  uint32_t cap_q, cap_c;
  uint32_t pad;
  uint32_t* rec;  // the stream's check record
};

__device__ __forceinline__ void wflag(WCtl* c, uint32_t bit) {
  atomicOr(&c->err, bit);
  record_err(c->rec, bit);
}

__global__ void k_winit(WCtl* ctl, uint32_t cap_q, uint32_t cap_c, uint32_t* rec) {
  uint32_t* w = reinterpret_cast<uint32_t*>(ctl);
  const uint32_t nw = offsetof(WCtl, cap_q) / 4;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nw; i += gridDim.x * blockDim.x) w[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->cap_q = cap_q;
    ctl->cap_c = cap_c;
    ctl->rec = rec;
  }
}

// Maximum composite over the wave, held by every lane (VALU lane operations).
template <int M>
__device__ __forceinline__ u128 wmax_cross(u128 c) {
  const uint32_t w0 = (uint32_t)c, w1 = (uint32_t)(c >> 32), w2 = (uint32_t)(c >> 64);
  const u128 o = ((u128)lane_cross32<M>(w2) << 64) | ((u128)lane_cross32<M>(w1) << 32) | lane_cross32<M>(w0);
  return wmax(c, o);
}
__device__ __forceinline__ u128 wave_max128(u128 c) {
  c = wmax_cross<1>(c);
  c = wmax_cross<2>(c);
  c = wmax_cross<4>(c);
  c = wmax_cross<8>(c);
  c = wmax_cross<16>(c);
  return wmax_cross<32>(c);
}

// ---------------------------------------------------------------------------
// Delegate pass.  One workgroup per chunk of `chunk` keys (a multiple of
// 4 * 1024 and of 2^alpha); wave w streams the w-th quarter of the chunk in
// steps of 1024 keys (eight 16-byte loads in flight per lane).  A wave-load
// covers 128 contiguous keys, never two subranges (2^alpha >= 128), so each
// lane folds the keys of the current subrange into a running maximum and the
// wave reduces it when the subrange ends.  A lane visits its positions in
// increasing order, so a later equal key never displaces the held one: the
// fold needs the key comparison only, the position rides along.
template <bool VEC>
__device__ __forceinline__ void wload2(const uint64_t* keys, uint64_t p, uint64_t& a, uint64_t& b) {
  if constexpr (VEC) {
    const u64x2 x = __builtin_nontemporal_load(reinterpret_cast<const u64x2*>(keys + p));
    a = x.x;
    b = x.y;
  } else {
    a = __builtin_nontemporal_load(keys + p);
    b = __builtin_nontemporal_load(keys + p + 1);
  }
}

template <bool VEC>
__global__ __launch_bounds__(kWThreads) void k_wdelegate(const uint64_t* __restrict__ keys, uint64_t n, int alpha,
                                                         uint64_t chunk, Codec64 cd, uint64_t* dkey,
                                                         uint32_t* didx) {
  constexpr int U = 8;
  const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
  const uint64_t L = 1ull << alpha;
  const uint64_t wlen = chunk >> 2;
  const uint64_t wlo = (uint64_t)blockIdx.x * chunk + wave * wlen;
  if (wlo >= n) return;
  if (wlo + wlen <= n) {
    uint64_t bk = 0;
    uint32_t bp = kInvalid;
    for (uint64_t j = 0; j < wlen; j += 128 * U) {
      uint64_t v[U][2];
#pragma unroll
      for (int u = 0; u < U; ++u) wload2<VEC>(keys, wlo + j + u * 128 + lane * 2, v[u][0], v[u][1]);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint64_t p = wlo + j + u * 128 + lane * 2;
        const uint64_t e0 = enc64(v[u][0], cd), e1 = enc64(v[u][1], cd);
        if (e0 > bk || bp == kInvalid) { bk = e0; bp = (uint32_t)p; }
        if (e1 > bk) { bk = e1; bp = (uint32_t)p + 1; }
        const uint64_t end = j + (uint64_t)(u + 1) * 128;  // offset in the wave's range after this load
        if ((end & (L - 1)) == 0) {                        // wave-uniform: a subrange ends here
          const u128 m = wave_max128(wcomp(bk, bp));
          if (lane == 0) {
            const uint64_t s = (wlo + end - 1) >> alpha;
            dkey[s] = wkey(m);
            didx[s] = wpos(m);
          }
          bk = 0;
          bp = kInvalid;
        }
      }
    }
    return;
  }
  // the part of the last chunk below n: subrange by subrange, bounds-checked
  const uint64_t hi = n;
  for (uint64_t s0 = wlo; s0 < wlo + wlen && s0 < hi; s0 += L) {
    u128 best = 0;
    const uint64_t se = s0 + L < hi ? s0 + L : hi;
    for (uint64_t p = s0 + lane; p < se; p += 64) best = wmax(best, wcomp(enc64(keys[p], cd), (uint32_t)p));
    best = wave_max128(best);
    if (lane == 0) {
      dkey[s0 >> alpha] = wkey(best);
      didx[s0 >> alpha] = wpos(best);
    }
  }
}

// ---------------------------------------------------------------------------
// Exact radix select over composites.  SRC 0: the input V (keys encoded at
// load, positions implicit); 1: explicit arrays of encoded keys and positions
// whose count is *count (clamped to cap).

template <int SRC>
__device__ __forceinline__ u128 wentry(const uint64_t* key, const uint32_t* pos, uint64_t i, Codec64 cd) {
  if constexpr (SRC == 0) return wcomp(enc64(key[i], cd), (uint32_t)i);
  else return wcomp(key[i], pos[i]);
}

// Bin holding the rank-th largest entry of a 4096-bin global histogram (each
// of the 256 threads owns 16 consecutive bins, highest first):
// out = {bin, rank within the bin, found, count of the bin}.
__device__ inline void wbucket(const uint32_t* gh, uint32_t rank, uint32_t* s_wsum, uint32_t* out) {
  constexpr int PER = kWBins / kWThreads;  // 16
  const int t = threadIdx.x;
  const uint32_t lane = lane_id(), wave = t >> 6;
  uint32_t c[PER], sum = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    c[j] = ld_coh(&gh[kWBins - 1 - PER * t - j]);
    sum += c[j];
  }
  uint32_t x = sum;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)x, o);
    if ((int)lane >= o) x += y;
  }
  if (lane == 63) s_wsum[wave] = x;
  if (t == 0) { out[0] = 0; out[1] = 0; out[2] = 0; out[3] = 0; }
  __syncthreads();
  uint32_t excl = x - sum;
  for (uint32_t w = 0; w < wave; ++w) excl += s_wsum[w];
  if (excl < rank && rank <= excl + sum) {
    uint32_t cum = excl;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      if (cum + c[j] >= rank) {
        out[0] = kWBins - 1 - PER * t - j;
        out[1] = rank - cum;
        out[2] = 1;
        out[3] = c[j];
        break;
      }
      cum += c[j];
    }
  }
  __syncthreads();
}

template <int SRC>
__global__ __launch_bounds__(kWThreads) void k_wpass(const uint64_t* __restrict__ key,
                                                     const uint32_t* __restrict__ pos, uint64_t n,
                                                     const uint32_t* count, uint32_t cap, Codec64 cd, int pass,
                                                     uint32_t rank0, int which, WCtl* ctl) {
  WSel* sel = &ctl->sel[which];
  if (ctl->finished || (pass > 0 && sel->done)) return;
  __shared__ uint32_t lh[kWBins];
  __shared__ uint32_t s_wsum[kWThreads / 64];
  __shared__ uint32_t s_out[4];
  __shared__ int s_last;
  for (int i = threadIdx.x; i < kWBins; i += kWThreads) lh[i] = 0;
  __syncthreads();
  const u128 prefix = pass ? sel->prefix : 0, mask = pass ? sel->mask : 0;
  if (count) {
    const uint32_t c = *count;
    n = c < cap ? c : cap;
  }
  const int sh = wshift(pass);
  for (uint64_t i = (uint64_t)blockIdx.x * kWThreads + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kWThreads) {
    const u128 c = wentry<SRC>(key, pos, i, cd);
    if ((c & mask) == prefix) atomicAdd(&lh[(uint32_t)(c >> sh) & (kWBins - 1)], 1u);
  }
  __syncthreads();
  uint32_t* gh = ctl->hist[which][pass];
  for (int i = threadIdx.x; i < kWBins; i += kWThreads)
    if (lh[i]) atomicAdd(&gh[i], lh[i]);
  // each wave waits for its own histogram atomics before the ticket; the last
  // block then reads the histogram with coherent loads
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) s_last = (atomicAdd(&ctl->ticket[which][pass], 1u) == gridDim.x - 1) ? 1 : 0;
  __syncthreads();
  if (!s_last) return;
  const uint32_t rank = pass ? sel->rank : rank0;
  wbucket(gh, rank, s_wsum, s_out);
  if (threadIdx.x == 0) {
    const u128 dm = (u128)(kWBins - 1) << sh;
    sel->prefix = prefix | ((u128)s_out[0] << sh);
    sel->mask = mask | dm;
    sel->rank = s_out[1];
    if (!s_out[2]) {
      wflag(ctl, ERR_SELECT);
      sel->done = 1;
    } else if (s_out[3] == 1 || pass == kWPasses - 1) {
      sel->done = 1;
    }
  }
}

// The selected composite: with every bit fixed it is the prefix; otherwise
// it is the one entry matching the prefix.
template <int SRC>
__global__ __launch_bounds__(kWThreads) void k_wfind(const uint64_t* __restrict__ key,
                                                     const uint32_t* __restrict__ pos, uint64_t n,
                                                     const uint32_t* count, uint32_t cap, Codec64 cd, int which,
                                                     WCtl* ctl) {
  WSel* sel = &ctl->sel[which];
  if (ctl->finished) return;
  if (!sel->done) {
    if (blockIdx.x == 0 && threadIdx.x == 0) wflag(ctl, ERR_SELECT);
    return;
  }
  const u128 prefix = sel->prefix, mask = sel->mask;
  const u128 all = ((u128)1 << 96) - 1;
  if (mask == all) {
    if (blockIdx.x == 0 && threadIdx.x == 0) sel->t = prefix;
    return;
  }
  if (count) {
    const uint32_t c = *count;
    n = c < cap ? c : cap;
  }
  for (uint64_t i = (uint64_t)blockIdx.x * kWThreads + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kWThreads) {
    const u128 c = wentry<SRC>(key, pos, i, cd);
    if ((c & mask) == prefix) sel->t = c;
  }
}

// Appends staged in LDS: the lanes of a wave take consecutive stage slots
// with one LDS atomic, and the block reserves global space with one device
// atomic per flush (a single global counter taking an atomic per wave is
// what the device serialises).  Entries at or past cap are dropped and
// flagged.
constexpr uint32_t kWStage = 2048;
struct WStage {
  uint64_t key[kWStage];
  uint32_t idx[kWStage];
  uint32_t n;
  uint32_t base;
};

__device__ __forceinline__ void wstage_init(WStage& S) {
  if (threadIdx.x == 0) S.n = 0;
  __syncthreads();
}

// Whole wave active.
__device__ __forceinline__ void wstage_push(WStage& S, bool pred, uint64_t k, uint32_t p) {
  const uint64_t b = __ballot(pred);
  if (!b) return;
  const int leader = __ffsll((unsigned long long)b) - 1;
  uint32_t off = 0;
  if ((int)lane_id() == leader) off = atomicAdd(&S.n, (uint32_t)__popcll(b));
  off = (uint32_t)__shfl((int)off, leader) + mbcnt(b);
  if (pred) {
    S.key[off] = k;
    S.idx[off] = p;
  }
}

// Block-uniform: flushes when `force` or when fewer than kWThreads slots are
// left (one more step of the block could fill them).  gidx may be null.
__device__ inline void wstage_flush(WStage& S, uint32_t* counter, uint32_t cap, uint64_t* gkey, uint32_t* gidx,
                                    WCtl* ctl, bool force) {
  __syncthreads();
  const uint32_t n = S.n;
  const bool doit = n != 0 && (force || n + kWThreads > kWStage);
  __syncthreads();
  if (!doit) return;
  if (threadIdx.x == 0) S.base = atomicAdd(counter, n);
  __syncthreads();
  const uint32_t base = S.base;
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
    if (base + i < cap) {
      gkey[base + i] = S.key[i];
      if (gidx) gidx[base + i] = S.idx[i];
    } else {
      wflag(ctl, ERR_CAP);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) S.n = 0;
  __syncthreads();
}

// Subranges whose delegate ranks at or above t: the only ones that can hold
// an element of the answer other than t itself (Rule 1 with Rule 2's t).
__global__ __launch_bounds__(kWThreads) void k_wqualify(const uint64_t* __restrict__ dkey,
                                                        const uint32_t* __restrict__ didx, uint64_t S, WCtl* ctl,
                                                        uint32_t* Q) {
  __shared__ uint32_t sq[kWStage];
  __shared__ uint32_t sn, sbase;
  if (threadIdx.x == 0) sn = 0;
  __syncthreads();
  const u128 t = ctl->sel[0].t;
  const uint32_t cap = ctl->cap_q;
  const uint64_t stride = (uint64_t)gridDim.x * kWThreads;
  for (uint64_t b = (uint64_t)blockIdx.x * kWThreads;; b += stride) {
    const bool more = b < S;
    if (more) {
      const uint64_t s = b + threadIdx.x;
      const bool q = s < S && wcomp(dkey[s], didx[s]) >= t;
      const uint64_t m = __ballot(q);
      if (m) {
        const int leader = __ffsll((unsigned long long)m) - 1;
        uint32_t off = 0;
        if ((int)lane_id() == leader) off = atomicAdd(&sn, (uint32_t)__popcll(m));
        off = (uint32_t)__shfl((int)off, leader) + mbcnt(m);
        if (q) sq[off] = (uint32_t)s;
      }
    }
    __syncthreads();
    const uint32_t n = sn;
    if (n != 0 && (!more || n + kWThreads > kWStage)) {
      __syncthreads();
      if (threadIdx.x == 0) sbase = atomicAdd(&ctl->nq, n);
      __syncthreads();
      for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        if (sbase + i < cap) Q[sbase + i] = sq[i];
        else wflag(ctl, ERR_CAP);
      }
      __syncthreads();
      if (threadIdx.x == 0) sn = 0;
    }
    __syncthreads();
    if (!more) break;
  }
}

// Re-read of the qualifying subranges as one virtual vector: element e is
// position Q[e >> alpha] * 2^alpha + (e mod 2^alpha); elements ranked at or
// above t survive.
__global__ __launch_bounds__(kWThreads) void k_wscan(const uint64_t* __restrict__ keys, uint64_t n, int alpha,
                                                     Codec64 cd, const uint32_t* __restrict__ Q, WCtl* ctl,
                                                     uint64_t* ckey, uint32_t* cidx) {
  __shared__ WStage st;
  wstage_init(st);
  const u128 t = ctl->sel[0].t;
  const uint32_t nq = ctl->nq < ctl->cap_q ? ctl->nq : ctl->cap_q;
  const uint64_t total = (uint64_t)nq << alpha, mask = (1ull << alpha) - 1;
  const uint64_t stride = (uint64_t)gridDim.x * kWThreads;
  const uint32_t cap = ctl->cap_c;
  for (uint64_t b = (uint64_t)blockIdx.x * kWThreads; b < total; b += stride) {
    const uint64_t e = b + threadIdx.x;
    bool keep = false;
    uint64_t k = 0;
    uint32_t p = 0;
    if (e < total) {
      const uint64_t q = ((uint64_t)Q[e >> alpha] << alpha) | (e & mask);
      if (q < n) {
        k = enc64(keys[q], cd);
        p = (uint32_t)q;
        keep = wcomp(k, p) >= t;
      }
    }
    wstage_push(st, keep, k, p);
    wstage_flush(st, &ctl->nc, cap, ckey, cidx, ctl, false);
  }
  wstage_flush(st, &ctl->nc, cap, ckey, cidx, ctl, true);
}

// LDS bitonic sort, descending, of P (power of two) composites.
__device__ inline void wlds_sort(u128* buf, uint32_t P) {
  for (uint32_t size = 2; size <= P; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t i = threadIdx.x; i < (P >> 1); i += blockDim.x) {
        const uint32_t lo = 2 * i - (i & (stride - 1));
        const uint32_t hi = lo + stride;
        const bool desc = (lo & size) == 0;
        const u128 a = buf[lo], b = buf[hi];
        if ((a < b) == desc) { buf[lo] = b; buf[hi] = a; }
      }
      __syncthreads();
    }
  }
}

__device__ __forceinline__ void wwrite_out(u128 c, uint32_t r, uint32_t k, Codec64 cd, uint64_t* out_vals,
                                           uint32_t* out_idx, uint64_t* out_kth) {
  const uint64_t v = dec64(wkey(c), cd);
  if (out_vals) out_vals[r] = v;
  if (out_idx) out_idx[r] = wpos(c);
  if (out_kth && r == k - 1) *out_kth = v;
}

// Few survivors (at most kWSmall): one workgroup sorts them all and writes the
// first k; the select over the survivors is then skipped.
__global__ __launch_bounds__(kWSortThreads) void k_wfinal(const uint64_t* __restrict__ ckey,
                                                          const uint32_t* __restrict__ cidx, uint32_t k, Codec64 cd,
                                                          WCtl* ctl, uint64_t* out_vals, uint32_t* out_idx,
                                                          uint64_t* out_kth) {
  const uint32_t nc = ctl->nc;
  if (nc > (uint32_t)kWSmall || nc > ctl->cap_c) return;
  __shared__ u128 buf[kWSmall];
  if (nc < k) {  // cannot happen: t ranks k-th among the delegates, so at least k elements rank >= t
    if (threadIdx.x == 0) wflag(ctl, ERR_FEW);
  }
  uint32_t P = 1;
  while (P < nc) P <<= 1;
  for (uint32_t i = threadIdx.x; i < P; i += blockDim.x) buf[i] = i < nc ? wcomp(ckey[i], cidx[i]) : (u128)0;
  __syncthreads();
  wlds_sort(buf, P);
  const uint32_t m = nc < k ? nc : k;
  for (uint32_t r = threadIdx.x; r < m; r += blockDim.x) wwrite_out(buf[r], r, k, cd, out_vals, out_idx, out_kth);
  if (threadIdx.x == 0) ctl->finished = 1;
}

// k-th value alone from a finished select.
__global__ void k_wkth(int which, Codec64 cd, WCtl* ctl, uint64_t* out_kth) {
  if (ctl->finished) return;
  if (threadIdx.x == 0) *out_kth = dec64(wkey(ctl->sel[which].t), cd);
}

// The k entries ranked at or above the selected composite T, unordered.
template <int SRC>
__global__ __launch_bounds__(kWThreads) void k_wcompact(const uint64_t* __restrict__ key,
                                                        const uint32_t* __restrict__ pos, uint64_t n,
                                                        const uint32_t* count, uint32_t cap, Codec64 cd, int which,
                                                        uint32_t k, WCtl* ctl, uint64_t* okey, uint32_t* oidx) {
  if (ctl->finished) return;
  __shared__ WStage st;
  wstage_init(st);
  const u128 T = ctl->sel[which].t;
  if (count) {
    const uint32_t c = *count;
    n = c < cap ? c : cap;
  }
  const uint64_t stride = (uint64_t)gridDim.x * kWThreads;
  for (uint64_t b = (uint64_t)blockIdx.x * kWThreads; b < n; b += stride) {
    const uint64_t i = b + threadIdx.x;
    bool keep = false;
    u128 c = 0;
    if (i < n) {
      c = wentry<SRC>(key, pos, i, cd);
      keep = c >= T;
    }
    wstage_push(st, keep, wkey(c), wpos(c));
    wstage_flush(st, &ctl->no, k, okey, oidx, ctl, false);
  }
  wstage_flush(st, &ctl->no, k, okey, oidx, ctl, true);
}

// Sort of the k compacted outputs, k <= kWSmall: one workgroup.
__global__ __launch_bounds__(kWSortThreads) void k_wsort(const uint64_t* __restrict__ okey,
                                                         const uint32_t* __restrict__ oidx, uint32_t k, Codec64 cd,
                                                         WCtl* ctl, uint64_t* out_vals, uint32_t* out_idx,
                                                         uint64_t* out_kth) {
  if (ctl->finished) return;
  __shared__ u128 buf[kWSmall];
  if (threadIdx.x == 0 && ctl->no != k) wflag(ctl, ERR_FEW);
  uint32_t P = 1;
  while (P < k) P <<= 1;
  for (uint32_t i = threadIdx.x; i < P; i += blockDim.x) buf[i] = i < k ? wcomp(okey[i], oidx[i]) : (u128)0;
  __syncthreads();
  wlds_sort(buf, P);
  for (uint32_t r = threadIdx.x; r < k; r += blockDim.x) wwrite_out(buf[r], r, k, cd, out_vals, out_idx, out_kth);
}

// Larger k: tiles of kWSmall sorted in LDS into A (padded with 0 up to M) ...
__global__ __launch_bounds__(kWSortThreads) void k_wblocksort(const uint64_t* __restrict__ okey,
                                                              const uint32_t* __restrict__ oidx, uint32_t k,
                                                              WCtl* ctl, u128* A) {
  if (ctl->finished) return;
  __shared__ u128 buf[kWSmall];
  if (blockIdx.x == 0 && threadIdx.x == 0 && ctl->no != k) wflag(ctl, ERR_FEW);
  const uint64_t base = (uint64_t)blockIdx.x * kWSmall;
  for (uint32_t i = threadIdx.x; i < (uint32_t)kWSmall; i += blockDim.x) {
    const uint64_t g = base + i;
    buf[i] = g < k ? wcomp(okey[g], oidx[g]) : (u128)0;
  }
  __syncthreads();
  wlds_sort(buf, kWSmall);
  for (uint32_t i = threadIdx.x; i < (uint32_t)kWSmall; i += blockDim.x) A[base + i] = buf[i];
}

// ... then runs of `run` merged pairwise: an entry's slot in the merged run is
// its index in its own run plus the number of entries of the other run ranked
// above it (entries of the left run win ties, which only padding zeros have).
// The last merge writes the decoded outputs.
__global__ __launch_bounds__(kWThreads) void k_wmerge(const u128* __restrict__ A, u128* B, uint64_t M, uint64_t run,
                                                      int last, uint32_t k, Codec64 cd, WCtl* ctl, uint64_t* out_vals,
                                                      uint32_t* out_idx, uint64_t* out_kth) {
  if (ctl->finished) return;
  const uint64_t i = (uint64_t)blockIdx.x * kWThreads + threadIdx.x;
  if (i >= M) return;
  const uint64_t pair = i / (2 * run), base = pair * 2 * run;
  const bool left = (i - base) < run;
  const uint64_t own = left ? i - base : i - base - run;
  const u128* other = A + (left ? base + run : base);
  const u128 x = A[i];
  // count of the other run ranked above x (left) or at or above x (right)
  uint64_t lo = 0, hi = run;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    const bool above = left ? other[mid] > x : other[mid] >= x;
    if (above) lo = mid + 1;
    else hi = mid;
  }
  const uint64_t slot = own + lo;
  if (last) {
    if (slot < k) wwrite_out(x, (uint32_t)slot, k, cd, out_vals, out_idx, out_kth);
  } else {
    B[base + slot] = x;
  }
}

}  // namespace drtopk
