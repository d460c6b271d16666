// Many independent top-k problems in one persistent launch.
//
// Each workgroup (kBT threads) takes whole problems from an atomic counter,
// largest first (the host orders them), and runs the delegate method for one
// problem entirely in its LDS:
//   delegate vector (Rules 1 and 3): the top beta (1 or 2) of each subrange
//     of 2^alpha keys, built in LDS by waves streaming the keys;
//   t = the k-th largest delegate: an LDS radix select over the delegates;
//   survivors (Rules 2 and 3): t itself, every element ranked >= t in the
//     subranges whose last delegate ranks above t (read as one virtual
//     concatenated vector), and with beta = 2 the first delegates above t of
//     the other subranges;
//   output: survivors sorted in registers, the first k written.
// Problems of at most kBSmallN keys are selected in LDS directly (the k-th
// by radix select, then the k at or above it sorted).  A problem whose
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
constexpr uint32_t kBSmallN = 4096;       // problems this small are selected in LDS directly
constexpr uint32_t kBMaxS = 4096;         // delegate vector capacity (LDS)
constexpr uint32_t kBMaxSG = 32768;       // delegate vector of a split problem (global memory)
constexpr uint32_t kBSurv = 4096;         // survivor capacity (LDS)
constexpr uint32_t kBMaxK = 2048;         // largest k handled in a workgroup
constexpr uint64_t kBMaxN = 1ull << 22;   // largest n handled in a workgroup
constexpr int kBU = 8;                    // 1 KiB wave loads in flight per wave step
constexpr uint32_t kBStep = 256 * kBU;    // keys per wave step
constexpr int kBufWord3 = 0x00020000;     // buffer resource word 3 for gfx9-family raw buffers
constexpr uint64_t kBSplitMinN = 1u << 16;  // problems above this may keep their delegate vector in global memory
constexpr uint32_t kBTileLog = 18;        // a split problem's delegate vector is built in tiles of
                                          // 2^max(kBTileLog, alpha) keys, one workgroup each (fewer where a
                                          // tile's delegates would not fit its LDS: at most 4096 entries)
__host__ __device__ constexpr uint32_t tile_log(uint32_t alpha, uint32_t beta) {
  return alpha + 12 - (beta > 1 ? 1 : 0) < kBTileLog ? alpha + 12 - (beta > 1 ? 1 : 0)
                                                     : (alpha > kBTileLog ? alpha : kBTileLog);
}

// One problem as the kernel sees it (64 bytes).
struct BatchDesc {
  const uint32_t* keys;
  uint64_t n;
  uint32_t k;
  uint32_t dtype;
  uint16_t alpha;  // subrange exponent, >= 2; 0 = radix select without delegates
  uint16_t beta;   // delegates per subrange (Rule 3): 1 or 2
  uint32_t tiles;  // > 1: the delegate vector is built by this many workgroups
  uint32_t* out_vals;
  uint32_t* out_idx;
  uint32_t* out_kth;
  uint64_t doff;   // tiles > 1: offset of the problem's delegate vector in the global buffer
};
static_assert(sizeof(BatchDesc) == 64, "BatchDesc layout");

struct BatchSmem {
  uint64_t D[kBMaxS];     // delegate composites; also the exchange buffer of small sorts
  uint64_t surv[kBSurv];  // survivors, also the exchange buffer of their sort
  uint32_t hist[kBins];   // digit histograms; then the list of qualifying subranges
  uint32_t wsum[kBWaves];
  uint32_t wbig[kBWaves];
  uint64_t red[2 * kBWaves];
  uint64_t sel;
  uint64_t tail_del;      // delegate of the subrange holding the last n mod 4 keys
  uint32_t nsurv;
  uint32_t nq;
  uint32_t item;
  uint32_t out[4];
};

template <int M>
__device__ __forceinline__ uint64_t max_cross(uint64_t m) {
  const uint64_t y = lane_cross64<M>(m);
  return y > m ? y : m;
}
// Maximum over each block of G consecutive lanes (G a wave-uniform power of
// two, at most 64), held by all of its lanes; VALU lane operations only.
__device__ __forceinline__ uint64_t group_max64(uint64_t m, uint32_t G) {
  if (G > 1) m = max_cross<1>(m);
  if (G > 2) m = max_cross<2>(m);
  if (G > 4) m = max_cross<4>(m);
  if (G > 8) m = max_cross<8>(m);
  if (G > 16) m = max_cross<16>(m);
  if (G > 32) m = max_cross<32>(m);
  return m;
}
__device__ __forceinline__ uint64_t wave_max64(uint64_t m) {
  return max_cross<32>(max_cross<16>(max_cross<8>(max_cross<4>(max_cross<2>(max_cross<1>(m))))));
}

// The top BETA (1 or 2) of a stream of distinct composites, m1 > m2 (0 =
// none yet; 0 is below every composite of a real element, so pushing it
// changes nothing).
template <int BETA>
__device__ __forceinline__ void top_push(uint64_t& m1, uint64_t& m2, uint64_t x) {
  if constexpr (BETA == 2) {
    const uint64_t lo = x < m1 ? x : m1;
    m2 = lo > m2 ? lo : m2;
  }
  m1 = x > m1 ? x : m1;
}
template <int BETA>
__device__ __forceinline__ void top_merge(uint64_t& m1, uint64_t& m2, uint64_t b1, uint64_t b2) {
  if constexpr (BETA == 2) {
    const uint64_t lo = b1 < m1 ? b1 : m1;
    const uint64_t hi2 = b2 > m2 ? b2 : m2;
    m2 = lo > hi2 ? lo : hi2;
  }
  m1 = b1 > m1 ? b1 : m1;
}
template <int BETA, int M>
__device__ __forceinline__ void top_cross(uint64_t& m1, uint64_t& m2) {
  const uint64_t b1 = lane_cross64<M>(m1);
  const uint64_t b2 = BETA == 2 ? lane_cross64<M>(m2) : 0ull;
  top_merge<BETA>(m1, m2, b1, b2);
}
// Top BETA over each block of G consecutive lanes (G a wave-uniform power of
// two, at most 64), held by all of its lanes.
template <int BETA>
__device__ __forceinline__ void group_top(uint64_t& m1, uint64_t& m2, uint32_t G) {
  if (G > 1) top_cross<BETA, 1>(m1, m2);
  if (G > 2) top_cross<BETA, 2>(m1, m2);
  if (G > 4) top_cross<BETA, 4>(m1, m2);
  if (G > 8) top_cross<BETA, 8>(m1, m2);
  if (G > 16) top_cross<BETA, 16>(m1, m2);
  if (G > 32) top_cross<BETA, 32>(m1, m2);
}

// Folds a block's top BETA (m1 > m2) into subrange j of an LDS delegate
// vector of BETA entries per subrange (zeroed first).  BETA 1: an atomic
// maximum.  BETA 2: m1 goes into the first entry by an atomic maximum, and
// the larger of m2 and whichever of m1 and the displaced value is smaller
// into the second.  Each update of the first entry hands the smaller of its
// two values to the second, so every value except the overall maximum
// reaches the second entry once: it ends as the runner-up in any order of
// updates.
template <int BETA>
__device__ __forceinline__ void d_fold(uint64_t* D, uint32_t j, uint64_t m1, uint64_t m2) {
  if constexpr (BETA == 1) {
    atomicMax((unsigned long long*)&D[j], (unsigned long long)m1);
  } else {
    const uint64_t old = atomicMax((unsigned long long*)&D[2 * j], (unsigned long long)m1);
    const uint64_t lo = old < m1 ? old : m1;
    const uint64_t v = lo > m2 ? lo : m2;
    if (v) atomicMax((unsigned long long*)&D[2 * j + 1], (unsigned long long)v);
  }
}

// The keys of one problem behind a raw buffer resource: loads are plain
// buffer loads (base address in scalar registers, 32-bit offsets), and whole
// dwords at or beyond `nrec` keys read 0.  VEC: 16-byte loads of 4 keys at a
// multiple of 4 (the base is 16-byte aligned and nrec a multiple of 4, so a
// load is either wholly inside or wholly outside); otherwise 4-byte loads.
template <bool VEC>
struct Keys {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ Keys(const uint32_t* p, uint32_t nrec)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t*>(p), (short)0, (int)(nrec * 4u), kBufWord3)) {}
  __device__ __forceinline__ void load4(uint32_t p, uint32_t (&v)[4]) const {
    if constexpr (VEC) {
      const u32x4 x = __builtin_amdgcn_raw_buffer_load_b128(r, (int)(p * 4u), 0, 0);
      v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) v[c] = __builtin_amdgcn_raw_buffer_load_b32(r, (int)((p + c) * 4u), 0, 0);
    }
  }
};

// Keys [0, n4) go through the streaming loops; with 16-byte loads n4 = n
// rounded down to a multiple of 4 and the last n - n4 keys are read one by one.
template <bool VEC>
__device__ __forceinline__ uint32_t vec_end(uint32_t n) {
  return VEC ? (n & ~3u) : n;
}

// Bin holding the rank-th largest entry of an LDS histogram (each thread owns
// kBins / kBT consecutive bins, highest first; wave prefix sums, one barrier):
// sm.out = {bin, rank within the bin, found, count of the bin}.
__device__ inline void bb_bucket(const uint32_t* h, uint32_t rank, BatchSmem& sm) {
  constexpr int PER = kBins / kBT;
  const int t = threadIdx.x;
  const uint32_t lane = lane_id(), wave = t >> 6;
  uint32_t c[PER], sum = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    c[j] = h[kBins - 1 - PER * t - j];
    sum += c[j];
  }
  uint32_t x = sum;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)x, o);
    if ((int)lane >= o) x += y;
  }
  if (lane == 63) sm.wsum[wave] = x;
  if (t == 0) { sm.out[0] = 0; sm.out[1] = 0; sm.out[2] = 0; sm.out[3] = 0; }
  __syncthreads();
  uint32_t excl = x - sum;
  for (uint32_t w = 0; w < wave; ++w) excl += sm.wsum[w];
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

// Key codec of a batched problem, applied at run time so one kernel serves
// batches that mix key types and orders: enc(b) = b ^ (sign(b) & a) ^ c
// equals enc<DT> of the problem's codec (float32: a = 0x7FFFFFFF, c = the
// sign bit; int32: a = 0, c = the sign bit; uint32: both 0; the k smallest:
// c complemented).  a leaves bit 31 alone, so b ^ (sign(b) & a) keeps b's
// sign and dec recovers b from it.
struct Codec {
  uint32_t a, c;
  __device__ __forceinline__ uint32_t enc(uint32_t b) const {
    return b ^ ((uint32_t)((int32_t)b >> 31) & a) ^ c;
  }
  __device__ __forceinline__ uint32_t dec(uint32_t e) const {
    const uint32_t v = e ^ c;
    return v ^ ((uint32_t)((int32_t)v >> 31) & a);
  }
};
__device__ __forceinline__ Codec codec_of(uint32_t code) {
  Codec x;
  x.a = (code & 3u) == (uint32_t)DT_F32 ? 0x7FFFFFFFu : 0u;
  x.c = ((code & 3u) == (uint32_t)DT_U32 ? 0u : 0x80000000u) ^ ((code & (uint32_t)DT_MIN) ? 0xFFFFFFFFu : 0u);
  return x;
}
__device__ __forceinline__ void b_write_out(uint64_t c, uint32_t r, uint32_t k, uint32_t* out_vals, uint32_t* out_idx,
                                            uint32_t* out_kth, Codec cx) {
  const uint32_t v = cx.dec(comp_key(c));
  if (out_vals) out_vals[r] = v;
  if (out_idx) out_idx[r] = comp_pos(c);
  if (out_kth && r == k - 1) *out_kth = v;
}

// Wave-wide append to an LDS list: the lanes with `pred` take consecutive
// slots from *count with one LDS atomic per wave (whole wave active); slots at
// or past cap are counted but not stored.
__device__ __forceinline__ void lds_append(bool pred, uint64_t x, uint32_t* count, uint64_t* list, uint32_t cap) {
  const uint64_t b = __ballot(pred);
  if (!b) return;
  const int leader = __ffsll((unsigned long long)b) - 1;
  uint32_t base = 0;
  if ((int)lane_id() == leader) base = atomicAdd(count, (uint32_t)__popcll(b));
  base = (uint32_t)__shfl((int)base, leader) + mbcnt(b);
  if (pred && base < cap) list[base] = x;
}

// Sorts `cnt` composites from LDS array `src` and writes the first `k` as
// outputs 0..k-1.  `src` holds at least E * kBT entries and serves as the
// exchange buffer of the sort once every thread has loaded its elements.
template <int E>
__device__ __noinline__ void b_sort_write_e(uint64_t* src, uint32_t cnt, uint32_t k, uint32_t* out_vals,
                                            uint32_t* out_idx, uint32_t* out_kth, Codec cx) {
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
    if (g < k) b_write_out(v[e], g, k, out_vals, out_idx, out_kth, cx);
  }
}

// Bucket-rank sort of the cnt (<= E * kBT) distinct composites src[0..cnt),
// writing the first k as outputs: the composites are binned by the top 11
// bits of their distance from the smallest (bin 0 holds the largest),
// counted in `bins` (kBins words), scattered bin by bin into `buf`, and each
// takes the slot (start of its bin) + (number of larger composites in its
// bin).  Gives up (false, nothing written) when a bin holds more than
// kRankMaxBin: keys crowded into a narrow range go to the network instead.
template <int E>
__device__ __noinline__ bool b_rank_write_e(const uint64_t* src, uint32_t cnt, uint32_t k, uint32_t* out_vals,
                                            uint32_t* out_idx, uint32_t* out_kth, Codec cx, uint64_t* buf,
                                            uint32_t* bins, BatchSmem& sm) {
  constexpr int NW = kBWaves, PER = kBins / kBT;
  const uint32_t t = threadIdx.x, lane = lane_id(), w = t >> 6;
  uint64_t v[E];
  uint64_t mx = 0, nmn = 0;  // largest composite, and the complement of the smallest
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint32_t g = e * kBT + t;
    v[e] = g < cnt ? src[g] : 0ull;
    if (g < cnt) {
      mx = v[e] > mx ? v[e] : mx;
      nmn = ~v[e] > nmn ? ~v[e] : nmn;
    }
  }
  mx = wave_max64(mx);
  nmn = wave_max64(nmn);
  __syncthreads();  // src may alias the reduction slots' neighbours: every load done
  if (lane == 0) {
    sm.red[w] = mx;
    sm.red[NW + w] = nmn;
  }
  for (int i = t; i < kBins; i += kBT) bins[i] = 0;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    mx = sm.red[i] > mx ? sm.red[i] : mx;
    nmn = sm.red[NW + i] > nmn ? sm.red[NW + i] : nmn;
  }
  const uint64_t lo = ~nmn;
  const uint32_t bits = bitlen64(mx - lo);
  const uint32_t sh = bits > 11u ? bits - 11u : 0u;
  uint32_t b[E], r[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint32_t g = e * kBT + t;
    b[e] = (uint32_t)(kBins - 1) - (uint32_t)((v[e] - lo) >> sh);
    r[e] = g < cnt ? atomicAdd(&bins[b[e]], 1u) : 0u;
  }
  __syncthreads();
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
    const uint32_t y = (uint32_t)__shfl_up((int)inc, d);
    if (lane >= d) inc += y;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const uint32_t y = (uint32_t)__shfl_xor((int)big, o);
    big = y > big ? y : big;
  }
  if (lane == 63) sm.wsum[w] = inc;
  if (lane == 0) sm.wbig[w] = big;
  __syncthreads();
  uint32_t off = inc - sum;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    if ((uint32_t)i < w) off += sm.wsum[i];
    big = sm.wbig[i] > big ? sm.wbig[i] : big;
  }
  if (big > kRankMaxBin) {  // block-uniform
    __syncthreads();
    return false;
  }
  __syncthreads();  // every count read before it becomes a bin start
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    bins[t * PER + j] = off;
    off += c[j];
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < E; ++e)
    if (e * kBT + t < cnt) buf[bins[b[e]] + r[e]] = v[e];
  __syncthreads();
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (e * kBT + t >= cnt) continue;
    const uint32_t st = bins[b[e]], en = b[e] + 1 < (uint32_t)kBins ? bins[b[e] + 1] : cnt;
    uint32_t slot = st;
    for (uint32_t j = st; j < en; ++j) slot += buf[j] > v[e] ? 1u : 0u;
    if (slot < k) b_write_out(v[e], slot, k, out_vals, out_idx, out_kth, cx);
  }
  __syncthreads();  // the caller reuses the LDS
  return true;
}

// cnt <= kBT * 8, k <= cnt.  `buf` (cnt entries) and `bins` (kBins words) are
// free LDS that the bucket-rank sort may use; src must not alias them.
__device__ inline void b_sort_write(uint64_t* src, uint32_t cnt, uint32_t k, uint32_t* out_vals, uint32_t* out_idx,
                                    uint32_t* out_kth, Codec cx, uint64_t* buf, uint32_t* bins, BatchSmem& sm) {
  if (cnt > 1u * kBT) {
    bool done;
    if (cnt <= 2u * kBT) done = b_rank_write_e<2>(src, cnt, k, out_vals, out_idx, out_kth, cx, buf, bins, sm);
    else if (cnt <= 4u * kBT) done = b_rank_write_e<4>(src, cnt, k, out_vals, out_idx, out_kth, cx, buf, bins, sm);
    else done = b_rank_write_e<8>(src, cnt, k, out_vals, out_idx, out_kth, cx, buf, bins, sm);
    if (done) return;
  }
  if (cnt <= 1u * kBT) b_sort_write_e<1>(src, cnt, k, out_vals, out_idx, out_kth, cx);
  else if (cnt <= 2u * kBT) b_sort_write_e<2>(src, cnt, k, out_vals, out_idx, out_kth, cx);
  else if (cnt <= 4u * kBT) b_sort_write_e<4>(src, cnt, k, out_vals, out_idx, out_kth, cx);
  else b_sort_write_e<8>(src, cnt, k, out_vals, out_idx, out_kth, cx);
}

// The rank-th largest (1-based) of the distinct composites a[0..cnt) in LDS:
// MSD radix select, one 11/11/10-bit digit per pass, stopping once the class
// holding rank r has a single member.  Identical in every thread.
__device__ inline uint64_t lds_select(const uint64_t* a, uint32_t cnt, uint32_t rank, BatchSmem& sm) {
  uint64_t prefix = 0, mask = 0;
  uint32_t r = rank;
  for (int p = 0; p < kPasses; ++p) {
    for (int i = threadIdx.x; i < kBins; i += kBT) sm.hist[i] = 0;
    __syncthreads();
    const int sh = pass_shift(p);
    const uint32_t dm = (1u << pass_bits(p)) - 1;
    for (uint32_t i = threadIdx.x; i < cnt; i += kBT) {
      const uint64_t x = a[i];
      if ((x & mask) == prefix) atomicAdd(&sm.hist[(uint32_t)(x >> sh) & dm], 1u);
    }
    __syncthreads();
    bb_bucket(sm.hist, r, sm);
    prefix |= (uint64_t)sm.out[0] << sh;
    mask |= (uint64_t)dm << sh;
    r = sm.out[1];
    if (sm.out[3] == 1u) break;  // always so after the last digit
  }
  for (uint32_t i = threadIdx.x; i < cnt; i += kBT) {
    const uint64_t x = a[i];
    if ((x & mask) == prefix) sm.sel = x;  // the class's single member
  }
  __syncthreads();
  const uint64_t t = sm.sel;
  __syncthreads();
  return t;
}

// Problems of at most kBSmallN keys: composites into LDS, the k-th by radix
// select, the k at or above it compacted and sorted.
template <bool VEC>
__device__ inline void b_small(const BatchDesc& d, BatchSmem& sm) {
  const Codec cx = codec_of(d.dtype);
  const uint32_t n = (uint32_t)d.n, k = d.k, n4 = vec_end<VEC>(n);
  const Keys<VEC> ks(d.keys, n4);
  for (uint32_t i = threadIdx.x * 4; i < n4; i += kBT * 4) {
    uint32_t v[4];
    ks.load4(i, v);
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (i + c < n4) sm.surv[i + c] = comp(cx.enc(v[c]), i + c);
  }
  if (threadIdx.x == 0)
    for (uint32_t i = n4; i < n; ++i) sm.surv[i] = comp(codec_of(d.dtype).enc(d.keys[i]), i);
  __syncthreads();
  uint32_t cnt = n;
  uint64_t* src = sm.surv;
  if (k < n) {
    const uint64_t T = lds_select(sm.surv, n, k, sm);
    if (threadIdx.x == 0) sm.nsurv = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n; i += kBT) {
      const uint64_t x = sm.surv[i];
      if (x >= T) sm.D[atomicAdd(&sm.nsurv, 1u)] = x;  // exactly k
    }
    __syncthreads();
    cnt = k;
    src = sm.D;
  }
  b_sort_write(src, cnt, k, d.out_vals, d.out_idx, d.out_kth, codec_of(d.dtype), src == sm.D ? sm.surv : sm.D,
               sm.hist, sm);
}

// Block-level MSD radix select over the problem's 64-bit composites: each
// pass histograms one digit of the elements in the current class (those
// matching the digits chosen so far) and picks the bin holding rank r.  As
// soon as the elements ranked above the class plus the class itself fit the
// LDS, they are compacted, sorted and the first k written: two passes over
// the keys for typical inputs, at most seven for massive ties.
template <bool VEC>
__device__ inline void b_radix(const BatchDesc& d, BatchSmem& sm, uint32_t* rec) {
  const Codec cx = codec_of(d.dtype);
  const uint32_t n = (uint32_t)d.n, k = d.k, n4 = vec_end<VEC>(n);
  const Keys<VEC> ks(d.keys, n4);
  const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
  uint64_t prefix = 0, mask = 0;
  uint32_t r = k, above = 0;
  for (int p = 0; p < kPasses; ++p) {
    for (int i = threadIdx.x; i < kBins; i += kBT) sm.hist[i] = 0;
    __syncthreads();
    const int sh = pass_shift(p);
    const uint32_t dm = (1u << pass_bits(p)) - 1;
    for (uint32_t base = wave * kBStep; base < n4; base += kBWaves * kBStep) {
      uint32_t v[kBU][4];
#pragma unroll
      for (int j = 0; j < kBU; ++j) ks.load4(base + j * 256 + lane * 4, v[j]);
#pragma unroll
      for (int j = 0; j < kBU; ++j)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const uint32_t i = base + j * 256 + lane * 4 + c;
          const uint64_t x = comp(cx.enc(v[j][c]), i);
          if (i < n4 && (x & mask) == prefix) atomicAdd(&sm.hist[(uint32_t)(x >> sh) & dm], 1u);
        }
    }
    if (threadIdx.x == 0)
      for (uint32_t i = n4; i < n; ++i) {
        const uint64_t x = comp(codec_of(d.dtype).enc(d.keys[i]), i);
        if ((x & mask) == prefix) atomicAdd(&sm.hist[(uint32_t)(x >> sh) & dm], 1u);
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
  for (uint32_t base = wave * kBStep; base < n4; base += kBWaves * kBStep) {
    uint32_t v[kBU][4];
#pragma unroll
    for (int j = 0; j < kBU; ++j) ks.load4(base + j * 256 + lane * 4, v[j]);
#pragma unroll
    for (int j = 0; j < kBU; ++j)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const uint32_t i = base + j * 256 + lane * 4 + c;
        const uint64_t x = comp(cx.enc(v[j][c]), i);
        lds_append(i < n4 && (x & mask) >= prefix, x, &sm.nsurv, sm.surv, kBSurv);
      }
  }
  if (threadIdx.x == 0)
    for (uint32_t i = n4; i < n; ++i) {
      const uint64_t x = comp(codec_of(d.dtype).enc(d.keys[i]), i);
      if ((x & mask) >= prefix) {
        const uint32_t slot = atomicAdd(&sm.nsurv, 1u);
        if (slot < kBSurv) sm.surv[slot] = x;
      }
    }
  __syncthreads();
  const uint32_t ns = sm.nsurv < kBSurv ? sm.nsurv : kBSurv;
  // the class chosen last fits by construction (a single member after the last digit)
  if (threadIdx.x == 0 && sm.nsurv > kBSurv) record_err(rec, ERR_CAP);
  b_sort_write(sm.surv, ns, k, d.out_vals, d.out_idx, d.out_kth, codec_of(d.dtype), sm.D, sm.hist, sm);
}

// Delegate vector for subranges of at least 256 keys, over the keys
// [lo, min(hi, n4)) (lo a multiple of kBStep and of 2^alpha): waves stream
// them in steps of kBStep with kBU 1 KiB loads in flight; each 256-key block
// lies inside one subrange s, whose BETA entries (from sm.D[(s - lo /
// 2^alpha) * BETA]) take the block's top BETA by LDS atomics (D starts at 0,
// below every composite of a real element).
template <bool VEC, int BETA>
__device__ inline void b_delegates_wide(const Keys<VEC>& ks, uint32_t lo, uint32_t hi, uint32_t n4, uint32_t alpha,
                                        Codec cx, BatchSmem& sm) {
  const uint32_t L = 1u << alpha;
  const uint32_t end = hi < n4 ? hi : n4;
  const uint32_t s0 = lo >> alpha;
  const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
  for (uint32_t base = lo + wave * kBStep; base < end; base += kBWaves * kBStep) {
    uint32_t v[kBU][4];
#pragma unroll
    for (int j = 0; j < kBU; ++j) ks.load4(base + j * 256 + lane * 4, v[j]);
    if (L >= kBStep) {
      uint64_t m1 = 0, m2 = 0;
#pragma unroll
      for (int j = 0; j < kBU; ++j)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const uint32_t p = base + j * 256 + lane * 4 + c;
          const uint64_t x = comp(cx.enc(v[j][c]), p);
          top_push<BETA>(m1, m2, p < end ? x : 0ull);
        }
      group_top<BETA>(m1, m2, 64);
      if (lane == 0) d_fold<BETA>(sm.D, (base >> alpha) - s0, m1, m2);
    } else {
#pragma unroll
      for (int j = 0; j < kBU; ++j) {
        uint64_t m1 = 0, m2 = 0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const uint32_t p = base + j * 256 + lane * 4 + c;
          const uint64_t x = comp(cx.enc(v[j][c]), p);
          top_push<BETA>(m1, m2, p < end ? x : 0ull);
        }
        group_top<BETA>(m1, m2, 64);
        if (lane == 0 && base + j * 256 < end) d_fold<BETA>(sm.D, ((base + j * 256) >> alpha) - s0, m1, m2);
      }
    }
  }
}

// The last n mod 4 keys (16-byte loads stop at n4), all in one subrange:
// one thread folds them into that subrange's delegates (index n4 / 2^alpha - s0).
template <int BETA>
__device__ __forceinline__ void b_delegates_tail(const BatchDesc& d, uint32_t n4, uint32_t s0, BatchSmem& sm) {
  const uint32_t n = (uint32_t)d.n;
  if (threadIdx.x == 0 && n4 < n) {
    uint64_t m1 = 0, m2 = 0;
    for (uint32_t i = n4; i < n; ++i) top_push<BETA>(m1, m2, comp(codec_of(d.dtype).enc(d.keys[i]), i));
    d_fold<BETA>(sm.D, (n4 >> d.alpha) - s0, m1, m2);
  }
}

// Delegate vector for subranges of 4..128 keys, over the keys
// [lo, min(hi, n4)) (lo a multiple of kBStep): each 256-key wave-load holds
// whole subranges, 2^(alpha-2) lanes each; a segmented butterfly gives each
// subrange's top BETA to its first lane, which folds them into entries
// (s - lo / 2^alpha) * BETA.. of sm.D.
template <bool VEC, int BETA>
__device__ inline void b_delegates_narrow(const Keys<VEC>& ks, uint32_t lo, uint32_t hi, uint32_t n4,
                                          uint32_t alpha, Codec cx, BatchSmem& sm) {
  const uint32_t G = 1u << (alpha - 2);  // lanes per subrange
  const uint32_t end = hi < n4 ? hi : n4;
  const uint32_t s0 = lo >> alpha;
  const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
  for (uint32_t base = lo + wave * kBStep; base < end; base += kBWaves * kBStep) {
    uint32_t v[kBU][4];
#pragma unroll
    for (int j = 0; j < kBU; ++j) ks.load4(base + j * 256 + lane * 4, v[j]);
#pragma unroll
    for (int j = 0; j < kBU; ++j) {
      const uint32_t p = base + j * 256 + lane * 4;
      uint64_t m1 = 0, m2 = 0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const uint64_t x = comp(cx.enc(v[j][c]), p + c);
        top_push<BETA>(m1, m2, p + c < end ? x : 0ull);
      }
      group_top<BETA>(m1, m2, G);
      if ((lane & (G - 1)) == 0 && p < end) d_fold<BETA>(sm.D, (p >> alpha) - s0, m1, m2);
    }
  }
}

// Survivors: every element ranked >= t in the nq subranges listed in Q,
// read as one virtual vector of nq * 2^alpha keys in 4-key pieces (a piece
// never crosses a subrange).
template <bool VEC>
__device__ inline void b_survivors(const Keys<VEC>& ks, uint32_t n4, uint32_t nq, uint32_t alpha, const uint32_t* Q,
                                   uint64_t t, Codec cx, BatchSmem& sm) {
  const uint32_t L = 1u << alpha;
  const uint32_t total = nq << alpha;
  const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
  for (uint32_t base = wave * kBStep; base < total; base += kBWaves * kBStep) {
    uint32_t v[kBU][4], pb[kBU];
#pragma unroll
    for (int j = 0; j < kBU; ++j) {
      const uint32_t e = base + j * 256 + lane * 4;
      // past the virtual vector: a position at n4 or beyond reads zeros and is ignored
      pb[j] = e < total ? (Q[e >> alpha] << alpha) + (e & (L - 1)) : n4;
      ks.load4(pb[j], v[j]);
    }
#pragma unroll
    for (int j = 0; j < kBU; ++j)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const uint32_t p = pb[j] + c;
        const uint64_t x = comp(cx.enc(v[j][c]), p);
        lds_append(p < n4 && x >= t, x, &sm.nsurv, sm.surv, kBSurv);
      }
  }
}

// Everything after the delegate vector: t, the qualifying subranges, the
// survivors and the output.  sm.D[0..cnt) holds every delegate ranked at or
// above the k-th (the whole vector, or its top part when a split problem's
// vector lives in global memory), BETA = 2 as (first, second) pairs of one
// subrange each; sm.tail_del is the last delegate of the subrange holding
// the last n mod 4 keys.
//   BETA 1: the k-1 subranges whose delegate ranks above t are re-read.
//   BETA 2 (Rule 3): a subrange is re-read only if its second delegate ranks
//     above t (at most (k-1)/2 of them); of any other subrange only its
//     first delegate can rank above t (every other element is at most its
//     second delegate, so at most t), and that delegate survives as is.
// t itself survives once: its subrange is never re-read.  False if the
// survivors overflow LDS (nothing has been written then).
template <bool VEC, int BETA>
__device__ inline bool b_finish(const BatchDesc& d, uint32_t cnt, BatchSmem& sm) {
  const uint32_t n = (uint32_t)d.n, k = d.k, alpha = d.alpha, n4 = vec_end<VEC>(n);
  const Keys<VEC> ks(d.keys, n4);
  const uint64_t t = lds_select(sm.D, cnt, k, sm);  // Rule 2: the k-th delegate
  uint32_t* Q = sm.hist;  // the subranges to re-read (order irrelevant)
  if (threadIdx.x == 0) { sm.nq = 0; sm.nsurv = 1; sm.surv[0] = t; }
  __syncthreads();
  if constexpr (BETA == 1) {
    for (uint32_t i = threadIdx.x; i < cnt; i += kBT) {
      const uint64_t x = sm.D[i];
      if (x > t) Q[atomicAdd(&sm.nq, 1u)] = comp_pos(x) >> alpha;
    }
  } else {
    for (uint32_t i = threadIdx.x; i < cnt / 2; i += kBT) {
      const uint64_t a = sm.D[2 * i], b = sm.D[2 * i + 1];
      if (b > t) Q[atomicAdd(&sm.nq, 1u)] = comp_pos(b) >> alpha;
      else if (a > t) sm.surv[atomicAdd(&sm.nsurv, 1u)] = a;  // fewer than k of them
    }
  }
  __syncthreads();
  b_survivors<VEC>(ks, n4, sm.nq, alpha, Q, t, codec_of(d.dtype), sm);
  if (threadIdx.x == 0 && n4 < n && sm.tail_del > t) {  // the last keys, when their subrange is re-read
    for (uint32_t i = n4; i < n; ++i) {
      const uint64_t x = comp(codec_of(d.dtype).enc(d.keys[i]), i);
      if (x >= t) {
        const uint32_t slot = atomicAdd(&sm.nsurv, 1u);
        if (slot < kBSurv) sm.surv[slot] = x;
      }
    }
  }
  __syncthreads();
  const uint32_t ns = sm.nsurv;
  if (ns > kBSurv) return false;
  b_sort_write(sm.surv, ns, k, d.out_vals, d.out_idx, d.out_kth, codec_of(d.dtype), sm.D, sm.hist, sm);
  return true;
}

template <bool VEC, int BETA>
__device__ inline void b_delegates(const Keys<VEC>& ks, uint32_t lo, uint32_t hi, uint32_t n4, uint32_t alpha,
                                   Codec cx, BatchSmem& sm) {
  if (alpha >= 8) b_delegates_wide<VEC, BETA>(ks, lo, hi, n4, alpha, cx, sm);
  else b_delegates_narrow<VEC, BETA>(ks, lo, hi, n4, alpha, cx, sm);
}

// The delegate method for one problem in one workgroup; false if the
// survivors overflow LDS (nothing has been written then).
template <bool VEC, int BETA>
__device__ inline bool b_delegate(const BatchDesc& d, BatchSmem& sm) {
  const uint32_t n = (uint32_t)d.n, alpha = d.alpha, n4 = vec_end<VEC>(n);
  const uint32_t E = ((n + (1u << alpha) - 1) >> alpha) * BETA;
  const Keys<VEC> ks(d.keys, n4);
  for (uint32_t i = threadIdx.x; i < E; i += kBT) sm.D[i] = 0;
  __syncthreads();
  b_delegates<VEC, BETA>(ks, 0, n, n4, alpha, codec_of(d.dtype), sm);
  b_delegates_tail<BETA>(d, n4, 0, sm);
  __syncthreads();
  if (threadIdx.x == 0) sm.tail_del = n4 < n ? sm.D[(n4 >> alpha) * BETA + BETA - 1] : 0;
  return b_finish<VEC, BETA>(d, E, sm);
}

// A split problem's delegate vector (S subranges of BETA entries, global
// memory, written by the tiles' workgroups with coherent stores) cut down to
// LDS: MSD digits of the composites are histogrammed over it until the
// class holding the k-th delegate plus everything ranked above the class
// fit sm.D (kBMaxS entries, counting BETA per such entry), then the
// subranges whose first delegate lies in that class or above are copied
// there whole (the k-th delegate and all delegates above it among them).
// Returns the number of entries copied, or 0 if no cut fits (massive ties).
template <int BETA>
__device__ inline uint32_t b_cut_global(const uint64_t* Dg, uint32_t S, uint32_t k, BatchSmem& sm) {
  const uint32_t E = S * BETA;
  uint64_t prefix = 0, mask = 0;
  uint32_t r = k, above = 0, cls = 0;
  bool fits = false;
  for (int p = 0; p < kPasses; ++p) {
    for (int i = threadIdx.x; i < kBins; i += kBT) sm.hist[i] = 0;
    __syncthreads();
    const int sh = pass_shift(p);
    const uint32_t dm = (1u << pass_bits(p)) - 1;
    // eight coherent loads in flight per thread before any is counted
    for (uint32_t i0 = threadIdx.x; i0 < E; i0 += 8 * kBT) {
      uint64_t x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = i0 + u * kBT < E ? ld_coh64(&Dg[i0 + u * kBT]) : 0ull;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (i0 + u * kBT < E && (x[u] & mask) == prefix) atomicAdd(&sm.hist[(uint32_t)(x[u] >> sh) & dm], 1u);
    }
    __syncthreads();
    bb_bucket(sm.hist, r, sm);
    prefix |= (uint64_t)sm.out[0] << sh;
    mask |= (uint64_t)dm << sh;
    above += r - sm.out[1];
    r = sm.out[1];
    cls = sm.out[3];
    __syncthreads();
    if ((above + cls) * BETA <= kBMaxS) {
      fits = true;
      break;
    }
  }
  if (!fits) return 0;
  if (threadIdx.x == 0) sm.nq = 0;
  __syncthreads();
  // a subrange's first delegate is its largest: any of its entries in the
  // class or above puts the first there, so at most above + cls subranges
  for (uint32_t s0 = threadIdx.x; s0 < S; s0 += 8 * kBT) {
    uint64_t x[8], y[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint32_t s = s0 + u * kBT;
      x[u] = s < S ? ld_coh64(&Dg[s * BETA]) : 0ull;
      y[u] = BETA == 2 && s < S ? ld_coh64(&Dg[s * BETA + 1]) : 0ull;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (s0 + u * kBT < S && (x[u] & mask) >= prefix) {
        const uint32_t j = atomicAdd(&sm.nq, 1u);
        sm.D[j * BETA] = x[u];
        if constexpr (BETA == 2) sm.D[j * BETA + 1] = y[u];
      }
  }
  __syncthreads();
  const uint32_t cnt = sm.nq * BETA;
  __syncthreads();
  return cnt;
}

// Tile `tile` of a split problem (alpha >= 4): this workgroup builds the
// delegates of its tile and publishes them to Dg with coherent stores, then
// counts itself in; the workgroup that arrives last loads the whole delegate
// vector and finishes the problem (radix select over the keys if its
// survivors overflow).  Nobody waits for anybody.
template <bool VEC, int BETA>
__device__ inline void b_tile(const BatchDesc& d, uint32_t tile, uint32_t* arrive, uint64_t* Dg, BatchSmem& sm,
                              uint32_t* rec);

template <bool VEC>
__device__ inline void b_problem_v(const BatchDesc& d, BatchSmem& sm, uint32_t* rec) {
  if (d.n <= kBSmallN) {
    b_small<VEC>(d, sm);
    return;
  }
  if (d.alpha >= 2) {
    const uint64_t E = ((d.n + (1ull << d.alpha) - 1) >> d.alpha) * d.beta;
    if (E <= kBMaxS && E > d.k && (d.beta == 2 ? b_delegate<VEC, 2>(d, sm) : b_delegate<VEC, 1>(d, sm))) return;
    __syncthreads();
  }
  b_radix<VEC>(d, sm, rec);
}

template <bool VEC, int BETA>
__device__ inline void b_tile(const BatchDesc& d, uint32_t tile, uint32_t* arrive, uint64_t* Dg, BatchSmem& sm,
                              uint32_t* rec) {
  const uint32_t n = (uint32_t)d.n, alpha = d.alpha, n4 = vec_end<VEC>(n);
  const uint32_t tlog = tile_log(alpha, BETA);
  const uint32_t lo = tile << tlog;
  const uint32_t hi = n - lo > (1u << tlog) ? lo + (1u << tlog) : n;
  const uint32_t s0 = lo >> alpha;
  const uint32_t ne = (((hi - lo) + (1u << alpha) - 1) >> alpha) * BETA;  // entries of this tile
  const Keys<VEC> ks(d.keys, n4);
  for (uint32_t i = threadIdx.x; i < ne; i += kBT) sm.D[i] = 0;
  __syncthreads();
  b_delegates<VEC, BETA>(ks, lo, hi, n4, alpha, codec_of(d.dtype), sm);
  if (hi == n) b_delegates_tail<BETA>(d, n4, s0, sm);
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < ne; i += kBT) st_coh64(&Dg[d.doff + s0 * BETA + i], sm.D[i]);
  __builtin_amdgcn_s_waitcnt(0);  // this thread's stores have completed
  __syncthreads();
  if (threadIdx.x == 0) sm.item = atomicAdd(arrive, 1u) == d.tiles - 1 ? 1u : 0u;
  __syncthreads();
  if (!sm.item) return;
  const uint32_t S = (n + (1u << alpha) - 1) >> alpha;
  if (threadIdx.x == 0) sm.tail_del = n4 < n ? ld_coh64(&Dg[d.doff + (n4 >> alpha) * BETA + BETA - 1]) : 0;
  uint32_t cnt = S * BETA;
  if (cnt <= kBMaxS) {
    for (uint32_t i0 = threadIdx.x; i0 < cnt; i0 += 8 * kBT) {  // eight loads in flight per thread
      uint64_t x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = i0 + u * kBT < cnt ? ld_coh64(&Dg[d.doff + i0 + u * kBT]) : 0ull;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (i0 + u * kBT < cnt) sm.D[i0 + u * kBT] = x[u];
    }
    __syncthreads();
  } else {
    cnt = b_cut_global<BETA>(Dg + d.doff, S, d.k, sm);
  }
  if (cnt && b_finish<VEC, BETA>(d, cnt, sm)) return;
  __syncthreads();
  b_radix<VEC>(d, sm, rec);
}

__device__ inline void b_problem(const BatchDesc& d, BatchSmem& sm, uint32_t* rec) {
  const bool vec = (reinterpret_cast<uintptr_t>(d.keys) & 15u) == 0;
  if (vec) b_problem_v<true>(d, sm, rec);
  else b_problem_v<false>(d, sm, rec);
}

__device__ inline void b_tile_any(const BatchDesc& d, uint32_t tile, uint32_t* arrive, uint64_t* Dg, BatchSmem& sm,
                                  uint32_t* rec) {
  const bool vec = (reinterpret_cast<uintptr_t>(d.keys) & 15u) == 0;
  if (d.beta == 2) {
    if (vec) b_tile<true, 2>(d, tile, arrive, Dg, sm, rec);
    else b_tile<false, 2>(d, tile, arrive, Dg, sm, rec);
  } else {
    if (vec) b_tile<true, 1>(d, tile, arrive, Dg, sm, rec);
    else b_tile<false, 1>(d, tile, arrive, Dg, sm, rec);
  }
}

// Work items (problem << 8 | tile), claimed from *counter (starts at 0):
// a problem with tiles <= 1 is one item and runs whole in the workgroup; a
// split problem is `tiles` items whose workgroups share its delegate vector
// through Dg, with arrive[problem] (starts at 0) counting finished tiles.
// Any grid size works: no workgroup waits for another.
__global__ __launch_bounds__(kBT) __attribute__((amdgpu_waves_per_eu(4))) void k_batched(
    const BatchDesc* __restrict__ descs, const uint32_t* __restrict__ items, uint32_t nitems, uint32_t* counter,
    uint32_t* arrive, uint64_t* Dg, uint32_t* rec) {
  __shared__ BatchSmem sm;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) sm.item = atomicAdd(counter, 1u);
    __syncthreads();
    const uint32_t w = sm.item;
    __syncthreads();
    if (w >= nitems) break;
    const uint32_t it = items[w];
    const uint32_t i = it >> 8;
    const BatchDesc d = descs[i];
    if (d.tiles > 1) b_tile_any(d, it & 0xFFu, &arrive[i], Dg, sm, rec);
    else b_problem(d, sm, rec);
  }
}

// Up to kBInline problems with the descriptors passed by value: no copy of
// descriptors and no claim counter.  Grid = count: workgroup i owns problem i.
constexpr uint32_t kBInline = 32;
struct BatchInline {
  BatchDesc d[kBInline];
};
__global__ __launch_bounds__(kBT) __attribute__((amdgpu_waves_per_eu(4))) void k_batched_inline(BatchInline b, uint32_t* rec) {
  __shared__ BatchSmem sm;
  b_problem(b.d[blockIdx.x], sm, rec);
}

// One problem, descriptor by value: the single-problem path for small inputs.
__global__ __launch_bounds__(kBT) __attribute__((amdgpu_waves_per_eu(4))) void k_one(BatchDesc d, uint32_t* rec) {
  __shared__ BatchSmem sm;
  b_problem(d, sm, rec);
}

}  // namespace drtopk
