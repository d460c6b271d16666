// Alternative top-k algorithms inside the delegate method (the paper's claim,
// Sections 5.1 and 6.1, that delegates assist radix-, bucket- and
// bitonic-based top-k alike).  The method's two selections -- the first
// top-k over the delegate vector (Rule 2's threshold t) and the second top-k
// over the survivors -- run on one of:
//   radix   the MSD radix select of k_pass (tail variant 1);
//   bucket  a bucket select: equal-width buckets over the live range
//           [lo, hi] of the composites, which shrinks to the bucket holding
//           the sought rank each pass (min and max from the data first);
//   bitonic (k <= 256) the bitonic top-k: groups of K = 2^ceil(log2 k)
//           entries sorted by a bitonic network, then pairs of sorted groups
//           combined by an element-wise maximum against the reversed partner
//           (a bitonic sequence holding the top K of both) and re-sorted by
//           half-cleaners, until one group is left.
// Rule 3 (the qualifying subranges) and the re-read are the shared kernels
// k_qualify and k_scan; every variant gives the same, exact answer.
#pragma once

#include "kernels.h"

namespace drtopk {

constexpr int kBtTile = 4096;  // entries per bitonic tile (LDS)
constexpr int kBtThreads = 256;

// Entry i of a selection's source as a composite: the delegate vector
// (SRC_D), the survivors (SRC_C, count on the device) or a list of
// composites (SRC_OUT: the partial lists of the bitonic rounds).
template <int SRC, int DT>
__device__ __forceinline__ uint64_t inner_entry(const uint32_t* key, const uint32_t* idx, const uint64_t* list,
                                                uint64_t i) {
  if constexpr (SRC == SRC_OUT) return list[i];
  else return comp(src_key<SRC, DT>(key, i), src_pos<SRC>(idx, i));
}

template <int SRC>
__device__ __forceinline__ uint64_t inner_count(const Ctl* ctl, uint64_t count_static) {
  return SRC == SRC_C ? (uint64_t)clamp_nc(ctl) : count_static;
}

// ---------------------------------------------------------------------------
// bitonic top-k

// Descending half-cleaner cascade over each of `groups` bitonic groups of K
// entries at the start of buf.
__device__ inline void bt_merge_groups(uint64_t* buf, uint32_t groups, uint32_t K) {
  for (uint32_t stride = K >> 1; stride > 0; stride >>= 1) {
    const uint32_t half = K >> 1;
    for (uint32_t i = threadIdx.x; i < groups * half; i += blockDim.x) {
      const uint32_t g = i / half, e = i % half;
      const uint32_t lo = g * K + 2 * e - (e & (stride - 1));
      const uint32_t hi = lo + stride;
      const uint64_t a = buf[lo], b = buf[hi];
      if (a < b) { buf[lo] = b; buf[hi] = a; }
    }
    __syncthreads();
  }
}

// One round of the bitonic top-k: each block folds tiles blockIdx.x,
// blockIdx.x + gridDim.x, ... of the source into its running top K (sorted
// descending), then
//   fin 0: writes it to out_list[blockIdx.x * K ..];
//   fin 1: (one block) sets the threshold t = the k-th entry (first top-k);
//   fin 2: (one block) writes the k outputs, decoded (second top-k).
template <int SRC, int DT>
__global__ __launch_bounds__(kBtThreads) void k_btopk(const uint32_t* __restrict__ key,
                                                      const uint32_t* __restrict__ idx,
                                                      const uint64_t* __restrict__ list, uint64_t count_static,
                                                      uint32_t K, int fin, uint32_t k, Ctl* ctl, uint64_t* out_list,
                                                      uint32_t* out_vals, uint32_t* out_idx, uint32_t* out_kth) {
  __shared__ uint64_t tile[kBtTile];
  __shared__ uint64_t run[kBtMaxK];
  const uint64_t count = inner_count<SRC>(ctl, count_static);
  const uint64_t ntiles = (count + kBtTile - 1) / kBtTile;
  for (uint32_t i = threadIdx.x; i < K; i += blockDim.x) run[i] = 0;
  for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint64_t base = t * kBtTile;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < (uint32_t)kBtTile; i += blockDim.x)
      tile[i] = base + i < count ? inner_entry<SRC, DT>(key, idx, list, base + i) : 0ull;
    __syncthreads();
    // every group of K sorted descending (the last size level sorts all of
    // them the same way)
    for (uint32_t size = 2; size <= K; size <<= 1) {
      for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
        for (uint32_t i = threadIdx.x; i < (uint32_t)kBtTile / 2; i += blockDim.x) {
          const uint32_t lo = 2 * i - (i & (stride - 1));
          const uint32_t hi = lo + stride;
          const bool desc = size == K || (lo & size) == 0;
          const uint64_t a = tile[lo], b = tile[hi];
          if ((a < b) == desc) { tile[lo] = b; tile[hi] = a; }
        }
        __syncthreads();
      }
    }
    // pairs of groups (j, j + half): max against the reversed partner, then re-sorted
    for (uint32_t groups = kBtTile / K; groups > 1; groups >>= 1) {
      const uint32_t half = groups >> 1;
      for (uint32_t i = threadIdx.x; i < half * K; i += blockDim.x) {
        const uint32_t g = i / K, e = i % K;
        const uint64_t a = tile[g * K + e], b = tile[(g + half) * K + K - 1 - e];
        tile[g * K + e] = a > b ? a : b;
      }
      __syncthreads();
      bt_merge_groups(tile, half, K);
    }
    // fold the tile's top K into the running list the same way
    for (uint32_t i = threadIdx.x; i < K; i += blockDim.x) {
      const uint64_t a = run[i], b = tile[K - 1 - i];
      run[i] = a > b ? a : b;
    }
    __syncthreads();
    bt_merge_groups(run, 1, K);
  }
  __syncthreads();
  if (fin == 0) {
    for (uint32_t i = threadIdx.x; i < K; i += blockDim.x) out_list[(uint64_t)blockIdx.x * K + i] = run[i];
  } else if (fin == 1) {
    if (threadIdx.x == 0) {
      ctl->selD.prefix = ctl->all ? 0ull : run[k - 1];
      ctl->selD.found = 1;
    }
  } else {
    if (count < k && threadIdx.x == 0) flag_err(ctl, ERR_FEW);
    for (uint32_t r = threadIdx.x; r < k; r += blockDim.x) write_out<DT>(run[r], r, k, out_vals, out_idx, out_kth);
  }
}

// ---------------------------------------------------------------------------
// bucket select

// Largest and smallest composite of the source (the smallest kept as its
// complement, so both are maxima over a zeroed control block).
template <int SRC, int DT>
__global__ __launch_bounds__(256) void k_bminmax(const uint32_t* __restrict__ key, const uint32_t* __restrict__ idx,
                                                 uint64_t count_static, int which, Ctl* ctl) {
  const uint64_t count = inner_count<SRC>(ctl, count_static);
  uint64_t mx = 0, nmn = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (uint64_t)gridDim.x * 256) {
    const uint64_t c = inner_entry<SRC, DT>(key, idx, nullptr, i);
    mx = c > mx ? c : mx;
    nmn = ~c > nmn ? ~c : nmn;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t a = shfl_xor64(mx, o), b = shfl_xor64(nmn, o);
    mx = a > mx ? a : mx;
    nmn = b > nmn ? b : nmn;
  }
  if (lane_id() == 0 && count) {
    atomicMax((unsigned long long*)&ctl->bmax[which], (unsigned long long)mx);
    atomicMax((unsigned long long*)&ctl->bnmin[which], (unsigned long long)nmn);
  }
}

// One pass: buckets of width 2^sh over [lo, hi] (at most 2048 of them, sh
// the smallest that fits), counted; the last block keeps the bucket holding
// the sought rank as the new [lo, hi].  Once lo == hi the range is the
// selected composite itself, stored as the select's result (selD or selC).
template <int SRC, int DT>
__global__ __launch_bounds__(256) void k_bpass(const uint32_t* __restrict__ key, const uint32_t* __restrict__ idx,
                                               uint64_t count_static, int p, int which, uint32_t k, Ctl* ctl) {
  __shared__ uint32_t lh[kBins];
  __shared__ uint32_t s_scan[256];
  __shared__ uint32_t s_out[4];
  __shared__ int s_last;
  if (ctl->bdone[which]) return;
  const uint64_t lo = p == 0 ? ~ctl->bnmin[which] : ctl->blo[which];
  const uint64_t hi = p == 0 ? ctl->bmax[which] : ctl->bhi[which];
  const uint32_t rank = p == 0 ? k : ctl->brank[which];
  const uint32_t bl = bitlen64(hi - lo);
  const uint32_t sh = bl > 11u ? bl - 11u : 0u;
  const uint64_t count = inner_count<SRC>(ctl, count_static);
  for (int i = threadIdx.x; i < kBins; i += 256) lh[i] = 0;
  __syncthreads();
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (uint64_t)gridDim.x * 256) {
    const uint64_t c = inner_entry<SRC, DT>(key, idx, nullptr, i);
    if (c >= lo && c <= hi) atomicAdd(&lh[(uint32_t)((c - lo) >> sh)], 1u);
  }
  __syncthreads();
  // own rows: the delegate pass has already used histD[0] and ticketD[0]
  uint32_t* gh = which ? ctl->histC[p] : ctl->histW[p];
  flush_hist(lh, gh);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  uint32_t* ticket = &ctl->bticket[which][p];
  if (threadIdx.x == 0) s_last = (atomicAdd(ticket, 1u) == gridDim.x - 1) ? 1 : 0;
  __syncthreads();
  if (!s_last) return;
  block_select_bucket(gh, rank, s_scan, s_out);
  if (threadIdx.x == 0) {
    const uint64_t nlo = lo + ((uint64_t)s_out[0] << sh);
    const uint64_t w = sh ? ((1ull << sh) - 1) : 0ull;
    const uint64_t nhi = hi - nlo > w ? nlo + w : hi;
    ctl->blo[which] = nlo;
    ctl->bhi[which] = nhi;
    ctl->brank[which] = s_out[1];
    if (!s_out[2]) {
      flag_err(ctl, ERR_SELECT);
      ctl->bdone[which] = 1;
    } else if (nlo == nhi) {
      Sel* sel = which ? &ctl->selC : &ctl->selD;
      sel->prefix = nlo;
      sel->found = 1;
      ctl->bdone[which] = 1;
    }
  }
}

}  // namespace drtopk
