// The single-problem path's kernel sequence for one codec.  Included only by
// the per-codec translation units, which instantiate run_codec and
// delegates_codec.
#pragma once

#include "host.h"
#include "inner.h"
#include "kernels.h"
#include "tail.h"

namespace drtopk {

// ---------------------------------------------------------------------------
// kernel sequence
template <int DT>
struct Runner {
  static void delegate(const Plan& p, const uint32_t* keys, uint32_t* dkey, uint32_t* didx, Ctl* ctl,
                       hipStream_t st, DirectOut out = DirectOut{nullptr, nullptr, nullptr, 0}) {
    if (p.alpha >= 2) {
      const unsigned g = (unsigned)((p.n + p.chunk - 1) / p.chunk);
#define DRTOPK_DEL(B, V) \
  hipLaunchKernelGGL((k_delegate<DT, B, V>), dim3(g), dim3(256), 0, st, keys, p.n, p.alpha, p.chunk, dkey, didx, ctl, p.kD, \
                     out)
      switch (p.beta * 2 + (p.vec ? 1 : 0)) {
        case 2: DRTOPK_DEL(1, false); break;
        case 3: DRTOPK_DEL(1, true); break;
        case 4: DRTOPK_DEL(2, false); break;
        case 5: DRTOPK_DEL(2, true); break;
        case 8: DRTOPK_DEL(4, false); break;
        case 9: DRTOPK_DEL(4, true); break;
        case 16: DRTOPK_DEL(8, false); break;
        default: DRTOPK_DEL(8, true); break;
      }
#undef DRTOPK_DEL
    } else {
      const unsigned g = grid_for(p.S, 256, 4096);
#define DRTOPK_DELT(B) \
  hipLaunchKernelGGL((k_delegate_thread<DT, B>), dim3(g), dim3(256), 0, st, keys, p.n, p.alpha, p.S, dkey, didx, ctl, \
                     p.kD, out)
      switch (p.beta) {
        case 1: DRTOPK_DELT(1); break;
        case 2: DRTOPK_DELT(2); break;
        case 4: DRTOPK_DELT(4); break;
        default: DRTOPK_DELT(8); break;
      }
#undef DRTOPK_DELT
    }
  }

  template <int B, bool V>
  static void launch_tail_t(TailArgs& ta, hipStream_t st) {
    static int blocks = 0;  // blocks that fit the device at once (phases need no co-residency)
    if (blocks == 0) {
      int dev = 0, cus = 0, per = 0;
      (void)hipGetDevice(&dev);
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(&k_tail<DT, B, V>),
                                                          kTailThreads, 0);
      if (per > 2) per = 2;
      if (per < 1) per = 1;
      blocks = cus * per;
    }
    hipLaunchKernelGGL((k_tail<DT, B, V>), dim3(blocks), dim3(kTailThreads), 0, st, ta);
  }

  static void launch_tail(const Plan& p, TailArgs& ta, hipStream_t st) {
    switch (p.beta * 2 + (p.vec ? 1 : 0)) {
      case 2: launch_tail_t<1, false>(ta, st); break;
      case 3: launch_tail_t<1, true>(ta, st); break;
      case 4: launch_tail_t<2, false>(ta, st); break;
      case 5: launch_tail_t<2, true>(ta, st); break;
      case 8: launch_tail_t<4, false>(ta, st); break;
      case 9: launch_tail_t<4, true>(ta, st); break;
      case 16: launch_tail_t<8, false>(ta, st); break;
      default: launch_tail_t<8, true>(ta, st); break;
    }
  }

  static void qualify(const Plan& p, uint32_t* dkey, uint32_t* didx, Ctl* ctl, uint32_t* Q, uint32_t* ckey,
                      uint32_t* cidx, hipStream_t st) {
    const unsigned g = grid_for(p.S, 256 * 16, 1024);
    switch (p.beta) {
      case 1: hipLaunchKernelGGL((k_qualify<1>), dim3(g), dim3(256), 0, st, dkey, didx, p.S, ctl, Q, ckey, cidx); break;
      case 2: hipLaunchKernelGGL((k_qualify<2>), dim3(g), dim3(256), 0, st, dkey, didx, p.S, ctl, Q, ckey, cidx); break;
      case 4: hipLaunchKernelGGL((k_qualify<4>), dim3(g), dim3(256), 0, st, dkey, didx, p.S, ctl, Q, ckey, cidx); break;
      default: hipLaunchKernelGGL((k_qualify<8>), dim3(g), dim3(256), 0, st, dkey, didx, p.S, ctl, Q, ckey, cidx); break;
    }
  }

  // The k sorted outputs from okey/oidx (exactly k entries), k > kSmallCap.
  // gated: 0 always run, 1 only if the tail kernel set ctl->need_merge
  static void big_sort(const Plan& p, void* ws, uint32_t* out_vals, uint32_t* out_idx, uint32_t* out_kth,
                       int gated, Ctl* ctl, hipStream_t st) {
    uint64_t* A = at<uint64_t>(ws, p.off_A);
    uint64_t* B = at<uint64_t>(ws, p.off_B);
    hipLaunchKernelGGL(k_blocksort, dim3((unsigned)(p.M / kSortTile)), dim3(1024), 0, st,
                       at<uint32_t>(ws, p.off_okey), at<uint32_t>(ws, p.off_oidx), p.k, A, gated, ctl);
    for (uint64_t run = kSortTile; run < p.M; run <<= 1) {
      const int last = (2 * run == p.M) ? 1 : 0;
      hipLaunchKernelGGL((k_merge<DT>), dim3((unsigned)(p.M / 256)), dim3(256), 0, st, A, B, p.M, run, last, p.k,
                         out_vals, out_idx, out_kth, gated, ctl);
      std::swap(A, B);
    }
  }

  // Rounds of the bitonic top-k over `key`/`idx` (SRC_D or SRC_C, at most
  // `bound` entries) down to one block, which finishes with `fin` (1: the
  // threshold t, 2: the sorted outputs).  Each round's blocks fold tiles of
  // 4096 into one list of K = 2^ceil(log2 k) entries.
  template <int SRC>
  static void bitonic(const Plan& p, const uint32_t* key, const uint32_t* idx, uint64_t bound, int fin, Ctl* ctl,
                      void* ws, uint32_t* out_vals, uint32_t* out_idx, uint32_t* out_kth, hipStream_t st) {
    uint32_t K = 1;
    while (K < p.k) K <<= 1;
    uint64_t* cur = at<uint64_t>(ws, p.off_L0);
    uint64_t* nxt = at<uint64_t>(ws, p.off_L1);
    const auto blocks = [](uint64_t entries) {
      const uint64_t t = (entries + kBtTile - 1) / kBtTile;
      return (unsigned)(t < 1 ? 1 : t > kBtRoundBlocks ? kBtRoundBlocks : t);
    };
    unsigned g = blocks(bound);
    hipLaunchKernelGGL((k_btopk<SRC, DT>), dim3(g), dim3(kBtThreads), 0, st, key, idx, (const uint64_t*)nullptr,
                       bound, K, g == 1 ? fin : 0, p.k, ctl, cur, out_vals, out_idx, out_kth);
    uint64_t cnt = (uint64_t)g * K;
    while (g > 1) {
      g = blocks(cnt);
      hipLaunchKernelGGL((k_btopk<SRC_OUT, DT>), dim3(g), dim3(kBtThreads), 0, st, (const uint32_t*)nullptr,
                         (const uint32_t*)nullptr, cur, cnt, K, g == 1 ? fin : 0, p.k, ctl, nxt, out_vals, out_idx,
                         out_kth);
      cnt = (uint64_t)g * K;
      std::swap(cur, nxt);
    }
  }

  // Bucket select over `key`/`idx`: min/max, then at most kPasses passes that
  // each keep the bucket holding rank k; the result lands in selD (which 0)
  // or selC (which 1).
  template <int SRC>
  static void bucket(const Plan& p, const uint32_t* key, const uint32_t* idx, uint64_t bound, int which, Ctl* ctl,
                     hipStream_t st) {
    const unsigned g = grid_for(bound, 256 * 8, 1024);
    hipLaunchKernelGGL((k_bminmax<SRC, DT>), dim3(g), dim3(256), 0, st, key, idx, bound, which, ctl);
    for (int pass = 0; pass < kPasses; ++pass)
      hipLaunchKernelGGL((k_bpass<SRC, DT>), dim3(g), dim3(256), 0, st, key, idx, bound, pass, which, p.k, ctl);
  }

  // The delegate method with the bitonic top-k (variant 2) or the bucket
  // select (variant 3) as both of its selections; Rule 3 and the re-read are
  // variant 1's kernels.
  static void run_alt(const Plan& p, const uint32_t* keys, void* ws, uint32_t* out_vals, uint32_t* out_idx,
                      uint32_t* out_kth, bool kth_only, bool filter_only, hipStream_t st, PhaseMarks& pm) {
    Ctl* ctl = at<Ctl>(ws, p.off_ctl);
    uint32_t* dkey = at<uint32_t>(ws, p.off_dkey);
    uint32_t* didx = at<uint32_t>(ws, p.off_didx);
    uint32_t* Q = at<uint32_t>(ws, p.off_q);
    uint32_t* ckey = at<uint32_t>(ws, p.off_ckey);
    uint32_t* cidx = at<uint32_t>(ws, p.off_cidx);
    const uint32_t k = p.k;
    delegate(p, keys, dkey, didx, ctl, st);
    pm.mid(st);
    // first top-k: t = the k-th delegate (none when fewer than k are real)
    if (!p.all) {
      if (p.variant == 2)
        bitonic<SRC_D>(p, dkey, didx, p.nd, 1, ctl, ws, nullptr, nullptr, nullptr, st);
      else
        bucket<SRC_D>(p, dkey, didx, p.nd, 0, ctl, st);
    }
    qualify(p, dkey, didx, ctl, Q, ckey, cidx, st);
    const unsigned gS = grid_for(((uint64_t)((k - 1) / p.beta) + 1) << p.alpha, 4096, 2048);
    if (p.vec)
      hipLaunchKernelGGL((k_scan<DT, true>), dim3(gS), dim3(256), 0, st, keys, p.n, p.alpha, ctl, Q, ckey, cidx);
    else
      hipLaunchKernelGGL((k_scan<DT, false>), dim3(gS), dim3(256), 0, st, keys, p.n, p.alpha, ctl, Q, ckey, cidx);
    if (filter_only) return;
    // second top-k over the survivors
    if (p.variant == 2) {
      bitonic<SRC_C>(p, ckey, cidx, p.cap_c, 2, ctl, ws, kth_only ? nullptr : out_vals, kth_only ? nullptr : out_idx,
                     out_kth, st);
      return;
    }
    bucket<SRC_C>(p, ckey, cidx, p.cap_c, 1, ctl, st);
    if (kth_only) {
      hipLaunchKernelGGL((k_kth_from_sel<DT>), dim3(1), dim3(64), 0, st, 0, ctl, out_kth);
      return;
    }
    uint32_t* okey = at<uint32_t>(ws, p.off_okey);
    uint32_t* oidx = at<uint32_t>(ws, p.off_oidx);
    const unsigned gC = grid_for(p.cap_c, 256 * 8, 1024);
    hipLaunchKernelGGL((k_compact<SRC_C, DT>), dim3(gC), dim3(256), 0, st, ckey, cidx, (uint64_t)0, 0, k, ctl, okey,
                       oidx);
    if (k <= (uint32_t)kSmallCap)
      hipLaunchKernelGGL((k_final_small<SRC_OUT, DT>), dim3(1), dim3(1024), 0, st, okey, oidx, (uint64_t)k, 0, k, ctl,
                         out_vals, out_idx, out_kth);
    else
      big_sort(p, ws, out_vals, out_idx, out_kth, 0, ctl, st);
  }

  // filter_only: stop once the survivors are known (stage checks).
  static void run(const Plan& p, const uint32_t* keys, void* ws, uint32_t* out_vals, uint32_t* out_idx,
                  uint32_t* out_kth, bool kth_only, bool filter_only, hipStream_t st) {
    PhaseMarks pm;
    if (p.marks) pm.begin(st);
    run_inner(p, keys, ws, out_vals, out_idx, out_kth, kth_only, filter_only, st, pm);
    pm.end(st);
  }

  static void run_inner(const Plan& p, const uint32_t* keys, void* ws, uint32_t* out_vals, uint32_t* out_idx,
                        uint32_t* out_kth, bool kth_only, bool filter_only, hipStream_t st, PhaseMarks& pm) {
    Ctl* ctl = at<Ctl>(ws, p.off_ctl);
    hipLaunchKernelGGL(k_init, dim3(8), dim3(1024), 0, st, ctl, (uint32_t)p.S, (uint32_t)p.cap_c,
                       p.all ? 1u : 0u, p.rec);
    pm.start(st);
    uint32_t* okey = at<uint32_t>(ws, p.off_okey);
    uint32_t* oidx = at<uint32_t>(ws, p.off_oidx);
    const uint32_t k = p.k;
    if (p.mode == 1 && p.variant == 0) {
      uint32_t* dkey = at<uint32_t>(ws, p.off_dkey);
      uint32_t* didx = at<uint32_t>(ws, p.off_didx);
      if (k == 1 && !filter_only) {  // the largest delegate is the answer (Rule 1)
        delegate(p, keys, dkey, didx, ctl, st, DirectOut{out_vals, out_idx, out_kth, 1});
        pm.mid(st);
        return;
      }
      delegate(p, keys, dkey, didx, ctl, st);
      pm.mid(st);
      TailArgs ta;
      ta.keys = keys;
      ta.n = p.n;
      ta.alpha = p.alpha;
      ta.S = p.S;
      ta.nd = p.nd;
      ta.k = k;
      ta.kD = p.kD;
      ta.slack = p.slack;
      ta.all = p.all ? 1 : 0;
      ta.kth_only = kth_only ? 1 : 0;
      ta.stop_after_scan = filter_only ? 1 : 0;
      ta.big_sort = (!kth_only && k > (uint32_t)kSmallCap) ? 1 : 0;
      ta.dkey = dkey;
      ta.didx = didx;
      ta.Q = at<uint32_t>(ws, p.off_q);
      ta.ckey = at<uint32_t>(ws, p.off_ckey);
      ta.cidx = at<uint32_t>(ws, p.off_cidx);
      ta.skey = at<uint32_t>(ws, p.off_skey);
      ta.sidx = at<uint32_t>(ws, p.off_sidx);
      ta.okey = okey;
      ta.oidx = oidx;
      ta.cap_s = (uint32_t)p.cap_c;
      ta.out_vals = out_vals;
      ta.out_idx = out_idx;
      ta.out_kth = out_kth;
      ta.A = ta.big_sort ? at<uint64_t>(ws, p.off_A) : nullptr;
      ta.B = ta.big_sort ? at<uint64_t>(ws, p.off_B) : nullptr;
      ta.M = p.M;
      ta.ctl = ctl;
      launch_tail(p, ta, st);
      return;
    }
    if (p.mode == 1 && p.variant >= 2) {
      run_alt(p, keys, ws, out_vals, out_idx, out_kth, kth_only, filter_only, st, pm);
      return;
    }
    if (p.mode == 1) {
      uint32_t* dkey = at<uint32_t>(ws, p.off_dkey);
      uint32_t* didx = at<uint32_t>(ws, p.off_didx);
      uint32_t* Q = at<uint32_t>(ws, p.off_q);
      uint32_t* ckey = at<uint32_t>(ws, p.off_ckey);
      uint32_t* cidx = at<uint32_t>(ws, p.off_cidx);
      delegate(p, keys, dkey, didx, ctl, st);
      pm.mid(st);
      const unsigned gD = grid_for(p.nd, 256 * 8, 1024);
      for (int pass = 1; pass < kPasses; ++pass)
        hipLaunchKernelGGL((k_pass<SRC_D, DT>), dim3(gD), dim3(256), 0, st, dkey, didx, p.nd, pass, 0, ctl, p.kD);
      qualify(p, dkey, didx, ctl, Q, ckey, cidx, st);
      // expected concatenated length: about k/beta subranges of 2^alpha (grid-stride covers more)
      const unsigned gS = grid_for(((uint64_t)((k - 1) / p.beta) + 1) << p.alpha, 4096, 2048);
      if (p.vec)
        hipLaunchKernelGGL((k_scan<DT, true>), dim3(gS), dim3(256), 0, st, keys, p.n, p.alpha, ctl, Q, ckey, cidx);
      else
        hipLaunchKernelGGL((k_scan<DT, false>), dim3(gS), dim3(256), 0, st, keys, p.n, p.alpha, ctl, Q, ckey, cidx);
      if (filter_only) return;
      const bool may_be_big = p.cap_c > (uint64_t)kSmallCap;
      hipLaunchKernelGGL((k_final_small<SRC_C, DT>), dim3(1), dim3(1024), 0, st, ckey, cidx, (uint64_t)0,
                         may_be_big ? 1 : 0, k, ctl, out_vals, out_idx, out_kth);
      if (!may_be_big) return;
      const unsigned gC = grid_for(p.cap_c, 256 * 8, 1024);
      for (int pass = 0; pass < kPasses; ++pass)
        hipLaunchKernelGGL((k_pass<SRC_C, DT>), dim3(gC), dim3(256), 0, st, ckey, cidx, (uint64_t)0, pass, 2, ctl, k);
      if (kth_only) {
        hipLaunchKernelGGL((k_kth_from_sel<DT>), dim3(1), dim3(64), 0, st, 2, ctl, out_kth);
        return;
      }
      hipLaunchKernelGGL((k_compact<SRC_C, DT>), dim3(gC), dim3(256), 0, st, ckey, cidx, (uint64_t)0, 2, k, ctl, okey,
                         oidx);
      if (k <= (uint32_t)kSmallCap)
        hipLaunchKernelGGL((k_final_small<SRC_OUT, DT>), dim3(1), dim3(1024), 0, st, okey, oidx, (uint64_t)k, 2, k,
                           ctl, out_vals, out_idx, out_kth);
      else
        big_sort(p, ws, out_vals, out_idx, out_kth, 0, ctl, st);
    } else {
      if (p.n <= (uint64_t)kSmallCap) {
        hipLaunchKernelGGL((k_final_small<SRC_V, DT>), dim3(1), dim3(1024), 0, st, keys, (const uint32_t*)nullptr,
                           p.n, 0, k, ctl, out_vals, out_idx, out_kth);
        return;
      }
      const unsigned gV = grid_for(p.n, 256 * 16, 2048);
      for (int pass = 0; pass < kPasses; ++pass) {
        hipLaunchKernelGGL((k_pass<SRC_V, DT>), dim3(gV), dim3(256), 0, st, keys, (const uint32_t*)nullptr, p.n, pass,
                           0, ctl, k);
        if (pass == 0) pm.mid(st);
      }
      if (kth_only) {
        hipLaunchKernelGGL((k_kth_from_sel<DT>), dim3(1), dim3(64), 0, st, 0, ctl, out_kth);
        return;
      }
      hipLaunchKernelGGL((k_compact<SRC_V, DT>), dim3(gV), dim3(256), 0, st, keys, (const uint32_t*)nullptr, p.n, 0,
                         k, ctl, okey, oidx);
      if (k <= (uint32_t)kSmallCap)
        hipLaunchKernelGGL((k_final_small<SRC_OUT, DT>), dim3(1), dim3(1024), 0, st, okey, oidx, (uint64_t)k, 0, k,
                           ctl, out_vals, out_idx, out_kth);
      else
        big_sort(p, ws, out_vals, out_idx, out_kth, 0, ctl, st);
    }
  }
};


template <int DT>
__global__ void k_decode_inplace(uint32_t* v, uint64_t m) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (uint64_t)gridDim.x * blockDim.x)
    v[i] = dec<DT>(v[i]);
}


template <int DT>
void run_codec(const Plan& p, const uint32_t* keys, void* ws, uint32_t* out_vals, uint32_t* out_idx,
               uint32_t* out_kth, bool kth_only, bool filter_only, hipStream_t st) {
  Runner<DT>::run(p, keys, ws, out_vals, out_idx, out_kth, kth_only, filter_only, st);
}

template <int DT>
void delegates_codec(const Plan& p, const uint32_t* keys, uint32_t* dkey, uint32_t* didx, Ctl* ctl, hipStream_t st) {
  hipLaunchKernelGGL(k_init, dim3(8), dim3(1024), 0, st, ctl, (uint32_t)p.S, (uint32_t)p.cap_c, 0u, p.rec);
  Runner<DT>::delegate(p, keys, dkey, didx, ctl, st);
  if constexpr (DT != DT_U32)
    hipLaunchKernelGGL((k_decode_inplace<DT>), dim3(grid_for(p.nd, 256 * 4, 4096)), dim3(256), 0, st, dkey, p.nd);
}

}  // namespace drtopk
