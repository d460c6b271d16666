// 64-bit keys (uint64, int64, float64): planner and kernel sequence.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "host.h"
#include "wide.h"
#include "wide_host.h"

namespace drtopk {

namespace {

size_t walign(size_t x) { return (x + 255) & ~(size_t)255; }

Codec64 codec_of(const WPlan& p) { return Codec64{p.codec_a, p.codec_c}; }

// Rule 4 (const 3, rounded down), plus one for inputs of 2^24 keys or more
// (at most 13), as for 32-bit keys; at least 7, so a wave-load of 128 keys
// never spans two subranges.
int wide_alpha(uint64_t n, uint32_t k) {
  int a = (int)std::floor(0.5 * (std::log2((double)n) - std::log2((double)k) + 3.0));
  if (n >= (1ull << 24)) a = a + 1 < 13 ? a + 1 : (a > 13 ? 13 : a);
  if (a < 7) a = 7;
  if (a > 24) a = 24;
  return a;
}

unsigned wgrid(uint64_t items, uint64_t per_block, unsigned cap) { return grid_for(items, per_block, cap); }

}  // namespace

int wide_plan(uint64_t n, uint32_t k, int dtype, bool vec, const drtopk_options_t* opt, WPlan* out, bool pos_in_ws) {
  WPlan p;
  p.n = n;
  p.k = k;
  p.dt = dtype;
  p.vec = vec;
  const int base = dtype & ~DRTOPK_SMALLEST;
  p.codec_a = base == DRTOPK_F64 ? 0x7FFFFFFFFFFFFFFFull : 0ull;
  p.codec_c = base == DRTOPK_U64 ? 0ull : 0x8000000000000000ull;
  if (dtype & DRTOPK_SMALLEST) p.codec_c = ~p.codec_c;
  int mode = opt ? opt->mode : 0;
  if (mode < 0 || mode > 2) return mode == 3 ? DRTOPK_EUNSUPPORTED : DRTOPK_EINVAL;
  if (opt && (opt->variant < 0 || opt->variant > 1)) return DRTOPK_EINVAL;
  if (opt && opt->beta > 1)  // one delegate per subrange (Rule 1) for 64-bit keys
    return (opt->beta == 2 || opt->beta == 4 || opt->beta == 8) ? DRTOPK_EUNSUPPORTED : DRTOPK_EINVAL;
  if (opt && opt->alpha > 24) return DRTOPK_EINVAL;
  if (opt && opt->alpha >= 0 && opt->alpha < 7) return DRTOPK_EINVAL;
  int alpha = (opt && opt->alpha >= 0) ? opt->alpha : wide_alpha(n, k);
  const auto subranges = [n](int a) { return (n + (1ull << a) - 1) >> a; };
  if (mode == 0) {
    mode = (n <= 8192 || (uint64_t)k * 16 > n) ? 2 : 1;
    // the threshold needs k delegates: shorten subranges down to 128 keys, else no delegates
    while (mode == 1 && subranges(alpha) < 4ull * k && alpha > 7 && !(opt && opt->alpha >= 0)) --alpha;
    if (mode == 1 && subranges(alpha) < (uint64_t)k) mode = 2;
  }
  if (mode == 1 && subranges(alpha) < (uint64_t)k) return DRTOPK_EINVAL;  // explicit alpha, too few delegates
  p.mode = mode;
  if (mode == 1) {
    p.alpha = alpha;
    const uint64_t L = 1ull << alpha;
    p.S = subranges(alpha);
    if (p.S >= (1ull << 32)) return DRTOPK_EINVAL;
    // survivors: t itself plus elements of the < k subranges whose delegate ranks above t
    const uint64_t c = (uint64_t)(k - 1) * L + 1;
    p.cap_c = c < n ? c : n;
    // a chunk holds whole wave steps (4 waves x 1024 keys) and whole subranges;
    // about 1024 workgroups, at most 4 MiB each
    const uint64_t cmin = 4 * (L > 1024 ? L : 1024);
    uint64_t ch = 1;
    while (ch * 2 <= n / 1024) ch *= 2;
    if (ch > (1ull << 19)) ch = 1ull << 19;
    if (ch < cmin) ch = cmin;
    p.chunk = ch;
  }
  if (k > (uint32_t)kWSmall) {
    uint64_t m = kWSmall;
    while (m < k) m <<= 1;
    p.M = m;
  }
  size_t off = 0;
  auto seg = [&](size_t bytes) {
    const size_t o = off;
    off = walign(off + bytes);
    return o;
  };
  p.off_ctl = seg(sizeof(WCtl));
  if (mode == 1) {
    p.off_dkey = seg(p.S * 8);
    p.off_didx = seg(p.S * 4);
    p.off_q = seg(p.S * 4);
    p.off_ckey = seg(p.cap_c * 8);
    p.off_cidx = seg(p.cap_c * 4);
  }
  p.off_okey = seg((size_t)k * 8);
  p.off_oidx = seg((size_t)k * 4);
  if (p.M) {
    p.off_A = seg(p.M * 16);
    p.off_B = seg(p.M * 16);
  }
  if (pos_in_ws) p.off_pos = seg((size_t)k * 4);
  p.total = off;
  *out = p;
  return DRTOPK_OK;
}

int wide_enqueue(const WPlan& p, const void* keys, void* ws, uint32_t* rec, void* out_vals_v, uint32_t* out_idx,
                 void* out_kth_v, bool kth_only, hipStream_t s) {
  const uint64_t* kp = static_cast<const uint64_t*>(keys);
  uint64_t* out_vals = kth_only ? nullptr : static_cast<uint64_t*>(out_vals_v);
  if (kth_only) out_idx = nullptr;
  uint64_t* out_kth = static_cast<uint64_t*>(out_kth_v);
  const Codec64 cd = codec_of(p);
  const uint32_t k = p.k;
  WCtl* ctl = at<WCtl>(ws, p.off_ctl);
  uint64_t* okey = at<uint64_t>(ws, p.off_okey);
  uint32_t* oidx = at<uint32_t>(ws, p.off_oidx);
  hipLaunchKernelGGL(k_winit, dim3(8), dim3(1024), 0, s, ctl, (uint32_t)p.S, (uint32_t)p.cap_c, rec);
  // which select decides the output: 1 (survivors, or the whole input in mode 2)
  const uint64_t* skey;
  const uint32_t* sidx;
  const uint32_t* scount;
  uint64_t sn;
  uint32_t scap;
  unsigned gsel;
  if (p.mode == 1) {
    uint64_t* dkey = at<uint64_t>(ws, p.off_dkey);
    uint32_t* didx = at<uint32_t>(ws, p.off_didx);
    uint32_t* Q = at<uint32_t>(ws, p.off_q);
    uint64_t* ckey = at<uint64_t>(ws, p.off_ckey);
    uint32_t* cidx = at<uint32_t>(ws, p.off_cidx);
    const unsigned gdel = (unsigned)((p.n + p.chunk - 1) / p.chunk);
    if (p.vec)
      hipLaunchKernelGGL(k_wdelegate<true>, dim3(gdel), dim3(kWThreads), 0, s, kp, p.n, p.alpha, p.chunk, cd, dkey,
                         didx);
    else
      hipLaunchKernelGGL(k_wdelegate<false>, dim3(gdel), dim3(kWThreads), 0, s, kp, p.n, p.alpha, p.chunk, cd, dkey,
                         didx);
    // t = the k-th largest delegate (Rule 2), exactly
    const unsigned gD = wgrid(p.S, kWThreads * 8, 1024);
    for (int pass = 0; pass < kWPasses; ++pass)
      hipLaunchKernelGGL(k_wpass<1>, dim3(gD), dim3(kWThreads), 0, s, dkey, didx, p.S, (const uint32_t*)nullptr,
                         0u, cd, pass, k, 0, ctl);
    hipLaunchKernelGGL(k_wfind<1>, dim3(gD), dim3(kWThreads), 0, s, dkey, didx, p.S, (const uint32_t*)nullptr, 0u,
                       cd, 0, ctl);
    hipLaunchKernelGGL(k_wqualify, dim3(gD), dim3(kWThreads), 0, s, dkey, didx, p.S, ctl, Q);
    hipLaunchKernelGGL(k_wscan, dim3(1024), dim3(kWThreads), 0, s, kp, p.n, p.alpha, cd, Q, ctl, ckey, cidx);
    hipLaunchKernelGGL(k_wfinal, dim3(1), dim3(kWSortThreads), 0, s, ckey, cidx, k, cd, ctl, out_vals, out_idx,
                       out_kth);
    skey = ckey;
    sidx = cidx;
    scount = &ctl->nc;
    sn = 0;
    scap = (uint32_t)p.cap_c;
    // expected survivors are about k on i.i.d. inputs; the grid strides over more
    const uint64_t est = (uint64_t)k * 16 + 4096;
    gsel = wgrid(est < p.cap_c ? est : p.cap_c, kWThreads * 8, 1024);
  } else {
    skey = kp;
    sidx = nullptr;
    scount = nullptr;
    sn = p.n;
    scap = 0;
    gsel = wgrid(p.n, kWThreads * 16, 2048);
  }
  // the k-th of the survivors (or of the whole input)
  for (int pass = 0; pass < kWPasses; ++pass) {
    if (p.mode == 1)
      hipLaunchKernelGGL(k_wpass<1>, dim3(gsel), dim3(kWThreads), 0, s, skey, sidx, sn, scount, scap, cd, pass, k, 1,
                         ctl);
    else
      hipLaunchKernelGGL(k_wpass<0>, dim3(gsel), dim3(kWThreads), 0, s, skey, sidx, sn, scount, scap, cd, pass, k, 1,
                         ctl);
  }
  if (p.mode == 1)
    hipLaunchKernelGGL(k_wfind<1>, dim3(gsel), dim3(kWThreads), 0, s, skey, sidx, sn, scount, scap, cd, 1, ctl);
  else
    hipLaunchKernelGGL(k_wfind<0>, dim3(gsel), dim3(kWThreads), 0, s, skey, sidx, sn, scount, scap, cd, 1, ctl);
  if (kth_only) {
    hipLaunchKernelGGL(k_wkth, dim3(1), dim3(64), 0, s, 1, cd, ctl, out_kth);
    return hipGetLastError() == hipSuccess ? (int)DRTOPK_OK : (int)DRTOPK_EDEVICE;
  }
  if (p.mode == 1)
    hipLaunchKernelGGL(k_wcompact<1>, dim3(gsel), dim3(kWThreads), 0, s, skey, sidx, sn, scount, scap, cd, 1, k, ctl,
                       okey, oidx);
  else
    hipLaunchKernelGGL(k_wcompact<0>, dim3(gsel), dim3(kWThreads), 0, s, skey, sidx, sn, scount, scap, cd, 1, k, ctl,
                       okey, oidx);
  if (k <= (uint32_t)kWSmall) {
    hipLaunchKernelGGL(k_wsort, dim3(1), dim3(kWSortThreads), 0, s, okey, oidx, k, cd, ctl, out_vals, out_idx,
                       out_kth);
  } else {
    u128* A = at<u128>(ws, p.off_A);
    u128* B = at<u128>(ws, p.off_B);
    hipLaunchKernelGGL(k_wblocksort, dim3((unsigned)(p.M / kWSmall)), dim3(kWSortThreads), 0, s, okey, oidx, k, ctl,
                       A);
    for (uint64_t run = kWSmall; run < p.M; run <<= 1) {
      const int last = (2 * run == p.M) ? 1 : 0;
      hipLaunchKernelGGL(k_wmerge, dim3((unsigned)(p.M / kWThreads)), dim3(kWThreads), 0, s, A, B, p.M, run, last, k,
                         cd, ctl, out_vals, out_idx, out_kth);
      u128* tmp = A;
      A = B;
      B = tmp;
    }
  }
  return hipGetLastError() == hipSuccess ? (int)DRTOPK_OK : (int)DRTOPK_EDEVICE;
}

int wide_counters(const WPlan& p, void* ws, uint64_t* scanned, uint64_t* candidates, uint32_t* err,
                  uint64_t* t_key_bits, uint32_t* t_idx) {
  WCtl h;
  if (hipMemcpy(&h, at<WCtl>(ws, p.off_ctl), sizeof(WCtl), hipMemcpyDeviceToHost) != hipSuccess)
    return DRTOPK_EDEVICE;
  *scanned = h.nq;
  *candidates = p.mode == 1 ? h.nc : p.n;
  *err = h.err;
  const u128 t = h.sel[0].t;
  const uint64_t key = (uint64_t)(t >> 32) ^ p.codec_c;
  *t_key_bits = p.mode == 1 ? key ^ (((uint64_t)((int64_t)key >> 63)) & p.codec_a) : 0;
  *t_idx = p.mode == 1 ? ~(uint32_t)t : 0;
  return DRTOPK_OK;
}

}  // namespace drtopk
