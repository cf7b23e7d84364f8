// Per-tile work plan: which workgroup takes which tile, built on the device
// from a measured per-tile work count (no host synchronisation).
//
// Paper: Sec. IV (workload imbalance across tiles of dense and sparse
// regions, and adaptive thread-block merging by a density measure).  Here the
// measure is the tile's work count -- its list length before the forward,
// the largest number of entries any of its pixels walks (n_contrib) before the
// backward.  Tiles whose count exceeds kHeavyFactor times the mean are
// *heavy* and are taken first, largest first, so that the longest workgroups
// start at the beginning of the launch instead of forming its tail; tiles
// with at most kLightMax entries are *light* and are merged four to a
// workgroup (one wave per tile, four pixels per lane); the rest keep the
// plain one-workgroup-per-tile form.  Every tile's arithmetic is the same in
// every form, so the image and gradients do not depend on the plan.
//
// Plan layout (int32): [0] heavy count H, [1] medium count M, [2] light count
// L, [3] workgroups needed H + M + ceil(L / 4), then from kPlanHeader the
// tiles: heavy by decreasing count (ties by tile index), medium and light in
// tile order.
#include "gs_internal.h"

namespace gs {

constexpr int kPlanThreads = 1024;
constexpr int kPlanRegs = 16;   // tiles per thread held in registers by k_batch_plan
constexpr int kHeavyCap = 1024;    // at most this many heavy tiles are ordered

// Plan workspace in int32 values for ntiles tiles.
size_t plan_ints(int ntiles) { return kPlanHeader + static_cast<size_t>(ntiles); }

// counts == NULL: a tile's count is its list length from ranges.  Thread t
// owns a contiguous run of tiles, so one block-wide scan of three class
// counts gives every tile its place (tile order inside each class).
__global__ __launch_bounds__(kPlanThreads) void k_tile_plan(int ntiles, const uint2* __restrict__ ranges,
                                                            const uint32_t* __restrict__ counts,
                                                            float heavy_factor, int light_max,
                                                            int32_t* __restrict__ plan) {
  __shared__ float s_red[kPlanThreads / 64];
  __shared__ uint32_t s_scan[3][kPlanThreads / 64];
  __shared__ uint32_t s_hw[kHeavyCap];
  __shared__ int s_ht[kHeavyCap];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int32_t* const order = plan + kPlanHeader;
  auto count_of = [&](int t) -> uint32_t { return counts ? counts[t] : (ranges[t].y - ranges[t].x); };
  const int per = (ntiles + kPlanThreads - 1) / kPlanThreads;
  const int t0 = min(ntiles, tid * per), t1 = min(ntiles, t0 + per);

  float sum = 0.f;
  for (int t = t0; t < t1; ++t) sum += static_cast<float>(count_of(t));
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
  if (lane == 0) s_red[wave] = sum;
  __syncthreads();
  float total = 0.f;
  for (int w = 0; w < kPlanThreads / 64; ++w) total += s_red[w];
  const float thresh = fmaxf(heavy_factor * total / static_cast<float>(max(ntiles, 1)),
                             static_cast<float>(light_max));
  auto cls_of = [&](uint32_t w) -> int {
    return static_cast<float>(w) > thresh ? 0 : (static_cast<int>(w) <= light_max ? 2 : 1);
  };
  // per-thread class counts, then an exclusive scan over threads (wave
  // shuffles, then the wave totals in LDS)
  uint32_t c[3] = {0u, 0u, 0u};
  for (int t = t0; t < t1; ++t) ++c[cls_of(count_of(t))];
  uint32_t ex[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    uint32_t incl = c[k];
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t v = __shfl_up(incl, o, 64);
      if (lane >= o) incl += v;
    }
    ex[k] = incl - c[k];
    if (lane == 63) s_scan[k][wave] = incl;
  }
  __syncthreads();
  uint32_t tot[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    uint32_t before = 0, all = 0;
    for (int w = 0; w < kPlanThreads / 64; ++w) {
      const uint32_t v = s_scan[k][w];
      before += (w < wave) ? v : 0u;
      all += v;
    }
    ex[k] += before;
    tot[k] = all;
  }
  const int H = static_cast<int>(min(tot[0], static_cast<uint32_t>(kHeavyCap)));
  const int O = static_cast<int>(tot[0]) - H;          // heavy beyond the cap: placed after the medium ones
  const int M = static_cast<int>(tot[1]), L = static_cast<int>(tot[2]);
  for (int t = t0; t < t1; ++t) {
    const uint32_t w = count_of(t);
    const int k = cls_of(w);
    const int pos = static_cast<int>(ex[k]++);
    if (k == 0) {
      if (pos < kHeavyCap) { s_hw[pos] = w; s_ht[pos] = t; }
      else order[H + M + (pos - kHeavyCap)] = t;
    } else if (k == 1) {
      order[H + pos] = t;
    } else {
      order[H + M + O + pos] = t;
    }
  }
  __syncthreads();
  // heavy tiles: rank by (count descending, tile ascending)
  for (int i = tid; i < H; i += kPlanThreads) {
    const uint32_t wi = s_hw[i];
    const int ti = s_ht[i];
    int r = 0;
    for (int j = 0; j < H; ++j) {
      const uint32_t wj = s_hw[j];
      r += (wj > wi || (wj == wi && s_ht[j] < ti)) ? 1 : 0;
    }
    order[r] = ti;
  }
  if (tid == 0) {
    plan[0] = H;
    plan[1] = M + O;
    plan[2] = L;
    plan[3] = H + M + O + (L + 3) / 4;
  }
}

// Backward work items: every batch of 256 list entries that some pixel of
// the tile walks becomes its own workgroup, (tile, batch) in tile order.  A
// tile's walk length is min(list length, largest n_contrib) -- the count the
// forward left in `work`.  Tiles with a count of at most light_max go to the
// light list instead (a plan with H = M = 0), or nowhere when light is NULL
// (with light_max = 0: the tiles whose pixels blend nothing).
// items: [0] item count, from kPlanHeader pairs (tile, batch).
// Workgroup 0 builds the plan; the others, if any, clear zero[0, zero_n4)
// meanwhile (the backward's accumulator rows), so that the fill runs under
// the one-workgroup plan instead of after it.
__global__ __launch_bounds__(kPlanThreads) void k_batch_plan(int ntiles, const uint2* __restrict__ ranges,
                                                             const uint32_t* __restrict__ work, int light_max,
                                                             int32_t* __restrict__ items,
                                                             int32_t* __restrict__ light,
                                                             float4* __restrict__ zero, int64_t zero_n4) {
  if (blockIdx.x > 0) {
    const int64_t stride = static_cast<int64_t>(gridDim.x - 1) * kPlanThreads;
    for (int64_t i = static_cast<int64_t>(blockIdx.x - 1) * kPlanThreads + threadIdx.x; i < zero_n4; i += stride)
      zero[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  __shared__ uint32_t s_scan[2][kPlanThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int per = (ntiles + kPlanThreads - 1) / kPlanThreads;
  const int t0 = min(ntiles, tid * per), t1 = min(ntiles, t0 + per);
  auto batches_of = [&](uint2 rg, uint32_t wk) -> uint32_t {
    const uint32_t len = min(rg.y - rg.x, wk);
    return static_cast<int>(wk) <= light_max ? 0u : (len + 255u) / 256u;
  };
  auto is_light = [&](uint32_t wk) -> bool { return wk > 0u && static_cast<int>(wk) <= light_max; };
  // up to kPlanRegs tiles per thread are read once, all loads in flight
  // together; larger grids read them in the loops
  const bool regs = per <= kPlanRegs;
  uint32_t nbr[kPlanRegs];
  bool lgt[kPlanRegs];
  uint32_t c[2] = {0u, 0u};
  if (regs) {
    uint2 rg[kPlanRegs];
    uint32_t wk[kPlanRegs];
#pragma unroll
    for (int k = 0; k < kPlanRegs; ++k) {
      rg[k] = t0 + k < t1 ? ranges[t0 + k] : make_uint2(0u, 0u);
      wk[k] = t0 + k < t1 ? work[t0 + k] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kPlanRegs; ++k) {
      nbr[k] = t0 + k < t1 ? batches_of(rg[k], wk[k]) : 0u;
      lgt[k] = t0 + k < t1 && is_light(wk[k]);
      c[0] += nbr[k];
      c[1] += lgt[k] ? 1u : 0u;
    }
  } else {
    for (int t = t0; t < t1; ++t) {
      c[0] += batches_of(ranges[t], work[t]);
      c[1] += is_light(work[t]) ? 1u : 0u;
    }
  }
  uint32_t ex[2], tot[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    uint32_t incl = c[k];
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t v = __shfl_up(incl, o, 64);
      if (lane >= o) incl += v;
    }
    ex[k] = incl - c[k];
    if (lane == 63) s_scan[k][wave] = incl;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    uint32_t before = 0, all = 0;
    for (int w = 0; w < kPlanThreads / 64; ++w) {
      const uint32_t v = s_scan[k][w];
      before += (w < wave) ? v : 0u;
      all += v;
    }
    ex[k] += before;
    tot[k] = all;
  }
  // (tile, batch) pairs, two per 16-byte store where they pair up (items
  // is 16-byte aligned)
  int2* const pairs = reinterpret_cast<int2*>(items + kPlanHeader);
  int4* const quads = reinterpret_cast<int4*>(items + kPlanHeader);
  auto put = [&](int t, uint32_t nb, bool lt) {
    uint32_t e = ex[0], j = 0;
    if ((e & 1u) && j < nb) pairs[e++] = make_int2(t, static_cast<int32_t>(j++));
    for (; j + 1 < nb; j += 2, e += 2)
      quads[e >> 1] = make_int4(t, static_cast<int32_t>(j), t, static_cast<int32_t>(j + 1));
    if (j < nb) pairs[e++] = make_int2(t, static_cast<int32_t>(j++));
    ex[0] = e;
    if (light && lt) light[kPlanHeader + ex[1]++] = t;
  };
  if (regs) {
#pragma unroll
    for (int k = 0; k < kPlanRegs; ++k)
      if (t0 + k < t1) put(t0 + k, nbr[k], lgt[k]);
  } else {
    for (int t = t0; t < t1; ++t) put(t, batches_of(ranges[t], work[t]), is_light(work[t]));
  }
  if (tid == 0) {
    items[0] = static_cast<int32_t>(tot[0]);
    if (light) { light[0] = 0; light[1] = 0; light[2] = static_cast<int32_t>(tot[1]); light[3] = 0; }
  }
}

gs_status launch_batch_plan(int ntiles, const uint32_t* ranges, const uint32_t* work, int light_max, int32_t* items,
                            int32_t* light, float4* zero, int64_t zero_n4, hipStream_t s) {
  const unsigned fill = zero_n4 > 0 ? static_cast<unsigned>(std::min<int64_t>(ceil_div(zero_n4, kPlanThreads), 1024)) : 0u;
  { TimedLaunch gs_tl("k_batch_plan", s); k_batch_plan<<<1 + fill, kPlanThreads, 0, s>>>(ntiles, reinterpret_cast<const uint2*>(ranges), work, light_max, items,
                                          light, zero, zero_n4); }
  return check_launch("k_batch_plan");
}

gs_status launch_tile_plan(int ntiles, const uint32_t* ranges, const uint32_t* counts, float heavy_factor,
                           int light_max, int32_t* plan, hipStream_t s) {
  { TimedLaunch gs_tl("k_tile_plan", s); k_tile_plan<<<1, kPlanThreads, 0, s>>>(ntiles, reinterpret_cast<const uint2*>(ranges), counts, heavy_factor,
                                         light_max, plan); }
  return check_launch("k_tile_plan");
}

}  // namespace gs
