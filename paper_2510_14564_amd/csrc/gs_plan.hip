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
constexpr int kHeavyCap = 1024;    // at most this many heavy tiles are ordered

// Plan workspace in int32 values for ntiles tiles.
size_t plan_ints(int ntiles) { return kPlanHeader + 4 * static_cast<size_t>(ntiles); }

// counts == NULL: a tile's count is its list length from ranges.
__global__ __launch_bounds__(kPlanThreads) void k_tile_plan(int ntiles, const uint2* __restrict__ ranges,
                                                            const uint32_t* __restrict__ counts,
                                                            float heavy_factor, int light_max,
                                                            int32_t* __restrict__ plan) {
  __shared__ float s_red[kPlanThreads / 64];
  __shared__ uint32_t s_hw[kHeavyCap];
  __shared__ int s_ht[kHeavyCap];
  __shared__ int s_wave_cnt[3][kPlanThreads / 64];
  __shared__ int s_base[3];
  __shared__ int s_over;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int32_t* const order = plan + kPlanHeader;
  int32_t* const med = order + ntiles;           // staging: medium tiles in tile order
  int32_t* const lig = med + ntiles;             // staging: light tiles in tile order
  int32_t* const over = lig + ntiles;            // staging: heavy tiles beyond the cap
  auto count_of = [&](int t) -> uint32_t { return counts ? counts[t] : (ranges[t].y - ranges[t].x); };

  float sum = 0.f;
  for (int t = tid; t < ntiles; t += kPlanThreads) sum += static_cast<float>(count_of(t));
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
  if (lane == 0) s_red[wave] = sum;
  if (tid < 3) s_base[tid] = 0;
  if (tid == 0) s_over = 0;
  __syncthreads();
  float total = 0.f;
  for (int w = 0; w < kPlanThreads / 64; ++w) total += s_red[w];
  const float thresh = fmaxf(heavy_factor * total / static_cast<float>(max(ntiles, 1)),
                             static_cast<float>(light_max));
  const uint64_t below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));

  // chunked, order-preserving split into the three classes
  for (int c0 = 0; c0 < ntiles; c0 += kPlanThreads) {
    const int t = c0 + tid;
    int cls = -1;
    uint32_t w = 0;
    if (t < ntiles) {
      w = count_of(t);
      cls = static_cast<float>(w) > thresh ? 0 : (static_cast<int>(w) <= light_max ? 2 : 1);
    }
    int rank = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const uint64_t bal = __ballot(cls == k);
      if (cls == k) rank = __popcll(bal & below);
      if (lane == 0) s_wave_cnt[k][wave] = __popcll(bal);
    }
    __syncthreads();
    if (cls >= 0) {
      int pos = s_base[cls] + rank;
      for (int v = 0; v < wave; ++v) pos += s_wave_cnt[cls][v];
      if (cls == 0) {
        if (pos < kHeavyCap) { s_hw[pos] = w; s_ht[pos] = t; }
        else over[atomicAdd(&s_over, 1)] = t;
      } else if (cls == 1) {
        med[pos] = t;
      } else {
        lig[pos] = t;
      }
    }
    __syncthreads();
    if (tid < 3) {
      int add = 0;
      for (int v = 0; v < kPlanThreads / 64; ++v) add += s_wave_cnt[tid][v];
      s_base[tid] += add;
    }
    __syncthreads();
  }
  const int H = min(s_base[0], kHeavyCap), O = s_over, M = s_base[1], L = s_base[2];
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
  for (int i = tid; i < M; i += kPlanThreads) order[H + i] = med[i];
  for (int i = tid; i < O; i += kPlanThreads) order[H + M + i] = over[i];
  for (int i = tid; i < L; i += kPlanThreads) order[H + M + O + i] = lig[i];
  if (tid == 0) {
    plan[0] = H;
    plan[1] = M + O;
    plan[2] = L;
    plan[3] = H + M + O + (L + 3) / 4;
  }
}

gs_status launch_tile_plan(int ntiles, const uint32_t* ranges, const uint32_t* counts, float heavy_factor,
                           int light_max, int32_t* plan, hipStream_t s) {
  k_tile_plan<<<1, kPlanThreads, 0, s>>>(ntiles, reinterpret_cast<const uint2*>(ranges), counts, heavy_factor,
                                         light_max, plan);
  return check_launch("k_tile_plan");
}

}  // namespace gs
