// Front-to-back compositing over per-tile depth-ordered lists, and its backward.
//
// Paper: Sec. II-A, C = sum_i c_i alpha_i prod_{j<i} (1 - alpha_j) over the
// Gaussians reaching a pixel in depth order, with alpha from the projected
// Gaussian G(x) and the opacity; Sec. IV-C.1, 16x16 pixel tiles sharing one
// list; Sec. V, interleaved per-Gaussian records loaded in batches into fast
// on-chip memory.
//
// One 256-thread workgroup per tile, one pixel per thread (a wave64 covers 4
// rows of 16 pixels).  The tile's records are gathered in batches of 256 into
// LDS (one 48-byte record per thread, three 16-byte loads) and every lane
// reads them back as broadcasts.  The per-pair body is branch-free; a wave
// leaves a batch as soon as all its lanes are done (ballot), and the workgroup
// leaves the tile when all 256 pixels are done.  Tiles are mapped so that
// neighbouring tiles run on the same XCD and share its L2.
//
// This file is compiled with -ffp-contract=off: the forward and the backward
// evaluate alpha through the same inline function with explicit fmaf, so the
// backward re-derives exactly the forward's skip decisions and transmittances.
#include "gs_internal.h"

#include <type_traits>

namespace gs {

constexpr int kBatch = 256;
constexpr int kUnroll = 4;
constexpr float kLog2e = 1.4426950408889634f;

// Transmittance checkpoints: the forward stores every pixel's T at the start of
// each 256-entry batch b >= 1 of its tile, in slot floor(S_t / 256) + t + b
// (S_t = first entry of tile t).  Slots of different tiles never collide and
// all are below floor(K / 256) + T + 1.
__device__ __forceinline__ size_t ckpt_slot0(uint32_t start, int tile) {
  return static_cast<size_t>(start / kBatch) + static_cast<size_t>(tile);
}

// Records are staged in LDS with the conic (A, B, C) pre-scaled by
// -log2(e)/2: a = -log2(e) A / 2, b = -log2(e) B / 2, c = -log2(e) C / 2, so
// that with n = (a dx + b dy, b dx + c dy) the base-2 exponent is
//   p2 = dx n.x + dy n.y = power * log2(e),
// alpha's Gaussian factor is a single v_exp_f32, and n (= -log2(e)/2 times
// the conic applied to d) is what the backward's covariance gradient needs:
// p = (u, v, a, b), q = (c, opacity, r, g).  Slots past the end of a batch
// hold a null record (opacity 0), which every pixel skips.
// p2 (base-2 power), 2^p2, the unclamped o 2^p2 and n for one (pixel, entry) pair.
__device__ __forceinline__ void eval_pair(const float4& p, const float4& q, float px, float py, float& dx,
                                          float& dy, float& p2, float& eg, float& og, float& nx, float& ny) {
  dx = p.x - px;
  dy = p.y - py;
  nx = fmaf(p.z, dx, p.w * dy);
  ny = fmaf(q.x, dy, p.w * dx);
  p2 = fmaf(dx, nx, dy * ny);
  eg = __builtin_amdgcn_exp2f(p2);
  og = q.y * eg;
}

// Wave w of a tile's workgroup covers the 8x8 quadrant (w & 1, w >> 1); lane
// l of it the pixel (l & 7, l >> 3) inside the quadrant.
__device__ __forceinline__ void tile_pixel(int tid, int& lx, int& ly) {
  const int w = tid >> 6, l = tid & 63;
  lx = ((w & 1) << 3) + (l & 7);
  ly = ((w >> 1) << 3) + (l >> 3);
}

// Smallest q(d) = A dx^2 + 2 B dx dy + C dy^2 over the rectangle
// dx in [xa, xb], dy in [ya, yb] (A, C > 0, A C > B^2): zero if it holds
// the origin, else the least of the four edge minima (on an edge q is a
// parabola in the free coordinate, minimised at -B X / C or -B Y / A and
// clamped to the edge).
__device__ __forceinline__ float conic_min_rect(float A, float B, float C, float iA, float iC, float xa, float xb,
                                                float ya, float yb) {
  if (xa <= 0.0f && xb >= 0.0f && ya <= 0.0f && yb >= 0.0f) return 0.0f;
  float best = 3.0e38f;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const float X = k ? xb : xa;
    const float y = fminf(fmaxf(-B * X * iC, ya), yb);
    best = fminf(best, fmaf(fmaf(A, X, 2.0f * B * y), X, C * y * y));
    const float Y = k ? yb : ya;
    const float x = fminf(fmaxf(-B * Y * iA, xa), xb);
    best = fminf(best, fmaf(fmaf(C, Y, 2.0f * B * x), Y, A * x * x));
  }
  return best;
}

// Quadrants of the tile whose pixel centres can reach alpha >= 1/255 (bit w =
// quadrant of wave w): first the record's alpha-support box, then the exact
// support ellipse q(d) <= rho^2 = 2 ln(255 o) against each remaining
// quadrant's rectangle of pixel centres.  A wave whose bit is clear would skip
// the entry at every pixel anyway.  The ellipse test takes twice the box's
// slack (rho^2 x 1.04 + 4e-4, the rectangle widened by the box's 1e-3 px +
// 1e-6 |u|), covering the FP32 error of both its own evaluation and the
// per-pixel one for footprints with condition number up to 1e5 (larger ones
// have an unbounded box and keep their box mask).
__device__ __forceinline__ uint32_t quad_mask(const float4& r0, const float4& r1, const float4& r2, float x0,
                                              float y0) {
  const float u = r0.x, v = r0.y, ex = r2.z, ey = r2.w;
  if (!(ex >= 0.0f)) return 0u;
  const bool xl = (u - ex <= x0 + 7.5f) && (u + ex >= x0 + 0.5f);
  const bool xr = (u - ex <= x0 + 15.5f) && (u + ex >= x0 + 8.5f);
  const bool yt = (v - ey <= y0 + 7.5f) && (v + ey >= y0 + 0.5f);
  const bool yb = (v - ey <= y0 + 15.5f) && (v + ey >= y0 + 8.5f);
  const uint32_t box = (xl && yt ? 1u : 0u) | (xr && yt ? 2u : 0u) | (xl && yb ? 4u : 0u) | (xr && yb ? 8u : 0u);
  if (box == 0u || !(ex < 1.0e30f)) return box;
  const float A = r0.z, B = r0.w, C = r1.x;
  const float iA = 1.0f / A, iC = 1.0f / C;
  const float rho2 = (2.0f * 1.04f) * logf(255.0f * r1.y) + 4e-4f;
  const float dl = 1e-3f + 1e-6f * fmaxf(fabsf(u), fabsf(v));
  uint32_t m = 0u;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (!((box >> k) & 1u)) continue;
    const float xa = x0 + ((k & 1) ? 8.5f : 0.5f) - dl - u;
    const float ya = y0 + ((k & 2) ? 8.5f : 0.5f) - dl - v;
    if (conic_min_rect(A, B, C, iA, iC, xa, xa + 7.0f + 2.0f * dl, ya, ya + 7.0f + 2.0f * dl) <= rho2) m |= 1u << k;
  }
  return m;
}

constexpr int kNull = kBatch;           // LDS slot of a null record (opacity 0)

// A value every lane of the wave holds, moved to a scalar register so that
// branches on it are scalar.
__device__ __forceinline__ uint32_t uniform(uint32_t x) {
  return static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(x)));
}
constexpr int kListStride = kBatch + 4; // per-wave list of staged slots, padded to kUnroll

// The forward's only work count before it runs is the list length, which does
// not predict where pixels saturate (measured: ordering the forward by it made
// the launch slower), so its plan never marks tiles heavy and serves only to
// merge light tiles.
constexpr float kHeavyFactorFwd = 3.0e38f;

// Tile of workgroup `bid`.  Plain form: XCD-aware spatial map.  With a plan
// (balanced form): heavy tiles first, largest first, one per workgroup in
// dispatch order (so they spread over the XCDs and start at once), then the
// others through the XCD-aware map of their own sequence.
// Light tiles (no more than kLightMax entries to walk) go to the merged
// kernels instead; -1 = nothing for this workgroup.
__device__ __forceinline__ int tile_of_block(const int32_t* __restrict__ plan, int bid, int ntiles) {
  if (!plan) return xcd_remap(bid, ntiles);
  const int H = plan[0], M = plan[1];
  const int32_t* order = plan + kPlanHeader;
  if (bid < H) return order[bid];
  return bid < H + M ? order[H + xcd_remap(bid - H, M)] : -1;
}

constexpr int kLightMax = 64;

// Per-wave staging of a light tile's entries (one batch of at most 64).
struct LightStage {
  float4 p[kLightMax];
  float4 q[kLightMax];
  float2 c[kLightMax];                  // blue, quadrant mask bits
  uint32_t gid[kLightMax];
};

// Light tile of wave `wave` of workgroup `bid`, or -1.
__device__ __forceinline__ int light_tile(const int32_t* __restrict__ plan, int bid, int wave) {
  const int H = plan[0], M = plan[1], L = plan[2];
  const int i = bid * 4 + wave;
  return i < L ? plan[kPlanHeader + H + M + i] : -1;
}

__device__ __forceinline__ void stage_light(LightStage& ls, const float4* __restrict__ rec,
                                            const uint32_t* __restrict__ point_list, uint32_t first, int cnt,
                                            float x0, float y0, int lane) {
  if (lane < cnt) {
    const uint32_t gid = point_list[first + lane];
    const float4 r0 = rec[3 * gid];
    const float4 r1 = rec[3 * gid + 1];
    const float4 r2 = rec[3 * gid + 2];
    ls.p[lane] = make_float4(r0.x, r0.y, -0.5f * kLog2e * r0.z, -0.5f * kLog2e * r0.w);
    ls.q[lane] = make_float4(-0.5f * kLog2e * r1.x, r1.y, r1.z, r1.w);
    ls.c[lane] = make_float2(r2.x, __uint_as_float(quad_mask(r0, r1, r2, x0, y0)));
    ls.gid[lane] = gid;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Shared per-batch staging: records (pre-scaled conic), colour + quadrant mask,
// and each wave's list of the staged slots it must visit, in list order and
// padded with the null slot to a multiple of kUnroll.
// One staged record, all fields at one LDS address (a wave-uniform index
// reads them with one base register and immediate offsets).
struct StageRec {
  float4 p;
  float4 q;
  float2 c;                             // blue, quadrant mask bits
  uint32_t gid;
  uint32_t pad;
};
struct Stage {
  StageRec r[kBatch + 1];
  alignas(16) uint32_t list[4][kListStride];
  int len[4];
};

__device__ __forceinline__ void stage_batch(Stage& st, const float4* __restrict__ rec,
                                            const uint32_t* __restrict__ point_list, uint32_t first, int cnt,
                                            float x0, float y0) {
  const int t = threadIdx.x;
  if (t < cnt) {
    const uint32_t gid = point_list[first + t];
    const float4 r0 = rec[3 * gid];
    const float4 r1 = rec[3 * gid + 1];
    const float4 r2 = rec[3 * gid + 2];
    st.r[t].p = make_float4(r0.x, r0.y, -0.5f * kLog2e * r0.z, -0.5f * kLog2e * r0.w);
    st.r[t].q = make_float4(-0.5f * kLog2e * r1.x, r1.y, r1.z, r1.w);
    st.r[t].c = make_float2(r2.x, __uint_as_float(quad_mask(r0, r1, r2, x0, y0)));
    st.r[t].gid = gid;
  } else {
    st.r[t].p = make_float4(0.f, 0.f, 0.f, 0.f);
    st.r[t].q = make_float4(0.f, 0.f, 0.f, 0.f);
    st.r[t].c = make_float2(0.f, __uint_as_float(0u));
    st.r[t].gid = 0u;
  }
}

// The wave's LDS writes are visible to its own lanes (no workgroup barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Stream compaction of the staged batch for this wave (ballot + prefix count).
// all = true keeps every staged entry (no culling).
__device__ __forceinline__ void build_list(Stage& st, int cnt, bool all) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint64_t below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  int L = 0;
#pragma unroll
  for (int r = 0; r < kBatch / 64; ++r) {
    const int j = r * 64 + lane;
    const bool in = (j < cnt) && (all || ((__float_as_uint(st.r[j].c.y) >> wave) & 1u));
    const uint64_t bal = __ballot(in);
    if (in) st.list[wave][L + __popcll(bal & below)] = static_cast<uint32_t>(j);
    L += __popcll(bal);
  }
  const int Lp = (L + kUnroll - 1) & ~(kUnroll - 1);
  if (lane < Lp - L) st.list[wave][L + lane] = kNull;
  if (lane == 0) st.len[wave] = Lp;
}

// ------------------------------------------------------ colour-hash sampling
// Sec. IV-C.1 (similarity-based sampling with colour hashing), an optional
// approximate mode of both compositing directions.  Each channel's 8-bit value
// v8 = floor(255 clamp(c, 0, 1) + 1/2) (FP32, product then sum; NaN counts as
// 0) gives the level v8 >> 4 = floor(v8 / 256 * 16), and the bucket is
// R_q 256 + G_q 16 + B_q (4096 buckets).  Inside each 256-entry batch of a
// tile's list (the LDS staging window), the entries whose colours share a
// bucket form a group; a group of two or more is composited as its front-most
// member with the members' mean colour and the accumulated opacity
// 1 - prod (1 - o_j), and its other members are not composited.  The grouping
// is done in LDS with a 4096-bucket table: per bucket one byte per wave, the
// lane (+1) of the wave's first member, and per wave-first member the ballot
// mask of its wave's members, so a representative walks its members in list
// order (wave by wave, lanes ascending) and the result does not depend on
// timing.  The backward regroups each batch identically, so the aggregated
// opacity and colour -- and every skip and stop decision -- are the forward's
// bit for bit; the gradient that reaches a group's aggregated opacity and
// colour is handed to its members by the chain rule (opacity: times the
// product of the other members' (1 - o); colour: over the group size), the
// footprint's gradient to the representative alone.
constexpr int kChsBuckets = 4096;
constexpr uint32_t kChsNone = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t chs_level(float c) {
  const float cc = c > 0.0f ? fminf(c, 1.0f) : 0.0f;
  const float t = __fadd_rn(__fmul_rn(cc, 255.0f), 0.5f);
  return static_cast<uint32_t>(floorf(t)) >> 4;
}

__device__ __forceinline__ uint32_t chs_bucket(float r, float g, float b) {
  return chs_level(r) * 256u + chs_level(g) * 16u + chs_level(b);
}

struct ChsStage {
  uint32_t table[kChsBuckets];  // byte w: 1 + lane of wave w's first member of the bucket (0: none)
  uint64_t wmask[kBatch];       // at a wave's first member of a bucket: the wave's members of it
  uint32_t rep[kBatch];         // slot of the group's representative (groups of >= 2), else kChsNone
  float share_o[kBatch];        // product over the group's other members of (1 - o)
  float inv_n[kBatch];          // 1 / group size
};

// Thread t's bucket and whether it is its wave's first member of the bucket
// (it then resets the bucket's table word once nobody reads it any more).
struct ChsSlot {
  uint32_t bucket;
  bool wave_first;
};

__device__ __forceinline__ void chs_clear(ChsStage& cs) {
  for (int i = threadIdx.x; i < kChsBuckets; i += 256) cs.table[i] = 0u;
}

// Alpha-support box of a representative whose opacity rose from o to o_hat:
// the half-extents grow with rho = sqrt(2 ln(255 o) 1.02 + 2e-4) (the slack
// the projection gives rho^2), so the pixel-independent part of each extent
// scales by rho_hat / rho (times 1 + 1e-5 for the rounding of the rescale).
__device__ __forceinline__ void chs_support(float o, float o_hat, float u, float v, float& ex, float& ey) {
  if (!(ex < 1.0e30f)) return;                 // unbounded box stays unbounded
  const float lo_new = logf(255.0f * o_hat);
  if (!(lo_new > 0.0f)) { ex = -1.0f; ey = -1.0f; return; }
  const float lo_old = logf(255.0f * o);
  if (!(lo_old > 0.0f) || !(ex >= 0.0f)) { ex = 3.0e38f; ey = 3.0e38f; return; }
  const float scale = sqrtf((2.0f * lo_new * 1.02f + 2e-4f) / (2.0f * lo_old * 1.02f + 2e-4f)) * (1.0f + 1e-5f);
  const float mx = 1e-3f + 1e-6f * fabsf(u), my = 1e-3f + 1e-6f * fabsf(v);
  ex = fmaxf(ex - mx, 0.0f) * scale + mx;
  ey = fmaxf(ey - my, 0.0f) * scale + my;
}

// Groups the staged batch (slots 0..cnt-1 in list order) by colour bucket and
// rewrites it in place: a representative of a group of two or more gets the
// mean colour, the accumulated opacity and the quadrant mask of that opacity;
// the other members get an empty quadrant mask.  SHARES also fills rep,
// share_o and inv_n for the backward.  cs.table must be zero on entry; call
// chs_release after the next workgroup barrier.  One barrier inside.
template <bool SHARES>
__device__ ChsSlot chs_group(Stage& st, ChsStage& cs, const float4* __restrict__ rec, int cnt, float x0, float y0) {
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const bool valid = t < cnt;
  const uint32_t h = valid ? chs_bucket(st.r[t].q.z, st.r[t].q.w, st.r[t].c.x) : 0u;
  // lanes of this wave whose bucket equals this lane's (12 ballots)
  uint64_t same = __ballot(valid);
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const bool bit = (h >> k) & 1u;
    const uint64_t b = __ballot(bit);
    same &= bit ? b : ~b;
  }
  const bool wfirst = valid && static_cast<int>(__builtin_ctzll(same)) == lane;
  if (wfirst) {
    cs.wmask[t] = same;
    atomicOr(&cs.table[h], static_cast<uint32_t>(lane + 1) << (8 * wave));
  }
  if (SHARES) cs.rep[t] = kChsNone;
  __syncthreads();
  if (valid) {
    const uint32_t word = cs.table[h];
    const int w0 = static_cast<int>(__builtin_ctz(word)) >> 3;
    const int r = 64 * w0 + static_cast<int>((word >> (8 * w0)) & 0xFFu) - 1;
    int n = 0;
    for (int w = w0; w < 4; ++w) {
      const uint32_t b = (word >> (8 * w)) & 0xFFu;
      if (b) n += __popcll(cs.wmask[64 * w + static_cast<int>(b) - 1]);
    }
    if (n > 1) {
      if (SHARES) {
        cs.rep[t] = static_cast<uint32_t>(r);
        cs.inv_n[t] = 1.0f / static_cast<float>(n);
      }
      if (t == r) {
        // members in list order: waves ascending, lanes ascending
        float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, keep = 1.0f;
        for (int w = w0; w < 4; ++w) {
          const uint32_t b = (word >> (8 * w)) & 0xFFu;
          if (!b) continue;
          uint64_t m = cs.wmask[64 * w + static_cast<int>(b) - 1];
          while (m) {
            const int j = 64 * w + static_cast<int>(__builtin_ctzll(m));
            m &= m - 1;
            const float4 q = st.r[j].q;
            s0 += q.z;
            s1 += q.w;
            s2 += st.r[j].c.x;
            if (SHARES) cs.share_o[j] = keep;   // product over the members before j
            keep *= 1.0f - q.y;
          }
        }
        if (SHARES) {
          // times the product over the members after j
          float suf = 1.0f;
          for (int w = 3; w >= w0; --w) {
            const uint32_t b = (word >> (8 * w)) & 0xFFu;
            if (!b) continue;
            uint64_t m = cs.wmask[64 * w + static_cast<int>(b) - 1];
            while (m) {
              const int bit = 63 - static_cast<int>(__builtin_clzll(m));
              m &= ~(1ull << bit);
              const int j = 64 * w + bit;
              cs.share_o[j] *= suf;
              suf *= 1.0f - st.r[j].q.y;
            }
          }
        }
        const float inv = 1.0f / static_cast<float>(n);
        const float o_hat = 1.0f - keep;
        const uint32_t gid = st.r[t].gid;
        const float4 r0 = rec[3 * gid];
        float4 r1 = rec[3 * gid + 1];
        float4 r2 = rec[3 * gid + 2];
        chs_support(r1.y, o_hat, r0.x, r0.y, r2.z, r2.w);
        r1.y = o_hat;
        float4 q = st.r[t].q;
        q.y = o_hat;
        q.z = s0 * inv;
        q.w = s1 * inv;
        st.r[t].q = q;
        st.r[t].c = make_float2(s2 * inv, __uint_as_float(quad_mask(r0, r1, r2, x0, y0)));
      } else {
        st.r[t].c.y = __uint_as_float(0u);  // not composited: no wave visits it
      }
    }
  }
  return ChsSlot{h, wfirst};
}

__device__ __forceinline__ void chs_release(ChsStage& cs, const ChsSlot& sl) {
  if (sl.wave_first) cs.table[sl.bucket] = 0u;
}

// ------------------------------------------------------------------- forward

// One (pixel, entry) step of the front-to-back walk; m1 = 1 + the entry's
// position in the tile list.  Shared by every work-split form so that they
// produce the same bits.  Returns whether the entry was blended.
__device__ __forceinline__ bool fwd_pair(const float4& p, const float4& q, float cb, float px, float py, uint32_t m1,
                                         float& T, float& acc0, float& acc1, float& acc2, uint32_t& contrib,
                                         bool& done) {
  float dx, dy, p2, eg, og, nx, ny;
  eval_pair(p, q, px, py, dx, dy, p2, eg, og, nx, ny);
  const float alpha = fminf(kAlphaMax, og);
  const bool ok = !done && (p2 <= 0.0f) && (alpha >= kAlphaMin);
  const float Tn = T * (1.0f - alpha);
  const bool stop = ok && (Tn < kTMin);
  const bool blend = ok && !stop;
  const float w = blend ? alpha * T : 0.0f;
  acc0 = fmaf(q.z, w, acc0);
  acc1 = fmaf(q.w, w, acc1);
  acc2 = fmaf(cb, w, acc2);
  T = blend ? Tn : T;
  contrib = blend ? m1 : contrib;
  done = done || stop;
  return blend;
}

// COUNT = true runs the same decisions on every entry (no culling) but only
// counts, per pixel, the pairs examined (alpha evaluated before the walk ends)
// and the pairs blended, and adds them to counts[0], counts[1].
template <bool COUNT, bool CHS = false>
__global__ __launch_bounds__(256) void k_render_fwd(const uint2* __restrict__ ranges,
                                                    const uint32_t* __restrict__ point_list,
                                                    const float4* __restrict__ rec, DevCam cam,
                                                    float* __restrict__ image, float* __restrict__ final_T,
                                                    uint32_t* __restrict__ n_contrib, float* __restrict__ t_ckpt,
                                                    unsigned long long* __restrict__ counts,
                                                    const int32_t* __restrict__ plan,
                                                    uint32_t* __restrict__ tile_work,
                                                    float* __restrict__ c_ckpt, size_t cplane) {
  __shared__ Stage st;
  __shared__ uint32_t s_work;
  __shared__ typename std::conditional<CHS, ChsStage, char>::type cs;
  const int tile = tile_of_block(plan, blockIdx.x, gridDim.x);
  if (tile < 0) return;
  if constexpr (CHS) chs_clear(cs);
  const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
  int lx, ly;
  tile_pixel(threadIdx.x, lx, ly);
  const int px_i = tx * kTile + lx, py_i = ty * kTile + ly;
  const bool inside = px_i < cam.width && py_i < cam.height;
  const float px = static_cast<float>(px_i) + 0.5f, py = static_cast<float>(py_i) + 0.5f;
  const float x0 = static_cast<float>(tx * kTile), y0 = static_cast<float>(ty * kTile);
  const uint2 rg = ranges[tile];
  const int wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) {
    st.r[kNull].p = make_float4(0.f, 0.f, 0.f, 0.f);
    st.r[kNull].q = make_float4(0.f, 0.f, 0.f, 0.f);
    st.r[kNull].c = make_float2(0.f, 0.f);
    s_work = 0;
  }

  float T = 1.0f, acc0 = 0.0f, acc1 = 0.0f, acc2 = 0.0f;
  uint32_t contrib = 0, n_exam = 0, n_blend = 0;
  bool done = !inside;
  const size_t slot0 = ckpt_slot0(rg.x, tile);
  // colour is summed per batch and the batch sums are added up; for tiles of
  // several batches each batch sum is kept (c_ckpt), so that a backward walk
  // can start at any batch end from the light behind it
  const bool multi = (rg.y - rg.x) > static_cast<uint32_t>(kBatch);

  for (uint32_t base = rg.x, b = 0; base < rg.y; base += kBatch, ++b) {
    if (__syncthreads_count(done) == 256) break;
    if (!COUNT && b > 0 && t_ckpt) t_ckpt[(slot0 + b) * kBatch + threadIdx.x] = T;
    const int cnt = static_cast<int>(min(static_cast<uint32_t>(kBatch), rg.y - base));
    stage_batch(st, rec, point_list, base, cnt, x0, y0);
    __syncthreads();
    ChsSlot sl{0u, false};
    if constexpr (CHS) {
      sl = chs_group<false>(st, cs, rec, cnt, x0, y0);
      __syncthreads();
    }
    build_list(st, cnt, COUNT);
    if constexpr (CHS) {
      __syncthreads();
      chs_release(cs, sl);
    } else {
      wave_lds_sync();   // a wave walks only the list it built
    }
    const uint32_t m0 = base - rg.x + 1u;
    // the wave's list length and row as scalars: the loop control is scalar
    const int wave_u = static_cast<int>(uniform(static_cast<uint32_t>(wave)));
    const int L = static_cast<int>(uniform(static_cast<uint32_t>(st.len[wave_u])));
    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
    for (int i0 = 0; i0 < L; i0 += kUnroll) {
      if (__builtin_amdgcn_ballot_w64(!done) == 0) break;  // whole wave finished: leave the batch
      const uint4 jj = *reinterpret_cast<const uint4*>(&st.list[wave_u][i0]);
      const uint32_t js[kUnroll] = {uniform(jj.x), uniform(jj.y), uniform(jj.z), uniform(jj.w)};
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const uint32_t j = js[u];
        if (COUNT) n_exam += (!done && j != kNull) ? 1u : 0u;
        const bool blend = fwd_pair(st.r[j].p, st.r[j].q, st.r[j].c.x, px, py, m0 + j, T, s0, s1, s2, contrib, done);
        if (COUNT) n_blend += blend ? 1u : 0u;
      }
    }
    if (!COUNT && c_ckpt && multi) {
      const size_t o = (slot0 + b) * kBatch + threadIdx.x;
      c_ckpt[o] = s0;
      c_ckpt[cplane + o] = s1;
      c_ckpt[2 * cplane + o] = s2;
    }
    acc0 += s0;
    acc1 += s1;
    acc2 += s2;
  }
  if (COUNT) {
    __shared__ unsigned long long s_cnt[2];
    __syncthreads();
    if (threadIdx.x == 0) { s_cnt[0] = 0; s_cnt[1] = 0; }
    __syncthreads();
    if (inside) {
      atomicAdd(&s_cnt[0], static_cast<unsigned long long>(n_exam));
      atomicAdd(&s_cnt[1], static_cast<unsigned long long>(n_blend));
    }
    __syncthreads();
    if (threadIdx.x == 0) { atomicAdd(&counts[0], s_cnt[0]); atomicAdd(&counts[1], s_cnt[1]); }
    return;
  }
  if (inside) {
    const int64_t HW = static_cast<int64_t>(cam.width) * cam.height;
    const int64_t pix = static_cast<int64_t>(py_i) * cam.width + px_i;
    image[pix] = fmaf(T, cam.bg[0], acc0);
    image[HW + pix] = fmaf(T, cam.bg[1], acc1);
    image[2 * HW + pix] = fmaf(T, cam.bg[2], acc2);
    final_T[pix] = T;
    n_contrib[pix] = contrib;
  }
  if (tile_work) {
    // the tile's backward work count: the largest n_contrib of its pixels
    uint32_t mx = contrib;
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, static_cast<uint32_t>(__shfl_xor(static_cast<int>(mx), o, 64)));
    if ((threadIdx.x & 63) == 0 && mx) atomicMax(&s_work, mx);
    __syncthreads();
    if (threadIdx.x == 0) tile_work[tile] = s_work;
  }
}


// Forward of light tiles, merged four to a workgroup: one wave per tile, each
// lane four pixels (the same lane position in each 8x8 quadrant).  The
// entries of a pixel's quadrant are visited in list order through the same
// fwd_pair as the one-workgroup-per-tile form, so the outputs are identical.
__global__ __launch_bounds__(256) void k_render_fwd_light(const uint2* __restrict__ ranges,
                                                          const uint32_t* __restrict__ point_list,
                                                          const float4* __restrict__ rec, DevCam cam,
                                                          float* __restrict__ image, float* __restrict__ final_T,
                                                          uint32_t* __restrict__ n_contrib,
                                                          const int32_t* __restrict__ plan,
                                                          uint32_t* __restrict__ tile_work) {
  __shared__ LightStage stage[4];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tile = light_tile(plan, blockIdx.x, wave);
  if (tile < 0) return;
  LightStage& ls = stage[wave];
  const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
  const float x0 = static_cast<float>(tx * kTile), y0 = static_cast<float>(ty * kTile);
  const uint2 rg = ranges[tile];
  const int cnt = static_cast<int>(min(rg.y - rg.x, static_cast<uint32_t>(kLightMax)));
  stage_light(ls, rec, point_list, rg.x, cnt, x0, y0, lane);
  float T[4], a0[4], a1[4], a2[4], px[4], py[4];
  uint32_t con[4];
  bool done[4];
  int pxi[4], pyi[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    pxi[k] = tx * kTile + ((k & 1) << 3) + (lane & 7);
    pyi[k] = ty * kTile + ((k >> 1) << 3) + (lane >> 3);
    px[k] = static_cast<float>(pxi[k]) + 0.5f;
    py[k] = static_cast<float>(pyi[k]) + 0.5f;
    T[k] = 1.0f; a0[k] = a1[k] = a2[k] = 0.0f; con[k] = 0;
    done[k] = !(pxi[k] < cam.width && pyi[k] < cam.height);
  }
  for (int j = 0; j < cnt; ++j) {
    const uint32_t mask = uniform(__float_as_uint(ls.c[j].y));
    if (mask == 0) continue;
    if (__builtin_amdgcn_ballot_w64(!(done[0] && done[1] && done[2] && done[3])) == 0) break;
    const float4 p = ls.p[j];
    const float4 q = ls.q[j];
    const float cb = ls.c[j].x;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if ((mask >> k) & 1u) fwd_pair(p, q, cb, px[k], py[k], static_cast<uint32_t>(j) + 1u, T[k], a0[k], a1[k], a2[k],
                                      con[k], done[k]);
  }
  const int64_t HW = static_cast<int64_t>(cam.width) * cam.height;
  uint32_t mx = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    mx = max(mx, con[k]);
    if (pxi[k] < cam.width && pyi[k] < cam.height) {
      const int64_t pix = static_cast<int64_t>(pyi[k]) * cam.width + pxi[k];
      image[pix] = fmaf(T[k], cam.bg[0], a0[k]);
      image[HW + pix] = fmaf(T[k], cam.bg[1], a1[k]);
      image[2 * HW + pix] = fmaf(T[k], cam.bg[2], a2[k]);
      final_T[pix] = T[k];
      n_contrib[pix] = con[k];
    }
  }
  for (int o = 32; o > 0; o >>= 1) mx = max(mx, static_cast<uint32_t>(__shfl_xor(static_cast<int>(mx), o, 64)));
  if (lane == 0) tile_work[tile] = mx;
}

// Bucket table of the colour-hash sampling mode over every list entry of the
// frame (every 256-entry window, whether or not compositing reaches it), and
// optionally each entry's bucket and representative.  Two stages, as the
// paper describes the aggregation: within the workgroup each window's groups
// are summed at their representative in LDS; then each group adds its count
// and sums to the frame's 4096-bucket table with device atomics.  One
// workgroup per tile, windows in list order.
__global__ __launch_bounds__(256) void k_chs_table(const uint2* __restrict__ ranges,
                                                   const uint32_t* __restrict__ point_list,
                                                   const float4* __restrict__ rec, DevCam cam,
                                                   uint32_t* __restrict__ tab_count, float* __restrict__ tab_sum,
                                                   uint16_t* __restrict__ bucket_out, uint32_t* __restrict__ rep_out) {
  __shared__ Stage st;
  __shared__ ChsStage cs;
  __shared__ float4 s_sum[kBatch];    // colour and opacity sums of a group, at its representative
  __shared__ uint32_t s_n[kBatch];
  const int tile = blockIdx.x;
  const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
  const float x0 = static_cast<float>(tx * kTile), y0 = static_cast<float>(ty * kTile);
  const uint2 rg = ranges[tile];
  const int t = threadIdx.x;
  chs_clear(cs);
  for (uint32_t base = rg.x; base < rg.y; base += kBatch) {
    const int cnt = static_cast<int>(min(static_cast<uint32_t>(kBatch), rg.y - base));
    __syncthreads();
    stage_batch(st, rec, point_list, base, cnt, x0, y0);
    s_sum[t] = make_float4(0.f, 0.f, 0.f, 0.f);
    s_n[t] = 0u;
    __syncthreads();
    const bool valid = t < cnt;
    // the entry's own colour and opacity, before the grouping rewrites the batch
    const float4 own = valid ? make_float4(st.r[t].q.z, st.r[t].q.w, st.r[t].c.x, st.r[t].q.y) : make_float4(0.f, 0.f, 0.f, 0.f);
    const ChsSlot sl = chs_group<true>(st, cs, rec, cnt, x0, y0);
    __syncthreads();
    chs_release(cs, sl);
    const int r = valid && cs.rep[t] != kChsNone ? static_cast<int>(cs.rep[t]) : t;
    if (valid) {
      if (bucket_out) bucket_out[base + t] = static_cast<uint16_t>(sl.bucket);
      if (rep_out) rep_out[base + t] = base + static_cast<uint32_t>(r);
      if (tab_count || tab_sum) {
        // stage 1: the group's sums at its representative (LDS)
        atomicAdd(&s_n[r], 1u);
        atomicAdd(&s_sum[r].x, own.x);
        atomicAdd(&s_sum[r].y, own.y);
        atomicAdd(&s_sum[r].z, own.z);
        atomicAdd(&s_sum[r].w, own.w);
      }
    }
    __syncthreads();
    // stage 2: one set of device atomics per group
    if (valid && r == t && (tab_count || tab_sum)) {
      const uint32_t h = sl.bucket;
      if (tab_count) atomicAdd(&tab_count[h], s_n[t]);
      if (tab_sum) {
        const float4 v = s_sum[t];
        unsafeAtomicAdd(&tab_sum[4 * h], v.x);
        unsafeAtomicAdd(&tab_sum[4 * h + 1], v.y);
        unsafeAtomicAdd(&tab_sum[4 * h + 2], v.z);
        unsafeAtomicAdd(&tab_sum[4 * h + 3], v.w);
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_chs_table_clear(uint32_t* __restrict__ tab_count, float* __restrict__ tab_sum) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= kChsBuckets) return;
  if (tab_count) tab_count[i] = 0u;
  if (tab_sum) reinterpret_cast<float4*>(tab_sum)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

gs_status launch_chs_table(const gs_projected& proj, const uint32_t* point_list, const uint32_t* ranges,
                           const DevCam& cam, uint32_t* tab_count, float* tab_sum, uint16_t* bucket_out,
                           uint32_t* rep_out, hipStream_t s) {
  const int ntiles = cam.tiles_x * cam.tiles_y;
  if (tab_count || tab_sum) {
    { TimedLaunch gs_tl("k_chs_table_clear", s); k_chs_table_clear<<<kChsBuckets / 256, 256, 0, s>>>(tab_count, tab_sum); }
    gs_status st = check_launch("k_chs_table_clear");
    if (st != GS_OK) return st;
  }
  { TimedLaunch gs_tl("k_chs_table", s); k_chs_table<<<ntiles, 256, 0, s>>>(reinterpret_cast<const uint2*>(ranges), point_list,
                                                   reinterpret_cast<const float4*>(proj.records), cam, tab_count,
                                                   tab_sum, bucket_out, rep_out); }
  return check_launch("k_chs_table");
}

gs_status launch_render_fwd(const gs_projected& proj, const uint32_t* point_list, const uint32_t* ranges, int64_t k,
                            const DevCam& cam, float* image, float* final_T, uint32_t* n_contrib, float* t_ckpt,
                            int schedule_flags, hipStream_t s) {
  const int ntiles = cam.tiles_x * cam.tiles_y;
  const bool chs = (schedule_flags & GS_RENDER_COLOUR_HASH) != 0;
  const int schedule = schedule_flags & 0xFF;
  int32_t* plan = nullptr;
  uint32_t* tile_work = nullptr;
  float* c_ckpt = nullptr;
  const size_t cplane = ckpt_core_floats(k, ntiles);
  if (t_ckpt) {
    float* tail = t_ckpt + ckpt_core_floats(k, ntiles);
    plan = reinterpret_cast<int32_t*>(tail);
    tile_work = reinterpret_cast<uint32_t*>(tail + plan_ints(ntiles));
    c_ckpt = tail + plan_ints(ntiles) + ntiles;
    if (schedule == 2) {
      gs_status st = launch_tile_plan(ntiles, ranges, nullptr, kHeavyFactorFwd, kLightMax, plan, s);
      if (st != GS_OK) return st;
      { TimedLaunch gs_tl("k_render_fwd_light", s); k_render_fwd_light<<<static_cast<unsigned>(ceil_div(ntiles, 4)), 256, 0, s>>>(
          reinterpret_cast<const uint2*>(ranges), point_list, reinterpret_cast<const float4*>(proj.records), cam,
          image, final_T, n_contrib, plan, tile_work); }
      st = check_launch("k_render_fwd_light");
      if (st != GS_OK) return st;
    } else {
      plan = nullptr;
    }
  }
  if (chs) {
    TimedLaunch gs_tl("k_render_fwd<false, true>", s);
    k_render_fwd<false, true><<<ntiles, 256, 0, s>>>(reinterpret_cast<const uint2*>(ranges), point_list,
                                                      reinterpret_cast<const float4*>(proj.records), cam, image,
                                                      final_T, n_contrib, t_ckpt, nullptr, plan, tile_work, c_ckpt,
                                                      cplane);
  } else {
    TimedLaunch gs_tl("k_render_fwd<false, false>", s);
    k_render_fwd<false><<<ntiles, 256, 0, s>>>(reinterpret_cast<const uint2*>(ranges), point_list,
                                               reinterpret_cast<const float4*>(proj.records), cam, image, final_T,
                                               n_contrib, t_ckpt, nullptr, plan, tile_work, c_ckpt, cplane);
  }
  return check_launch("k_render_fwd");
}

gs_status launch_render_count(const gs_projected& proj, const uint32_t* point_list, const uint32_t* ranges,
                              const DevCam& cam, unsigned long long* counts, hipStream_t s) {
  const int ntiles = cam.tiles_x * cam.tiles_y;
  gs_status st = check_hip(hipMemsetAsync(counts, 0, 2 * sizeof(unsigned long long), s), "hipMemsetAsync(counts)");
  if (st != GS_OK) return st;
  { TimedLaunch gs_tl("k_render_fwd<true, false>", s); k_render_fwd<true><<<ntiles, 256, 0, s>>>(reinterpret_cast<const uint2*>(ranges), point_list,
                                            reinterpret_cast<const float4*>(proj.records), cam, nullptr, nullptr,
                                            nullptr, nullptr, counts, nullptr, nullptr, nullptr, 0); }
  return check_launch("k_render_count");
}

// ------------------------------------------------------------------ backward

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_src(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}

// Sum over the 64 lanes of a wave with DPP; the total lands in lane 63 (the
// only lane whose result is defined).  After the row sums, the two row
// broadcasts leave the rows outside their masks holding whatever the
// destination register held: lane 63 reads only rows inside the masks
// (row 3 takes lane 47, then lane 31, which took lane 15), so no zeroed
// register is needed for the others.
__device__ __forceinline__ float wave_sum_to_lane63(float v) {
  v += dpp_src<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp_src<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp_src<0x124, 0xF>(v);  // row_ror:4
  v += dpp_src<0x128, 0xF>(v);  // row_ror:8
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x142, 0xA, 0xF, false));  // row_bcast:15 into rows 1, 3
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x143, 0xC, 0xF, false));  // row_bcast:31 into rows 2, 3
  return v;
}

// Swap halves (32 lanes) / odd-even 16-lane rows between two registers and add:
// the transpose-reduce steps that halve the number of registers per level.
__device__ __forceinline__ float add_swap32(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float add_swap16(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Wave sums of eight values with a transpose-reduce: 18 instructions instead
// of 8 x 6 DPP steps.  On return, lane 16 r + 8 h holds the total of value
// kReduceSlot[2 r + h] (every lane of that 8-lane group holds it).
constexpr int kReduceSlot[8] = {0, 4, 2, 6, 1, 5, 3, 7};
__device__ __forceinline__ float wave_sum8(const float v[8], bool lo8) {
  const float a01 = add_swap32(v[0], v[1]);   // lanes <32: v0 half sums, >=32: v1
  const float a23 = add_swap32(v[2], v[3]);
  const float a45 = add_swap32(v[4], v[5]);
  const float a67 = add_swap32(v[6], v[7]);
  const float b0 = add_swap16(a01, a23);      // rows: v0 v2 v1 v3 (quarter sums)
  const float b1 = add_swap16(a45, a67);      // rows: v4 v6 v5 v7
  const float keep = lo8 ? b0 : b1;
  const float send = lo8 ? b1 : b0;
  float c = keep + dpp_src<0x128, 0xF>(send); // row_ror:8 pairs lane i with i^8
  c += dpp_src<0x141, 0xF>(c);                // row_half_mirror within 8 lanes
  c += dpp_src<0xB1, 0xF>(c);                 // quad_perm [1,0,3,2]
  c += dpp_src<0x4E, 0xF>(c);                 // quad_perm [2,3,0,1]
  return c;
}

// Gradient terms of one (pixel, entry) pair of the back-to-front walk, after
// the alpha evaluation: recovers T before the entry, updates the light behind
// (as G.S) and writes the nine per-pair terms (all zero when !ok).
__device__ __forceinline__ void bwd_terms(const float4& q, float cb, bool ok, float nx, float ny, float alpha,
                                          float eg, float og, float G0, float G1, float G2, float& T, float& GS,
                                          float v[9]) {
  // hardware reciprocal (1 ulp): T is re-anchored every 256 entries, so its
  // rounding stays far below the tolerance of the recovered transmittance
  const float inv = __builtin_amdgcn_rcpf(1.0f - alpha);
  const float Tm = ok ? T * inv : T;
  // gradient terms only (alpha itself is not re-derived here): fused
  const float Gc = fmaf(G2, cb, fmaf(G1, q.w, G0 * q.z));
  const float dalpha = fmaf(Tm, Gc, -(inv * GS));
  const float w = ok ? alpha * Tm : 0.0f;
  GS = fmaf(w, Gc, GS);
  T = Tm;
  const bool unclamped = og < kAlphaMax;
  // dL/dpower (natural-log power) and dL/do = e^power dL/dalpha
  const float dpow = (ok && unclamped) ? alpha * dalpha : 0.0f;
  const float dop = (ok && unclamped) ? eg * dalpha : 0.0f;
  // n = (nx, ny) = -log2(e)/2 K d with K the conic and d = (dx, dy).  The
  // pair's conic gradient -1/2 dpow d d^T is carried to Sigma' = K^-1 right
  // here, -K (.) K = 1/2 dpow (K d)(K d)^T, before any summation: converting
  // the summed conic gradient cancels badly for elongated footprints.  The
  // constant factors (powers of ln 2 and 2) are applied once per Gaussian
  // after the sums (kGradScale).
  const float ux = dpow * nx, uy = dpow * ny;
  v[0] = ux;                                 // dL/du            / (2 ln2)
  v[1] = uy;                                 // dL/dv            / (2 ln2)
  v[2] = ux * nx;                            // dL/dSigma'_xx    / (2 ln2^2)
  v[3] = ux * ny;                            // dL/dSigma'_xy    / (4 ln2^2), both entries
  v[4] = uy * ny;                            // dL/dSigma'_yy    / (2 ln2^2)
  v[5] = dop;                                // dL/dopacity
  v[6] = G0 * w;                             // dL/dr
  v[7] = G1 * w;                             // dL/dg
  v[8] = G2 * w;                             // dL/db
}

// g2d[k][i] = acc[i][k]: the [9][n] output from the per-Gaussian rows.
__global__ __launch_bounds__(256) void k_acc_to_g2d(int n, const float4* __restrict__ acc, float* __restrict__ g2d) {
  static_assert(kAccStride % 4 == 0 && kAccStride >= GS_G2D, "rows of whole float4s holding the nine sums");
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float4* row = acc + static_cast<int64_t>(kAccStride / 4) * i;
  const float4 a = row[0];
  const float4 b = row[1];
  const float4 c = row[2];
  const float v[9] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x};
#pragma unroll
  for (int k = 0; k < GS_G2D; ++k) g2d[static_cast<int64_t>(k) * n + i] = v[k] * grad_scale(k);
}

// ------------------------------------------------- deterministic reduction
// Every (tile, Gaussian) entry gets its own row of nine partial sums; the rows
// of one Gaussian are contiguous, in the row-major order of its tile
// rectangle:  row = base_g + (ty - y0) w + (tx - x0), with base the exclusive
// prefix sum of the rectangle areas in Gaussian order (the areas sum to K).
// The backward writes each entry's row once -- a workgroup adds its four
// waves' sums in wave order -- and the reduction adds a Gaussian's rows in
// rectangle order.  No atomics: the result is the same bit for bit on every
// run (for a given schedule).  Rows of entries no pixel reaches stay zero.
constexpr int kDetRow = 9;

__global__ __launch_bounds__(256) void k_det_count(int n, const float4* __restrict__ rec,
                                                   const int* __restrict__ radius, int tiles_x, int tiles_y,
                                                   uint32_t* __restrict__ cnt) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  int x0, x1, y0, y1;
  cnt[i] = static_cast<uint32_t>(tile_rect(rec[3 * static_cast<int64_t>(i)].x, rec[3 * static_cast<int64_t>(i)].y,
                                           radius[i], tiles_x, tiles_y, x0, x1, y0, y1));
}

// row_of[i] = (base_i - (y0 w + x0), w) in wrap-around uint32 arithmetic, so
// that the row of tile (tx, ty) is row_of.x + ty w + tx.
__global__ __launch_bounds__(256) void k_det_rows(int n, const float4* __restrict__ rec,
                                                  const int* __restrict__ radius, int tiles_x, int tiles_y,
                                                  const uint32_t* __restrict__ base, uint2* __restrict__ row_of) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  int x0, x1, y0, y1;
  tile_rect(rec[3 * static_cast<int64_t>(i)].x, rec[3 * static_cast<int64_t>(i)].y, radius[i], tiles_x, tiles_y,
            x0, x1, y0, y1);
  const uint32_t w = static_cast<uint32_t>(max(x1 - x0 + 1, 0));
  row_of[i] = make_uint2(base[i] - (static_cast<uint32_t>(y0) * w + static_cast<uint32_t>(x0)), w);
}

__device__ __forceinline__ uint32_t det_row(uint2 ro, int tx, int ty) {
  return ro.x + static_cast<uint32_t>(ty) * ro.y + static_cast<uint32_t>(tx);
}

__global__ __launch_bounds__(256) void k_zero4(float4* __restrict__ p, int64_t n4) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n4;
       i += static_cast<int64_t>(gridDim.x) * 256)
    p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// g2d[c][i] = sum over the Gaussian's rows, in rectangle order.
__global__ __launch_bounds__(256) void k_det_reduce(int n, const uint32_t* __restrict__ cnt,
                                                    const uint32_t* __restrict__ base,
                                                    const float* __restrict__ part, uint32_t rows,
                                                    float* __restrict__ g2d) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  float s[kDetRow];
#pragma unroll
  for (int c = 0; c < kDetRow; ++c) s[c] = 0.0f;
  const uint32_t b = base[i], e = min(b + cnt[i], rows);
  for (uint32_t r = b; r < e; ++r) {
    const float* row = part + static_cast<size_t>(r) * kDetRow;
#pragma unroll
    for (int c = 0; c < kDetRow; ++c) s[c] += row[c];
  }
#pragma unroll
  for (int c = 0; c < GS_G2D; ++c) g2d[static_cast<int64_t>(c) * n + i] = s[c] * grad_scale(c);
}

// Per (pixel, entry) derivative, walked back to front.  Starting from the light
// S = T_f bg behind the last entry, each blended entry m (going backwards)
// recovers T_m = T_{m+1} / (1 - alpha_m) and uses the light behind it,
// S_m = sum_{j>m} c_j alpha_j T_j + T_f bg:
//   dL/dalpha_m = sum_k G_k (c_k T_m - S_mk / (1 - alpha_m)),  S += c_m alpha_m T_m.
// Only G.S enters, so the walk carries the scalar GS = G.S.  Accumulating it
// (instead of subtracting from the pixel value) keeps its rounding error
// relative to itself.  T restarts at every batch end from the forward's
// checkpoint (or T_f for the last batch), so the division walks at most 256
// entries and its rounding cannot build up along long lists.  Skips are
// re-derived from the same alpha evaluation as the forward; entries past
// n_contrib are never touched; a wave visits only the entries whose
// alpha-support box meets its quadrant.  The nine per-pair gradients are summed
// over the wave and added by nine lanes at once to the Gaussian's row of the
// accumulator acc[n][kAccStride]: a 48-byte row per Gaussian, so the nine
// atomics of an instruction meet in one or two L2 lines (the [9][n] output
// is written from it afterwards).  DET: the sums go to the entry's row of `part` instead
// (deterministic reduction above).
template <bool DET, bool CHS = false>
__global__ __launch_bounds__(256) void k_render_bwd(const uint2* __restrict__ ranges,
                                                    const uint32_t* __restrict__ point_list,
                                                    const float4* __restrict__ rec, DevCam cam,
                                                    const float* __restrict__ final_T,
                                                    const uint32_t* __restrict__ n_contrib,
                                                    const float* __restrict__ t_ckpt,
                                                    const float* __restrict__ dL_dimage, int n,
                                                    float* __restrict__ acc, const int32_t* __restrict__ plan,
                                                    const int32_t* __restrict__ items,
                                                    const uint32_t* __restrict__ tile_work,
                                                    const float* __restrict__ c_ckpt, size_t cplane,
                                                    float* __restrict__ part, const uint2* __restrict__ row_of,
                                                    uint32_t rows) {
  __shared__ Stage st;
  __shared__ uint32_t s_max;
  // DET: each wave's nine sums per staged entry, [wave][entry][9]
  __shared__ float4 s_part4[DET ? 4 * kBatch * kDetRow / 4 : 1];
  float* const s_part = reinterpret_cast<float*>(s_part4);
  // CHS: the grouping, and per staged entry the sums of the gradient reaching
  // its group's aggregated opacity and colour (representatives only)
  __shared__ typename std::conditional<CHS, ChsStage, char>::type cs;
  __shared__ float4 s_chs4[CHS ? kBatch : 1];
  float* const s_chs = reinterpret_cast<float*>(s_chs4);
  // items: this workgroup walks one batch of one tile (the batch plan);
  // otherwise the whole tile (plain map, or the plan's order)
  int tile, b_only = -1;
  if (items) {
    const int nitems = items[0];
    if (static_cast<int>(blockIdx.x) >= nitems) return;
    const int it = xcd_remap(blockIdx.x, nitems);
    tile = items[kPlanHeader + 2 * it];
    b_only = items[kPlanHeader + 2 * it + 1];
  } else {
    tile = tile_of_block(plan, blockIdx.x, gridDim.x);
    if (tile < 0) return;
  }
  if constexpr (CHS) chs_clear(cs);
  const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
  int lx, ly;
  tile_pixel(threadIdx.x, lx, ly);
  const int px_i = tx * kTile + lx, py_i = ty * kTile + ly;
  const bool inside = px_i < cam.width && py_i < cam.height;
  const float px = static_cast<float>(px_i) + 0.5f, py = static_cast<float>(py_i) + 0.5f;
  const float x0 = static_cast<float>(tx * kTile), y0 = static_cast<float>(ty * kTile);
  const uint2 rg = ranges[tile];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const bool lo8 = (lane & 8) == 0;
  const int out_slot = (lane == 63) ? 8 : kReduceSlot[((lane >> 4) << 1) | ((lane >> 3) & 1)];
  const bool writer = ((lane & 7) == 0) || lane == 63;

  float G0 = 0.f, G1 = 0.f, G2 = 0.f, T = 1.0f;
  uint32_t ncon = 0;
  if (inside) {
    const int64_t HW = static_cast<int64_t>(cam.width) * cam.height;
    const int64_t pix = static_cast<int64_t>(py_i) * cam.width + px_i;
    G0 = dL_dimage[pix]; G1 = dL_dimage[HW + pix]; G2 = dL_dimage[2 * HW + pix];
    T = final_T[pix];
    ncon = n_contrib[pix];
  }
  const float T_final = T;
  const size_t slot0 = ckpt_slot0(rg.x, tile);
  float GS = T * (G0 * cam.bg[0] + G1 * cam.bg[1] + G2 * cam.bg[2]);
  uint32_t smax;
  if (tile_work) {
    smax = tile_work[tile];  // the largest n_contrib of the tile, from the forward
  } else {
    if (threadIdx.x == 0) s_max = 0;
    __syncthreads();
    if (ncon) atomicMax(&s_max, ncon);
    __syncthreads();
    smax = s_max;
  }
  const uint32_t len = min(rg.y - rg.x, smax);  // n_contrib never exceeds the list
  const int nbatch = static_cast<int>((len + kBatch - 1) / kBatch);
  int b_hi = nbatch - 1, b_lo = 0;
  if (b_only >= 0) {
    b_hi = b_lo = b_only;
    // light behind the end of this batch: the forward's colour sums of the
    // pixel's later batches (each a sum of non-negative terms), dotted with G
    const int last = ncon ? static_cast<int>((ncon - 1) / kBatch) : -1;
    for (int bb = b_only + 1; bb <= last; ++bb) {
      const size_t o = (slot0 + bb) * kBatch + threadIdx.x;
      GS += G0 * c_ckpt[o] + G1 * c_ckpt[cplane + o] + G2 * c_ckpt[2 * cplane + o];
    }
  }

  for (int bi = b_hi; bi >= b_lo; --bi) {
    const uint32_t m0 = static_cast<uint32_t>(bi) * kBatch;
    const int cnt = static_cast<int>(min(static_cast<uint32_t>(kBatch), len - m0));
    T = (bi + 1 < nbatch) ? t_ckpt[(slot0 + bi + 1) * kBatch + threadIdx.x] : T_final;
    // CHS groups the whole 256-entry window, walked or not, as the forward did
    const int cnt_all = CHS ? static_cast<int>(min(static_cast<uint32_t>(kBatch), rg.y - rg.x - m0)) : cnt;
    __syncthreads();
    stage_batch(st, rec, point_list, rg.x + m0, cnt_all, x0, y0);
    if constexpr (DET) {
      for (int i = threadIdx.x; i < 4 * kBatch * kDetRow / 4; i += 256) s_part4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    if constexpr (CHS) s_chs4[threadIdx.x] = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    ChsSlot sl{0u, false};
    if constexpr (CHS) {
      sl = chs_group<true>(st, cs, rec, cnt_all, x0, y0);
      __syncthreads();
    }
    build_list(st, cnt, false);
    if constexpr (CHS) {
      __syncthreads();
      chs_release(cs, sl);
    } else {
      wave_lds_sync();   // a wave walks only the list it built
    }
    // the wave's list length and row as scalars: the loop control is scalar
    const int wave_u = static_cast<int>(uniform(static_cast<uint32_t>(wave)));
    // entry m0 + j reaches this pixel iff j < ncon - m0 (one compare per entry)
    const uint32_t nrel = ncon > m0 ? ncon - m0 : 0u;
    for (int i = static_cast<int>(uniform(static_cast<uint32_t>(st.len[wave_u]))) - 1; i >= 0; --i) {
      const uint32_t j = uniform(st.list[wave_u][i]);
      if (j == kNull) continue;
      const bool live = j < nrel;
      const uint64_t reach = __builtin_amdgcn_ballot_w64(live);
      if (reach == 0) continue;  // no lane of this wave reaches entry m yet
      const float4 p = st.r[j].p;
      const float4 q = st.r[j].q;
      const float cb = st.r[j].c.x;
      float dx, dy, p2, eg, og, nx, ny;
      eval_pair(p, q, px, py, dx, dy, p2, eg, og, nx, ny);
      const float alpha = fminf(kAlphaMax, og);
      const bool ok = live && (p2 <= 0.0f) && (alpha >= kAlphaMin);
      // the wave's test from the compares' own masks (a ballot of the
      // combined bool would first turn it into an integer and back)
      if ((reach & __builtin_amdgcn_ballot_w64(p2 <= 0.0f) & __builtin_amdgcn_ballot_w64(alpha >= kAlphaMin)) == 0)
        continue;
      float v[9];
      bwd_terms(q, cb, ok, nx, ny, alpha, eg, og, G0, G1, G2, T, GS, v);
      const float red8 = wave_sum8(v, lo8);
      const float red9 = wave_sum_to_lane63(v[8]);  // dL/db
      if constexpr (DET) {
        if (writer) s_part[(wave * kBatch + static_cast<int>(j)) * kDetRow + out_slot] = lane == 63 ? red9 : red8;
      } else {
        // CHS: a group's opacity and colour sums wait in LDS for the member pass below
        bool to_lds = false;
        if constexpr (CHS) to_lds = out_slot >= 5 && cs.rep[j] != kChsNone;
        // the Gaussian's row in scalar registers: the atomics take it as
        // their base and the lane's slot as a 32-bit offset
        float* const row = acc + static_cast<int64_t>(uniform(st.r[j].gid)) * kAccStride;
        if (writer) {
          if (to_lds)
            atomicAdd(&s_chs[4 * static_cast<int>(j) + out_slot - 5], lane == 63 ? red9 : red8);
          else
            unsafeAtomicAdd(row + out_slot, lane == 63 ? red9 : red8);
        }
      }
    }
    if constexpr (CHS) {
      // every member of a group of two or more (representative included) gets
      // its share of the gradient of the group's opacity and colour
      __syncthreads();
      const int t = threadIdx.x;
      if (t < cnt_all) {
        const uint32_t r = cs.rep[t];
        if (r != kChsNone) {
          const float4 tot = s_chs4[r];
          if (tot.x != 0.0f || tot.y != 0.0f || tot.z != 0.0f || tot.w != 0.0f) {
            float* const row = acc + static_cast<int64_t>(st.r[t].gid) * kAccStride;
            const float so = cs.share_o[t], sn = cs.inv_n[t];
            unsafeAtomicAdd(row + 5, tot.x * so);
            unsafeAtomicAdd(row + 6, tot.y * sn);
            unsafeAtomicAdd(row + 7, tot.z * sn);
            unsafeAtomicAdd(row + 8, tot.w * sn);
          }
        }
      }
    }
    if constexpr (DET) {
      // entry t's row: its four waves' sums added in wave order
      __syncthreads();
      const int t = threadIdx.x;
      if (t < cnt) {
        const uint32_t r = det_row(row_of[st.r[t].gid], tx, ty);
        if (r < rows) {
          float* const dst = part + static_cast<size_t>(r) * kDetRow;
#pragma unroll
          for (int c = 0; c < kDetRow; ++c)
            dst[c] = ((s_part[t * kDetRow + c] + s_part[(kBatch + t) * kDetRow + c]) +
                      s_part[(2 * kBatch + t) * kDetRow + c]) + s_part[(3 * kBatch + t) * kDetRow + c];
        }
      }
    }
  }
}


// Backward of light tiles (the largest n_contrib at most kLightMax): one wave
// per tile, four pixels per lane as in the forward.  Each lane adds its four
// pixels' terms before the wave sum, so one reduction and one set of atomics
// serve 256 pixels.  DET: the wave's sums are the entry's whole row.
template <bool DET>
__global__ __launch_bounds__(256) void k_render_bwd_light(const uint2* __restrict__ ranges,
                                                          const uint32_t* __restrict__ point_list,
                                                          const float4* __restrict__ rec, DevCam cam,
                                                          const float* __restrict__ final_T,
                                                          const uint32_t* __restrict__ n_contrib,
                                                          const float* __restrict__ dL_dimage, int n,
                                                          float* __restrict__ acc, const int32_t* __restrict__ plan,
                                                          float* __restrict__ part,
                                                          const uint2* __restrict__ row_of, uint32_t rows) {
  __shared__ LightStage stage[4];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tile = light_tile(plan, blockIdx.x, wave);
  if (tile < 0) return;
  LightStage& ls = stage[wave];
  const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
  const float x0 = static_cast<float>(tx * kTile), y0 = static_cast<float>(ty * kTile);
  const uint2 rg = ranges[tile];
  const bool lo8 = (lane & 8) == 0;
  const int out_slot = (lane == 63) ? 8 : kReduceSlot[((lane >> 4) << 1) | ((lane >> 3) & 1)];
  const bool writer = ((lane & 7) == 0) || lane == 63;
  float* const g_out = acc + out_slot;
  const int64_t HW = static_cast<int64_t>(cam.width) * cam.height;
  float G0[4], G1[4], G2[4], T[4], GS[4], px[4], py[4];
  uint32_t ncon[4];
  uint32_t mx = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int xi = tx * kTile + ((k & 1) << 3) + (lane & 7);
    const int yi = ty * kTile + ((k >> 1) << 3) + (lane >> 3);
    px[k] = static_cast<float>(xi) + 0.5f;
    py[k] = static_cast<float>(yi) + 0.5f;
    G0[k] = G1[k] = G2[k] = 0.0f; T[k] = 1.0f; ncon[k] = 0;
    if (xi < cam.width && yi < cam.height) {
      const int64_t pix = static_cast<int64_t>(yi) * cam.width + xi;
      G0[k] = dL_dimage[pix]; G1[k] = dL_dimage[HW + pix]; G2[k] = dL_dimage[2 * HW + pix];
      T[k] = final_T[pix];
      ncon[k] = n_contrib[pix];
    }
    GS[k] = T[k] * (G0[k] * cam.bg[0] + G1[k] * cam.bg[1] + G2[k] * cam.bg[2]);
    mx = max(mx, ncon[k]);
  }
  for (int o = 32; o > 0; o >>= 1) mx = max(mx, static_cast<uint32_t>(__shfl_xor(static_cast<int>(mx), o, 64)));
  const int len = static_cast<int>(min(min(rg.y - rg.x, mx), static_cast<uint32_t>(kLightMax)));
  stage_light(ls, rec, point_list, rg.x, len, x0, y0, lane);
  for (int j = len - 1; j >= 0; --j) {
    const uint32_t mask = uniform(__float_as_uint(ls.c[j].y));
    if (mask == 0) continue;
    const uint32_t m = static_cast<uint32_t>(j);
    const float4 p = ls.p[j];
    const float4 q = ls.q[j];
    const float cb = ls.c[j].x;
    float vs[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) vs[t] = 0.0f;
    bool any = false;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (!((mask >> k) & 1u)) continue;
      float dx, dy, p2, eg, og, nx, ny;
      eval_pair(p, q, px[k], py[k], dx, dy, p2, eg, og, nx, ny);
      const float alpha = fminf(kAlphaMax, og);
      const bool ok = (m < ncon[k]) && (p2 <= 0.0f) && (alpha >= kAlphaMin);
      float v[9];
      bwd_terms(q, cb, ok, nx, ny, alpha, eg, og, G0[k], G1[k], G2[k], T[k], GS[k], v);
#pragma unroll
      for (int t = 0; t < 9; ++t) vs[t] += v[t];
      any = any || ok;
    }
    if (__builtin_amdgcn_ballot_w64(any) == 0) continue;
    const float red8 = wave_sum8(vs, lo8);
    const float red9 = wave_sum_to_lane63(vs[8]);
    if constexpr (DET) {
      const uint32_t r = det_row(row_of[ls.gid[j]], tx, ty);
      if (writer && r < rows) part[static_cast<size_t>(r) * kDetRow + out_slot] = lane == 63 ? red9 : red8;
    } else {
      if (writer) unsafeAtomicAdd(&g_out[static_cast<int64_t>(ls.gid[j]) * kAccStride], lane == 63 ? red9 : red8);
    }
  }
}

// Workspace: 256 reserved bytes, the light-tile list (plan layout), the batch
// items, then the accumulator rows (256-byte aligned).
static size_t bwd_items_offset(int ntiles) { return (256 + sizeof(int32_t) * plan_ints(ntiles) + 15) / 16 * 16; }
static size_t bwd_acc_offset(int64_t k, int ntiles) {
  return (bwd_items_offset(ntiles) + sizeof(int32_t) * batch_item_ints(k, ntiles) + 255) / 256 * 256;
}

// Deterministic mode, after the items: per-Gaussian counts, bases and row
// maps, the scan's block sums, and the rows (9 floats per entry).
struct DetWs {
  uint32_t* cnt;
  uint32_t* base;
  uint2* row_of;
  uint32_t* sums;
  float* part;
  size_t part_floats;
};

static DetWs carve_det(void* det, int64_t n, int64_t k, size_t* used) {
  Carver c(det);
  DetWs d;
  d.cnt = c.take<uint32_t>(static_cast<size_t>(n));
  d.base = c.take<uint32_t>(static_cast<size_t>(n));
  d.row_of = c.take<uint2>(static_cast<size_t>(n));
  d.sums = c.take<uint32_t>(scan_sums_words(n));
  d.part_floats = (static_cast<size_t>(k) * kDetRow + 3) / 4 * 4;
  d.part = c.take<float>(d.part_floats);
  if (used) *used = c.off;
  return d;
}

size_t render_bwd_workspace(int64_t n, int64_t k, int ntiles, int deterministic) {
  if (deterministic) {
    size_t used = 0;
    carve_det(nullptr, n, k, &used);
    return bwd_acc_offset(k, ntiles) + used;
  }
  return bwd_acc_offset(k, ntiles) + sizeof(float) * kAccStride * static_cast<size_t>(n);
}

gs_status launch_render_bwd(int64_t n, const gs_projected& proj, const uint32_t* point_list, const uint32_t* ranges,
                            int64_t k, const DevCam& cam, const float* final_T,
                            const uint32_t* n_contrib, const float* t_ckpt, const float* dL_dimage, float* g2d, void* ws,
                            size_t ws_bytes, int deterministic, int schedule_flags, const float** rows_out, hipStream_t s) {
  (void)ws_bytes;
  const bool chs = (schedule_flags & GS_RENDER_COLOUR_HASH) != 0;
  const int schedule = schedule_flags & 0xFF;
  if (chs && (deterministic || schedule == GS_SCHEDULE_MERGED))
    return fail(GS_ERR_UNSUPPORTED, "render backward: colour-hash sampling needs atomic mode and PLAIN or BALANCED");
  if (!g2d && (deterministic || !rows_out)) return fail(GS_ERR_INVALID_ARG, "render backward: no output");
  const int ntiles = cam.tiles_x * cam.tiles_y;
  char* w = static_cast<char*>(ws);
  float* acc = reinterpret_cast<float*>(w + bwd_acc_offset(k, ntiles));
  const uint2* rg = reinterpret_cast<const uint2*>(ranges);
  const float4* rec = reinterpret_cast<const float4*>(proj.records);
  const unsigned gn = static_cast<unsigned>(ceil_div(n, 256));
  gs_status st;
  DetWs det{};
  const uint32_t rows = static_cast<uint32_t>(k);
  if (deterministic) {
    det = carve_det(acc, n, k, nullptr);
    acc = nullptr;
    { TimedLaunch gs_tl("k_det_count", s); k_det_count<<<gn, 256, 0, s>>>(static_cast<int>(n), rec, proj.radius, cam.tiles_x, cam.tiles_y, det.cnt); }
    if ((st = check_launch("k_det_count")) != GS_OK) return st;
    if ((st = launch_exclusive_scan(det.cnt, det.base, n, det.sums, nullptr, s)) != GS_OK) return st;
    { TimedLaunch gs_tl("k_det_rows", s); k_det_rows<<<gn, 256, 0, s>>>(static_cast<int>(n), rec, proj.radius, cam.tiles_x, cam.tiles_y, det.base,
                                  det.row_of); }
    if ((st = check_launch("k_det_rows")) != GS_OK) return st;
    if (det.part_floats) {
      const int64_t n4 = static_cast<int64_t>(det.part_floats / 4);
      { TimedLaunch gs_tl("k_zero4", s); k_zero4<<<static_cast<unsigned>(std::min<int64_t>(ceil_div(n4, 256), 8192)), 256, 0, s>>>(
          reinterpret_cast<float4*>(det.part), n4); }
      if ((st = check_launch("k_zero4")) != GS_OK) return st;
    }
  } else if (schedule == 0) {
    // a fill kernel rather than a memset node, so that the call can be captured
    // in a graph (the other schedules clear the rows under the batch plan)
    const int64_t n4 = static_cast<int64_t>(kAccStride / 4) * n;
    { TimedLaunch gs_tl("k_zero4", s); k_zero4<<<static_cast<unsigned>(std::min<int64_t>(ceil_div(n4, 256), 8192)), 256, 0, s>>>(
        reinterpret_cast<float4*>(acc), n4); }
    if ((st = check_launch("k_zero4")) != GS_OK) return st;
  }
  auto bwd = [&](unsigned grid, const int32_t* items, const uint32_t* tile_work, const float* c_ckpt,
                 size_t cplane) {
    if (deterministic)
      { TimedLaunch gs_tl("k_render_bwd<true, false>", s); k_render_bwd<true><<<grid, 256, 0, s>>>(rg, point_list, rec, cam, final_T, n_contrib, t_ckpt, dL_dimage,
                                              static_cast<int>(n), acc, nullptr, items, tile_work, c_ckpt, cplane,
                                              det.part, det.row_of, rows); }
    else if (chs)
      { TimedLaunch gs_tl("k_render_bwd<false, true>", s); k_render_bwd<false, true><<<grid, 256, 0, s>>>(rg, point_list, rec, cam, final_T, n_contrib, t_ckpt, dL_dimage,
                                                     static_cast<int>(n), acc, nullptr, items, tile_work, c_ckpt, cplane,
                                                     nullptr, nullptr, 0); }
    else
      { TimedLaunch gs_tl("k_render_bwd<false, false>", s); k_render_bwd<false><<<grid, 256, 0, s>>>(rg, point_list, rec, cam, final_T, n_contrib, t_ckpt, dL_dimage,
                                               static_cast<int>(n), acc, nullptr, items, tile_work, c_ckpt, cplane,
                                               nullptr, nullptr, 0); }
    return check_launch("k_render_bwd");
  };
  if (schedule == 0) {
    st = bwd(static_cast<unsigned>(ntiles), nullptr, nullptr, nullptr, 0);
  } else {
    // one workgroup per (tile, batch) walked, from the forward's work counts;
    // MERGED hands tiles with at most kLightMax entries to the merged kernel
    const float* tail = t_ckpt + ckpt_core_floats(k, ntiles);
    const uint32_t* tile_work = reinterpret_cast<const uint32_t*>(tail + plan_ints(ntiles));
    const float* c_ckpt = tail + plan_ints(ntiles) + ntiles;
    int32_t* light = schedule == 2 ? reinterpret_cast<int32_t*>(w + 256) : nullptr;
    int32_t* items = reinterpret_cast<int32_t*>(w + bwd_items_offset(ntiles));
    st = launch_batch_plan(ntiles, ranges, tile_work, schedule == 2 ? kLightMax : 0, items, light,
                           deterministic ? nullptr : reinterpret_cast<float4*>(acc),
                           deterministic ? 0 : static_cast<int64_t>(kAccStride / 4) * n, s);
    if (st != GS_OK) return st;
    if (light) {
      const unsigned lg = static_cast<unsigned>(ceil_div(ntiles, 4));
      if (deterministic)
        { TimedLaunch gs_tl("k_render_bwd_light<true>", s); k_render_bwd_light<true><<<lg, 256, 0, s>>>(rg, point_list, rec, cam, final_T, n_contrib, dL_dimage,
                                                    static_cast<int>(n), acc, light, det.part, det.row_of, rows); }
      else
        { TimedLaunch gs_tl("k_render_bwd_light<false>", s); k_render_bwd_light<false><<<lg, 256, 0, s>>>(rg, point_list, rec, cam, final_T, n_contrib, dL_dimage,
                                                     static_cast<int>(n), acc, light, nullptr, nullptr, 0); }
      st = check_launch("k_render_bwd_light");
      if (st != GS_OK) return st;
    }
    st = bwd(static_cast<unsigned>(k / kBatch + ntiles + 1), items, tile_work, c_ckpt, ckpt_core_floats(k, ntiles));
  }
  if (st != GS_OK) return st;
  if (deterministic) {
    { TimedLaunch gs_tl("k_det_reduce", s); k_det_reduce<<<gn, 256, 0, s>>>(static_cast<int>(n), det.cnt, det.base, det.part, rows, g2d); }
    return check_launch("k_det_reduce");
  }
  if (!g2d) {
    *rows_out = acc;
    return GS_OK;
  }
  { TimedLaunch gs_tl("k_acc_to_g2d", s); k_acc_to_g2d<<<gn, 256, 0, s>>>(static_cast<int>(n), reinterpret_cast<const float4*>(acc), g2d); }
  return check_launch("k_acc_to_g2d");
}

}  // namespace gs
