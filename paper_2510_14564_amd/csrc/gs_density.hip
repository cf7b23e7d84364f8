// Workload-sensitive density control (Sec. III-C): each point's local density
// (other points within a radius r), the statistical thresholds mu -/+ sigma of
// the densities, the mean distance to the k nearest points, one round of
// densification next to sparse points (Gaussian spread a d_bar plus a uniform
// perturbation, from noise the caller draws) and the merging of mutual
// nearest dense pairs within mu_d + gamma sigma_d.
//
// The neighbour searches run on a uniform grid of cells of side h = 1.07 r,
// hashed into a power-of-two table and counting-sorted by bucket (one pass of
// atomics, then the library's exclusive scan).  A point's cell is
// floor(x / h) per axis in FP32; with every coordinate below 2^18 h in
// magnitude the FP32 cell coordinates of two points differ from their exact
// value by less than 1/16 of a cell, so a point within r of another lies in
// the same or an adjacent cell (27 cells cover the radius search), and after
// the cells up to Chebyshev offset R have been scanned every point closer
// than (R - 1/16) h has been seen (the k-nearest search stops on that
// guarantee).  One thread per query scans rings 0-2; a query whose k-th
// nearest lies farther (isolated points, a few per cent) goes on to a wave
// of its own that scans rings 0-7 with the 64 lanes sharing each ring's cells,
// and the few left after that to a whole workgroup that scans every point;
// partial top-k lists are merged in LDS.
// Several cells can share a bucket; a scan visits only the points whose own
// cell is the one it wants, so nothing is counted twice.
//
// Every decision is taken exactly as the definition states it in the
// precision it names: FP32 squared distances (each operation rounded, no
// fused multiply-add), thresholds in FP64 from exact integer sums with
// correctly rounded operations, nearest points by (FP32 squared distance,
// index).  This file is compiled without contraction of products into fused
// multiply-adds; sqrt and division are IEEE-rounded (HIP's default for FP32
// square roots and quotients in source), so the square-root sums are the
// definition's too.  The densities, classes, neighbour lists and the merge pairing are
// therefore the definition's bit for bit; the new and merged parameters are
// FP32 evaluations of their formulas.
#include "gs_internal.h"

namespace gs {

constexpr int kDcRingsThread = 3;    // rings a thread scans alone (0-2)
constexpr int kDcRingsWave = 8;      // rings a wave scans for a query (0-7) before every point is scanned
constexpr float kDcCellScale = 1.07f;

struct DcPoint {   // a point in bucket order: position and its own cell
  float4 p;        // x, y, z, index (bits)
  int4 c;          // cell x, y, z, unused
};

__device__ __forceinline__ uint32_t dc_hash(int cx, int cy, int cz, uint32_t mask) {
  uint32_t h = static_cast<uint32_t>(cx) * 73856093u ^ static_cast<uint32_t>(cy) * 19349663u ^
               static_cast<uint32_t>(cz) * 83492791u;
  h ^= h >> 15;
  h *= 0x2c1b3c6du;
  h ^= h >> 12;
  return h & mask;
}

__device__ __forceinline__ int dc_cell(float x, float inv_h) { return static_cast<int>(floorf(__fmul_rn(x, inv_h))); }

// FP32 squared distance from the query q to point p, rounded step by step.
__device__ __forceinline__ float dc_d2(const float4& q, const float4& p) {
  const float dx = __fsub_rn(q.x, p.x), dy = __fsub_rn(q.y, p.y), dz = __fsub_rn(q.z, p.z);
  float s = __fmul_rn(dx, dx);
  s = __fadd_rn(s, __fmul_rn(dy, dy));
  return __fadd_rn(s, __fmul_rn(dz, dz));
}

// The far search splits each remaining query's scan over every point into S
// ranges, one workgroup each, while count * S fits kFarSlots partial lists
// (S = min(64, kFarSlots / count)); beyond that, one workgroup per query
// scans all points and writes the result itself.
constexpr uint32_t kFarSlots = 16384;
constexpr uint32_t kFarSplitMax = 64;
__host__ __device__ __forceinline__ uint32_t far_splits(uint32_t count) {
  return count == 0 || count > kFarSlots ? 1u : (kFarSlots / count < kFarSplitMax ? kFarSlots / count : kFarSplitMax);
}

struct DcWs {
  uint32_t* count;      // [T] points per bucket, then their exclusive prefix (bucket starts)
  uint32_t* fill;       // [T]
  uint32_t* sums;       // scan block sums
  DcPoint* pts;         // [n] in bucket order
  int4* cell;           // [n] each point's cell and bucket
  int32_t* rho;         // [n]
  int32_t* nn;          // [n] nearest other point
  float* dnn;           // [n] its distance
  float* dbar;          // [n] mean distance to the k nearest
  uint32_t* keep;       // [n] 1 if the point survives, then its exclusive prefix
  uint32_t* low;        // [n] 1 if the point spawns a new one, then its exclusive prefix
  int32_t* partner;     // [n] merge partner or -1
  unsigned long long* isum;  // [2] sum rho, sum rho^2
  double* dsum;         // [2] sum dnn, sum dnn^2 (FP64 atomics)
  double* stat;         // [8] mu, sigma, rho_low, rho_high, mu_d, sigma_d, d_merge, unused
  unsigned long long* total;  // [2] kept, low counts (from the scans)
  uint32_t* range;      // [1] set if a coordinate is out of the cells' range
  uint32_t* far;        // [n] queries the thread kernel left, [1] their count (far_n)
  uint32_t* far_n;
  uint32_t* far2;       // [n] queries the wave kernel left, [1] their count
  uint32_t* far2_n;
  float* cand_d;        // [kFarSlots][8] partial k-nearest lists of the split far search
  int32_t* cand_i;
  size_t bytes;
};

static uint32_t dc_table(int64_t n) {
  uint32_t t = 1024;
  while (static_cast<int64_t>(t) < 2 * n && t < (1u << 30)) t <<= 1;
  return t;
}

static DcWs carve_dc(void* base, int64_t n) {
  Carver c(base);
  DcWs w;
  const uint32_t T = dc_table(n);
  const size_t nn = static_cast<size_t>(std::max<int64_t>(n, 1));
  w.count = c.take<uint32_t>(T);
  w.fill = c.take<uint32_t>(T);
  w.sums = c.take<uint32_t>(std::max(scan_sums_words(T), scan_sums_words(n)));
  w.pts = c.take<DcPoint>(nn);
  w.cell = c.take<int4>(nn);
  w.rho = c.take<int32_t>(nn);
  w.nn = c.take<int32_t>(nn);
  w.dnn = c.take<float>(nn);
  w.dbar = c.take<float>(nn);
  w.keep = c.take<uint32_t>(nn);
  w.low = c.take<uint32_t>(nn);
  w.partner = c.take<int32_t>(nn);
  w.isum = c.take<unsigned long long>(2);
  w.dsum = c.take<double>(2);
  w.stat = c.take<double>(8);
  w.total = c.take<unsigned long long>(2);
  w.range = c.take<uint32_t>(1);
  w.far = c.take<uint32_t>(nn);
  w.far_n = c.take<uint32_t>(1);
  w.far2 = c.take<uint32_t>(nn);
  w.far2_n = c.take<uint32_t>(1);
  w.cand_d = c.take<float>(static_cast<size_t>(kFarSlots) * 8);
  w.cand_i = c.take<int32_t>(static_cast<size_t>(kFarSlots) * 8);
  w.bytes = c.off;
  return w;
}

size_t density_workspace(int64_t n) { return carve_dc(nullptr, n).bytes; }

__global__ __launch_bounds__(256) void k_dc_clear(uint32_t* __restrict__ a, uint32_t* __restrict__ b, uint32_t T,
                                                  unsigned long long* __restrict__ isum, double* __restrict__ dsum,
                                                  unsigned long long* __restrict__ total, uint32_t* __restrict__ range,
                                                  uint32_t* __restrict__ far_n, uint32_t* __restrict__ far2_n) {
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i < T) { a[i] = 0u; b[i] = 0u; }
  if (i == 0) {
    isum[0] = 0ull; isum[1] = 0ull; dsum[0] = 0.0; dsum[1] = 0.0;
    total[0] = 0ull; total[1] = 0ull; range[0] = 0u; far_n[0] = 0u; far2_n[0] = 0u;
  }
}

// Each point's cell and bucket, and the bucket counts.  A coordinate of 2^18
// cells or more (or not finite) sets *range: the cell guarantees above need
// |x| < 2^18 h.
__global__ __launch_bounds__(256) void k_dc_cells(int n, const float* __restrict__ means, float inv_h, uint32_t mask,
                                                  int4* __restrict__ cell, uint32_t* __restrict__ count,
                                                  uint32_t* __restrict__ range) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float x = means[i], y = means[static_cast<int64_t>(n) + i], z = means[2 * static_cast<int64_t>(n) + i];
  const float lim = 262144.0f;
  if (!(fabsf(__fmul_rn(x, inv_h)) < lim && fabsf(__fmul_rn(y, inv_h)) < lim && fabsf(__fmul_rn(z, inv_h)) < lim)) {
    atomicOr(range, 1u);
    cell[i] = make_int4(0, 0, 0, 0);
    atomicAdd(&count[0], 1u);
    return;
  }
  const int cx = dc_cell(x, inv_h), cy = dc_cell(y, inv_h), cz = dc_cell(z, inv_h);
  const uint32_t b = dc_hash(cx, cy, cz, mask);
  cell[i] = make_int4(cx, cy, cz, static_cast<int>(b));
  atomicAdd(&count[b], 1u);
}

__global__ __launch_bounds__(256) void k_dc_scatter(int n, const float* __restrict__ means,
                                                    const int4* __restrict__ cell, const uint32_t* __restrict__ start,
                                                    uint32_t* __restrict__ fill, DcPoint* __restrict__ pts) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int4 c = cell[i];
  const uint32_t b = static_cast<uint32_t>(c.w);
  const uint32_t pos = start[b] + atomicAdd(&fill[b], 1u);
  DcPoint d;
  d.p = make_float4(means[i], means[static_cast<int64_t>(n) + i], means[2 * static_cast<int64_t>(n) + i], __int_as_float(i));
  d.c = make_int4(c.x, c.y, c.z, 0);
  pts[pos] = d;
}

// rho_i = other points within r; sums of rho and rho^2 for the thresholds.
__global__ __launch_bounds__(256) void k_dc_density(int n, const DcPoint* __restrict__ pts,
                                                    const uint32_t* __restrict__ start, uint32_t T, float r2,
                                                    int32_t* __restrict__ rho, unsigned long long* __restrict__ isum) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  unsigned long long c1 = 0, c2 = 0;
  if (s < n) {
    const DcPoint q = pts[s];
    const int qi = __float_as_int(q.p.w);
    int cnt = 0;
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int cx = q.c.x + dx, cy = q.c.y + dy, cz = q.c.z + dz;
          const uint32_t b = dc_hash(cx, cy, cz, T - 1u);
          const uint32_t e = b + 1u < T ? start[b + 1u] : static_cast<uint32_t>(n);
          for (uint32_t p = start[b]; p < e; ++p) {
            const DcPoint o = pts[p];
            if (o.c.x != cx || o.c.y != cy || o.c.z != cz || __float_as_int(o.p.w) == qi) continue;
            if (dc_d2(q.p, o.p) <= r2) ++cnt;
          }
        }
    rho[qi] = cnt;
    c1 = static_cast<unsigned long long>(cnt);
    c2 = c1 * c1;
  }
  // wave sums, then one atomic per wave
  for (int o = 32; o > 0; o >>= 1) {
    c1 += __shfl_xor(c1, o, 64);
    c2 += __shfl_xor(c2, o, 64);
  }
  if ((threadIdx.x & 63) == 0 && (c1 || c2)) {
    atomicAdd(&isum[0], c1);
    atomicAdd(&isum[1], c2);
  }
}

// Thresholds from the exact integer sums, in FP64 with correctly rounded operations:
// mu = S1/n, sigma = sqrt(max(S2/n - mu^2, 0)), rho_low = mu - alpha sigma, rho_high = mu + beta sigma.
__global__ void k_dc_thresholds(int n, const unsigned long long* __restrict__ isum, double alpha, double beta,
                                double* __restrict__ stat) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double dn = static_cast<double>(n);
  const double mu = n > 0 ? __ddiv_rn(static_cast<double>(isum[0]), dn) : 0.0;
  const double var = n > 0 ? __dsub_rn(__ddiv_rn(static_cast<double>(isum[1]), dn), __dmul_rn(mu, mu)) : 0.0;
  const double sigma = __dsqrt_rn(var > 0.0 ? var : 0.0);
  stat[0] = mu;
  stat[1] = sigma;
  stat[2] = __dsub_rn(mu, __dmul_rn(alpha, sigma));
  stat[3] = __dadd_rn(mu, __dmul_rn(beta, sigma));
}

// Insert (d, j) into the K best, kept sorted by (d, index) in registers
// (unused slots hold (3e38, INT_MAX)): each slot keeps the smaller of its
// entry and the carried one and passes the larger on; the last falls off.
template <int K>
__device__ __forceinline__ void dc_insert(float (&bd)[K], int (&bi)[K], float d, int j) {
  if (!(d < bd[K - 1] || (d == bd[K - 1] && j < bi[K - 1]))) return;
  float cd = d;
  int cj = j;
#pragma unroll
  for (int m = 0; m < K; ++m) {
    const bool less = cd < bd[m] || (cd == bd[m] && cj < bi[m]);
    const float td = less ? bd[m] : cd;
    const int tj = less ? bi[m] : cj;
    bd[m] = less ? cd : bd[m];
    bi[m] = less ? cj : bi[m];
    cd = td;
    cj = tj;
  }
}

// A query's results from its K best: nearest point, its distance and the
// mean distance of the keff nearest; a1, a2 += the nearest distance and its square.
template <int K>
__device__ __forceinline__ void dc_finish(const float (&bd)[K], const int (&bi)[K], int keff, int qi,
                                          int32_t* __restrict__ nn, float* __restrict__ dnn,
                                          float* __restrict__ dbar, double& a1, double& a2) {
  float sum = 0.0f;
#pragma unroll
  for (int m = 0; m < K; ++m)
    if (m < keff) sum = __fadd_rn(sum, sqrtf(bd[m]));
  const float d0 = keff > 0 ? sqrtf(bd[0]) : 0.0f;
  nn[qi] = keff > 0 ? bi[0] : -1;
  dnn[qi] = d0;
  dbar[qi] = keff > 0 ? sum / static_cast<float>(keff) : 0.0f;
  if (keff > 0) {
    a1 += static_cast<double>(d0);
    a2 += static_cast<double>(d0) * static_cast<double>(d0);
  }
}

// Wave sums of the nearest-distance statistics, one atomic per wave.
__device__ __forceinline__ void dc_dsum(double a1, double a2, double* __restrict__ dsum) {
  for (int o = 32; o > 0; o >>= 1) {
    a1 += __shfl_xor(a1, o, 64);
    a2 += __shfl_xor(a2, o, 64);
  }
  if ((threadIdx.x & 63) == 0 && (a1 != 0.0 || a2 != 0.0)) {
    unsafeAtomicAdd(&dsum[0], a1);
    unsafeAtomicAdd(&dsum[1], a2);
  }
}

// The k nearest other points of every point, by (FP32 d2, index): nearest
// point, its distance and the mean distance of the k (FP32: square roots
// summed in order, over k); sums of the nearest distances for d_merge.
template <int K>
__global__ __launch_bounds__(256) void k_dc_knn(int n, const DcPoint* __restrict__ pts,
                                                const uint32_t* __restrict__ start, uint32_t T, float h,
                                                int32_t* __restrict__ nn, float* __restrict__ dnn,
                                                float* __restrict__ dbar, double* __restrict__ dsum,
                                                uint32_t* __restrict__ far, uint32_t* __restrict__ far_n) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  double a1 = 0.0, a2 = 0.0;
  if (s < n) {
    const DcPoint q = pts[s];
    const int qi = __float_as_int(q.p.w);
    const int keff = min(K, n - 1);
    float bd[K];
    int bi[K];
#pragma unroll
    for (int m = 0; m < K; ++m) { bd[m] = 3.0e38f; bi[m] = 0x7fffffff; }
    // fewer than K other points: no rings, straight to the scan of every point
    bool done = false;
    for (int R = 0; R < kDcRingsThread && !done && keff == K; ++R) {
      for (int dz = -R; dz <= R; ++dz)
        for (int dy = -R; dy <= R; ++dy)
          for (int dx = -R; dx <= R; ++dx) {
            if (max(max(abs(dx), abs(dy)), abs(dz)) != R) continue;   // the shell of ring R
            const int cx = q.c.x + dx, cy = q.c.y + dy, cz = q.c.z + dz;
            const uint32_t b = dc_hash(cx, cy, cz, T - 1u);
            const uint32_t e = b + 1u < T ? start[b + 1u] : static_cast<uint32_t>(n);
            for (uint32_t p = start[b]; p < e; ++p) {
              const DcPoint o = pts[p];
              const int oi = __float_as_int(o.p.w);
              if (o.c.x != cx || o.c.y != cy || o.c.z != cz || oi == qi) continue;
              dc_insert<K>(bd, bi, dc_d2(q.p, o.p), oi);
            }
          }
      // every point closer than (R - 1/16) h has been seen; the K-th best
      // (3e38 while fewer than K are held) must lie inside that
      const float g = (static_cast<float>(R) - 0.0625f) * h;
      if (g > 0.0f && bd[K - 1] <= g * g * 0.9999f) done = true;
    }
    if (!done) {
      // far neighbours (or fewer than K points): the wave kernel goes on with this query
      far[atomicAdd(far_n, 1u)] = static_cast<uint32_t>(s);
    } else {
      dc_finish<K>(bd, bi, keff, qi, nn, dnn, dbar, a1, a2);
    }
  }
  dc_dsum(a1, a2, dsum);
}

// Cell t of the shell of ring R (Chebyshev offset exactly R), t < shell(R):
// the two faces z = -R and z = +R ((2R+1)^2 cells each), then the ring of
// the 2R-1 layers between them (8R cells each).
__device__ __forceinline__ int3 dc_shell_cell(int R, int t) {
  const int side = 2 * R + 1, face = side * side;
  if (t < 2 * face) {
    const int z = t < face ? -R : R;
    const int u = t % face;
    return make_int3(u % side - R, u / side - R, z);
  }
  t -= 2 * face;
  const int per = 8 * R;
  const int z = t / per - (R - 1);
  int u = t % per;
  // walk the square's boundary: bottom row, right column, top row, left column
  if (u < side) return make_int3(u - R, -R, z);
  u -= side;
  if (u < side - 2) return make_int3(R, u - R + 1, z);
  u -= side - 2;
  if (u < side) return make_int3(R - u, R, z);
  u -= side;
  return make_int3(-R, R - 1 - u, z);
}

__device__ __forceinline__ int dc_shell_size(int R) { return R == 0 ? 1 : (2 * R + 1) * (2 * R + 1) * 2 + 8 * R * (2 * R - 1); }

// Queries the thread kernel left, one wave per query: rings 0-7, each ring's
// cells dealt to the 64 lanes, each lane its own top-k; the wave stops once
// K of the points its lanes hold lie inside the ring's guarantee.  Queries
// still open go on to the all-points kernel.
template <int K>
__global__ __launch_bounds__(256) void k_dc_knn_wave(int n, const DcPoint* __restrict__ pts,
                                                     const uint32_t* __restrict__ start, uint32_t T, float h,
                                                     const uint32_t* __restrict__ far, const uint32_t* __restrict__ far_n,
                                                     uint32_t* __restrict__ far2, uint32_t* __restrict__ far2_n,
                                                     int32_t* __restrict__ nn, float* __restrict__ dnn,
                                                     float* __restrict__ dbar, double* __restrict__ dsum) {
  __shared__ float s_d[4][64 * K];
  __shared__ int s_i[4][64 * K];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t count = *far_n;
  for (uint32_t f = blockIdx.x * 4 + wave; f < count; f += gridDim.x * 4) {
    const uint32_t slot = far[f];
    const DcPoint q = pts[slot];
    const int qi = __float_as_int(q.p.w);
    float bd[K];
    int bi[K];
#pragma unroll
    for (int m = 0; m < K; ++m) { bd[m] = 3.0e38f; bi[m] = 0x7fffffff; }
    bool done = false;
    const bool enough = n - 1 >= K;
    for (int R = 0; R < kDcRingsWave && !done && enough; ++R) {
      const int cells = dc_shell_size(R);
      for (int t = lane; t < cells; t += 64) {
        const int3 d = dc_shell_cell(R, t);
        const int cx = q.c.x + d.x, cy = q.c.y + d.y, cz = q.c.z + d.z;
        const uint32_t b = dc_hash(cx, cy, cz, T - 1u);
        const uint32_t e = b + 1u < T ? start[b + 1u] : static_cast<uint32_t>(n);
        for (uint32_t p = start[b]; p < e; ++p) {
          const DcPoint o = pts[p];
          const int oi = __float_as_int(o.p.w);
          if (o.c.x != cx || o.c.y != cy || o.c.z != cz || oi == qi) continue;
          dc_insert<K>(bd, bi, dc_d2(q.p, o.p), oi);
        }
      }
      const float g = (static_cast<float>(R) - 0.0625f) * h;
      if (g > 0.0f) {
        const float g2 = g * g * 0.9999f;
        int inside = 0;
#pragma unroll
        for (int m = 0; m < K; ++m) inside += __popcll(__ballot(bd[m] <= g2));
        done = inside >= K;
      }
    }
    if (!done) {
      if (lane == 0) far2[atomicAdd(far2_n, 1u)] = slot;
      continue;
    }
#pragma unroll
    for (int m = 0; m < K; ++m) {
      s_d[wave][lane * K + m] = bd[m];
      s_i[wave][lane * K + m] = bi[m];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane == 0) {
      for (int l = 1; l < 64; ++l)
        for (int m = 0; m < K; ++m) dc_insert<K>(bd, bi, s_d[wave][l * K + m], s_i[wave][l * K + m]);
      double a1 = 0.0, a2 = 0.0;
      dc_finish<K>(bd, bi, K, qi, nn, dnn, dbar, a1, a2);
      unsafeAtomicAdd(&dsum[0], a1);
      unsafeAtomicAdd(&dsum[1], a2);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// The queries the ring search left: a workgroup per (query, range of points)
// scans its range (each thread a strided share, its own top-k) and thread 0
// merges the 256 lists in LDS; with S > 1 ranges the lists go to cand_d /
// cand_i for k_dc_knn_far_merge, with one range the result is written here.
// Splitting keeps a few isolated queries from each holding one workgroup
// over every point (at 1M Gaussians, 44 queries took 1.7 ms that way).
template <int K>
__global__ __launch_bounds__(256) void k_dc_knn_far(int n, const DcPoint* __restrict__ pts,
                                                    const uint32_t* __restrict__ far, const uint32_t* __restrict__ far_n,
                                                    int32_t* __restrict__ nn, float* __restrict__ dnn,
                                                    float* __restrict__ dbar, double* __restrict__ dsum,
                                                    float* __restrict__ cand_d, int32_t* __restrict__ cand_i) {
  __shared__ float s_d[256 * K];
  __shared__ int s_i[256 * K];
  const uint32_t count = *far_n;
  const uint32_t S = far_splits(count);
  const uint32_t span = (static_cast<uint32_t>(n) + S - 1u) / S;
  // items (query f, range r): points [r span, (r + 1) span)
  for (uint32_t it = blockIdx.x; it < count * S; it += gridDim.x) {
    const uint32_t f = it / S, r = it - f * S;
    const DcPoint q = pts[far[f]];
    const int qi = __float_as_int(q.p.w);
    float bd[K];
    int bi[K];
#pragma unroll
    for (int m = 0; m < K; ++m) { bd[m] = 3.0e38f; bi[m] = 0x7fffffff; }
    const int p0 = static_cast<int>(r * span), p1 = min(n, static_cast<int>((r + 1u) * span));
    for (int p = p0 + threadIdx.x; p < p1; p += 256) {
      const DcPoint o = pts[p];
      const int oi = __float_as_int(o.p.w);
      if (oi != qi) dc_insert<K>(bd, bi, dc_d2(q.p, o.p), oi);
    }
#pragma unroll
    for (int m = 0; m < K; ++m) {
      s_d[threadIdx.x * K + m] = bd[m];
      s_i[threadIdx.x * K + m] = bi[m];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int t = 1; t < 256; ++t)
        for (int m = 0; m < K; ++m) dc_insert<K>(bd, bi, s_d[t * K + m], s_i[t * K + m]);
      if (S == 1) {
        double a1 = 0.0, a2 = 0.0;
        dc_finish<K>(bd, bi, min(K, n - 1), qi, nn, dnn, dbar, a1, a2);
        if (a1 != 0.0 || a2 != 0.0) {
          unsafeAtomicAdd(&dsum[0], a1);
          unsafeAtomicAdd(&dsum[1], a2);
        }
      } else {
#pragma unroll
        for (int m = 0; m < K; ++m) {
          cand_d[static_cast<size_t>(it) * 8 + m] = bd[m];
          cand_i[static_cast<size_t>(it) * 8 + m] = bi[m];
        }
      }
    }
    __syncthreads();
  }
}

// Merge of the split far search: query f's K nearest among its S ranges'
// lists, in (distance, index) order as every search keeps them.  One wave per
// query: lane r takes range r's list (r < S <= 64), then a butterfly over the
// lanes merges the lists pairwise (exact: the order is total).
template <int K>
__global__ __launch_bounds__(64) void k_dc_knn_far_merge(int n, const DcPoint* __restrict__ pts,
                                                         const uint32_t* __restrict__ far,
                                                         const uint32_t* __restrict__ far_n, int32_t* __restrict__ nn,
                                                         float* __restrict__ dnn, float* __restrict__ dbar,
                                                         double* __restrict__ dsum, const float* __restrict__ cand_d,
                                                         const int32_t* __restrict__ cand_i) {
  const uint32_t count = *far_n;
  const uint32_t S = far_splits(count);
  if (S == 1u) return;
  const uint32_t lane = threadIdx.x;
  for (uint32_t f = blockIdx.x; f < count; f += gridDim.x) {
    float bd[K];
    int bi[K];
#pragma unroll
    for (int m = 0; m < K; ++m) {
      const size_t o = (static_cast<size_t>(f) * S + lane) * 8 + m;
      bd[m] = lane < S ? cand_d[o] : 3.0e38f;
      bi[m] = lane < S ? cand_i[o] : 0x7fffffff;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      float od[K];
      int oi[K];
#pragma unroll
      for (int m = 0; m < K; ++m) {
        od[m] = __shfl_xor(bd[m], off, 64);
        oi[m] = __shfl_xor(bi[m], off, 64);
      }
#pragma unroll
      for (int m = 0; m < K; ++m) dc_insert<K>(bd, bi, od[m], oi[m]);
    }
    if (lane == 0) {
      const int qi = __float_as_int(pts[far[f]].p.w);
      double a1 = 0.0, a2 = 0.0;
      dc_finish<K>(bd, bi, min(K, n - 1), qi, nn, dnn, dbar, a1, a2);
      if (a1 != 0.0 || a2 != 0.0) {
        unsafeAtomicAdd(&dsum[0], a1);
        unsafeAtomicAdd(&dsum[1], a2);
      }
    }
  }
}

// d_merge = mu_d + gamma sigma_d over the nearest-neighbour distances.
__global__ void k_dc_merge_radius(int n, const double* __restrict__ dsum, double gamma, double* __restrict__ stat) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int m = n > 1 ? n : 0;
  const double dn = static_cast<double>(m);
  const double mu = m ? dsum[0] / dn : 0.0;
  const double var = m ? dsum[1] / dn - mu * mu : 0.0;
  const double sigma = sqrt(var > 0.0 ? var : 0.0);
  stat[4] = mu;
  stat[5] = sigma;
  stat[6] = mu + gamma * sigma;
}

// Classes and the merge pairing: keep[i] = 0 for the higher index of a
// merged pair, low[i] = 1 for a point that spawns a new one.
__global__ __launch_bounds__(256) void k_dc_classify(int n, const int32_t* __restrict__ rho,
                                                     const int32_t* __restrict__ nn, const float* __restrict__ dnn,
                                                     const double* __restrict__ stat, uint32_t* __restrict__ keep,
                                                     uint32_t* __restrict__ low, int32_t* __restrict__ partner,
                                                     uint8_t* __restrict__ cls_out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double lo = stat[2], hi = stat[3], dm = stat[6];
  auto cls = [&](int k) -> int {
    const double r = static_cast<double>(rho[k]);
    return r < lo ? 1 : (r > hi ? 2 : 0);
  };
  const int c = cls(i);
  const int j = nn[i];
  const bool pair = c == 2 && j >= 0 && cls(j) == 2 && nn[j] == i && static_cast<double>(dnn[i]) <= dm;
  partner[i] = pair ? j : -1;
  keep[i] = (pair && j < i) ? 0u : 1u;
  low[i] = c == 1 ? 1u : 0u;
  if (cls_out) cls_out[i] = static_cast<uint8_t>(c);
}

__device__ __forceinline__ float dc_sigmoid(float x) { return 1.0f / (1.0f + expf(-x)); }
__device__ __forceinline__ float dc_softplus(float x) { return x > 0.0f ? x + log1pf(expf(-x)) : log1pf(expf(x)); }

struct DcArrays {
  const float *means, *ls, *quats, *logits, *sh;
  float *o_means, *o_ls, *o_quats, *o_logits, *o_sh;
  int64_t cap;
  int nsh;  // 3 (D + 1)^2
};

// Output of every point: its own values, a merged pair's (at the lower index),
// and a new point next to each sparse point (after all kept points).
__global__ __launch_bounds__(256) void k_dc_write(int n, DcArrays A, const uint32_t* __restrict__ keep_pos,
                                                  const uint32_t* __restrict__ low_pos,
                                                  const int32_t* __restrict__ partner, const float* __restrict__ dbar,
                                                  const float* __restrict__ noise, float spread, float jitter,
                                                  const unsigned long long* __restrict__ total,
                                                  int32_t* __restrict__ fate) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int j = partner[i];
  const bool kept = !(j >= 0 && j < i);
  const int64_t cap = A.cap;
  const int64_t o = static_cast<int64_t>(keep_pos[i]);
  if (fate) fate[i] = kept ? static_cast<int32_t>(o) : -1;
  if (kept && o < cap) {
    if (j < 0) {
      for (int c = 0; c < 3; ++c) {
        A.o_means[c * cap + o] = A.means[c * static_cast<int64_t>(n) + i];
        A.o_ls[c * cap + o] = A.ls[c * static_cast<int64_t>(n) + i];
      }
      for (int c = 0; c < 4; ++c) A.o_quats[c * cap + o] = A.quats[c * static_cast<int64_t>(n) + i];
      A.o_logits[o] = A.logits[i];
      for (int c = 0; c < A.nsh; ++c) A.o_sh[c * cap + o] = A.sh[static_cast<int64_t>(c) * n + i];
    } else {
      // merge with j (j > i): opacity-weighted position and colour, mean
      // scale, accumulated opacity, the more opaque one's rotation
      const float li = A.logits[i], lj = A.logits[j];
      const float oi = dc_sigmoid(li), oj = dc_sigmoid(lj);
      const float w = oi + oj;
      for (int c = 0; c < 3; ++c) {
        A.o_means[c * cap + o] = (oi * A.means[c * static_cast<int64_t>(n) + i] + oj * A.means[c * static_cast<int64_t>(n) + j]) / w;
        A.o_ls[c * cap + o] = logf(0.5f * (expf(A.ls[c * static_cast<int64_t>(n) + i]) + expf(A.ls[c * static_cast<int64_t>(n) + j])));
      }
      const int qs = oj > oi ? j : i;
      for (int c = 0; c < 4; ++c) A.o_quats[c * cap + o] = A.quats[c * static_cast<int64_t>(n) + qs];
      // logit of 1 - (1 - oi)(1 - oj): log(o) + softplus(li) + softplus(lj)
      A.o_logits[o] = logf(oi + oj - oi * oj) + dc_softplus(li) + dc_softplus(lj);
      for (int c = 0; c < A.nsh; ++c) {
        const int64_t ci = static_cast<int64_t>(c) * n;
        A.o_sh[c * cap + o] = (oi * A.sh[ci + i] + oj * A.sh[ci + j]) / w;
      }
    }
  }
  const int64_t nl = static_cast<int64_t>(low_pos[i]);
  // low points: low_pos is the exclusive prefix of the low flags; the flag
  // itself is recovered from the next prefix (or the total)
  const int64_t next = i + 1 < n ? static_cast<int64_t>(low_pos[i + 1]) : static_cast<int64_t>(total[1]);
  if (next > nl) {
    const int64_t q = static_cast<int64_t>(total[0]) + nl;
    if (q < cap) {
      const float t = __fmul_rn(spread, dbar[i]);
      for (int c = 0; c < 3; ++c) {
        float p = __fadd_rn(A.means[c * static_cast<int64_t>(n) + i], __fmul_rn(t, noise[c * static_cast<int64_t>(n) + i]));
        p = __fadd_rn(p, __fmul_rn(jitter, noise[(3 + c) * static_cast<int64_t>(n) + i]));
        A.o_means[c * cap + q] = p;
        A.o_ls[c * cap + q] = A.ls[c * static_cast<int64_t>(n) + i];
      }
      for (int c = 0; c < 4; ++c) A.o_quats[c * cap + q] = A.quats[c * static_cast<int64_t>(n) + i];
      A.o_logits[q] = A.logits[i];
      for (int c = 0; c < A.nsh; ++c) A.o_sh[c * cap + q] = A.sh[static_cast<int64_t>(c) * n + i];
    }
  }
}

gs_status launch_density_control(const gs_gaussians& g, const gs_density_params& prm, const float* noise,
                                 gs_param_arrays& out, int64_t cap, void* ws, gs_density_report* rep,
                                 gs_density_points* pts_out, hipStream_t s) {
  const int n = static_cast<int>(g.n);
  DcWs w = carve_dc(ws, n);
  const uint32_t T = dc_table(n);
  const float h = prm.radius * kDcCellScale;
  const float inv_h = 1.0f / h;
  const float r2 = prm.radius * prm.radius;  // r r, rounded once
  const unsigned gn = static_cast<unsigned>(std::max<int64_t>(ceil_div(n, 256), 1));
  gs_status st;
  { TimedLaunch t("k_dc_clear", s); k_dc_clear<<<static_cast<unsigned>(ceil_div(T, 256)), 256, 0, s>>>(w.count, w.fill, T, w.isum, w.dsum,
                                                                                               w.total, w.range, w.far_n, w.far2_n); }
  if ((st = check_launch("k_dc_clear")) != GS_OK) return st;
  if (n > 0) {
    { TimedLaunch t("k_dc_cells", s); k_dc_cells<<<gn, 256, 0, s>>>(n, g.means, inv_h, T - 1u, w.cell, w.count, w.range); }
    if ((st = check_launch("k_dc_cells")) != GS_OK) return st;
    if ((st = launch_exclusive_scan(w.count, w.count, T, w.sums, nullptr, s)) != GS_OK) return st;
    { TimedLaunch t("k_dc_scatter", s); k_dc_scatter<<<gn, 256, 0, s>>>(n, g.means, w.cell, w.count, w.fill, w.pts); }
    if ((st = check_launch("k_dc_scatter")) != GS_OK) return st;
    { TimedLaunch t("k_dc_density", s); k_dc_density<<<gn, 256, 0, s>>>(n, w.pts, w.count, T, r2, w.rho, w.isum); }
    if ((st = check_launch("k_dc_density")) != GS_OK) return st;
  }
  { TimedLaunch t("k_dc_thresholds", s); k_dc_thresholds<<<1, 64, 0, s>>>(n, w.isum, static_cast<double>(prm.alpha),
                                                                         static_cast<double>(prm.beta), w.stat); }
  if ((st = check_launch("k_dc_thresholds")) != GS_OK) return st;
  if (n > 0) {
#define GS_DC_KNN(K)                                                                                             \
  {                                                                                                              \
    { TimedLaunch t("k_dc_knn<" #K ">", s);                                                                     \
      k_dc_knn<K><<<gn, 256, 0, s>>>(n, w.pts, w.count, T, h, w.nn, w.dnn, w.dbar, w.dsum, w.far, w.far_n); }   \
    { TimedLaunch t("k_dc_knn_wave<" #K ">", s);                                                                \
      k_dc_knn_wave<K><<<2048, 256, 0, s>>>(n, w.pts, w.count, T, h, w.far, w.far_n, w.far2, w.far2_n, w.nn,      \
                                            w.dnn, w.dbar, w.dsum); }                                             \
    { TimedLaunch t("k_dc_knn_far<" #K ">", s);                                                                 \
      k_dc_knn_far<K><<<1024, 256, 0, s>>>(n, w.pts, w.far2, w.far2_n, w.nn, w.dnn, w.dbar, w.dsum, w.cand_d,     \
                                           w.cand_i); }                                                          \
    { TimedLaunch t("k_dc_knn_far_merge<" #K ">", s);                                                           \
      k_dc_knn_far_merge<K><<<256, 64, 0, s>>>(n, w.pts, w.far2, w.far2_n, w.nn, w.dnn, w.dbar, w.dsum, w.cand_d,  \
                                              w.cand_i); }                                                       \
  }
    switch (prm.knn) {
      case 1: GS_DC_KNN(1); break;
      case 2: GS_DC_KNN(2); break;
      case 3: GS_DC_KNN(3); break;
      case 4: GS_DC_KNN(4); break;
      case 5: GS_DC_KNN(5); break;
      case 6: GS_DC_KNN(6); break;
      case 7: GS_DC_KNN(7); break;
      default: GS_DC_KNN(8); break;
    }
#undef GS_DC_KNN
    if ((st = check_launch("k_dc_knn")) != GS_OK) return st;
  }
  { TimedLaunch t("k_dc_merge_radius", s); k_dc_merge_radius<<<1, 64, 0, s>>>(n, w.dsum, static_cast<double>(prm.gamma), w.stat); }
  if ((st = check_launch("k_dc_merge_radius")) != GS_OK) return st;
  int64_t kept = 0, nlow = 0;
  if (n > 0) {
    { TimedLaunch t("k_dc_classify", s); k_dc_classify<<<gn, 256, 0, s>>>(n, w.rho, w.nn, w.dnn, w.stat, w.keep, w.low, w.partner,
                                                                       pts_out ? pts_out->cls : nullptr); }
    if ((st = check_launch("k_dc_classify")) != GS_OK) return st;
    if (pts_out) {
      // the per-point statistics, before the scans overwrite the flags
      if (pts_out->rho && (st = check_hip(hipMemcpyAsync(pts_out->rho, w.rho, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s),
                                          "hipMemcpyAsync(rho)")) != GS_OK) return st;
      if (pts_out->nn && (st = check_hip(hipMemcpyAsync(pts_out->nn, w.nn, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s),
                                         "hipMemcpyAsync(nn)")) != GS_OK) return st;
      if (pts_out->dbar && (st = check_hip(hipMemcpyAsync(pts_out->dbar, w.dbar, sizeof(float) * n, hipMemcpyDeviceToDevice, s),
                                           "hipMemcpyAsync(dbar)")) != GS_OK) return st;
    }
    if ((st = launch_exclusive_scan(w.keep, w.keep, n, w.sums, &w.total[0], s)) != GS_OK) return st;
    if ((st = launch_exclusive_scan(w.low, w.low, n, w.sums, &w.total[1], s)) != GS_OK) return st;
    DcArrays A{g.means, g.log_scales, g.quats, g.logits, g.sh,
               out.means, out.log_scales, out.quats, out.logits, out.sh, cap, 3 * (g.sh_degree + 1) * (g.sh_degree + 1)};
    { TimedLaunch t("k_dc_write", s); k_dc_write<<<gn, 256, 0, s>>>(n, A, w.keep, w.low, w.partner, w.dbar, noise, prm.spread, prm.jitter,
                                                                 w.total, pts_out ? pts_out->fate : nullptr); }
    if ((st = check_launch("k_dc_write")) != GS_OK) return st;
    unsigned long long tot[2] = {0, 0};
    uint32_t range = 0;
    if ((st = check_hip(hipMemcpyAsync(tot, w.total, sizeof tot, hipMemcpyDeviceToHost, s), "hipMemcpyAsync(total)")) != GS_OK)
      return st;
    if ((st = check_hip(hipMemcpyAsync(&range, w.range, sizeof range, hipMemcpyDeviceToHost, s), "hipMemcpyAsync(range)")) != GS_OK)
      return st;
    double stat[8];
    if ((st = check_hip(hipMemcpyAsync(stat, w.stat, sizeof stat, hipMemcpyDeviceToHost, s), "hipMemcpyAsync(stat)")) != GS_OK)
      return st;
    if ((st = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize")) != GS_OK) return st;
    if (range)
      return fail(GS_ERR_UNSUPPORTED, "gs_density_control: a coordinate is not finite or lies 2^18 cells (of 1.07 r) "
                                      "or more from the origin; the outputs are undefined");
    kept = static_cast<int64_t>(tot[0]);
    nlow = static_cast<int64_t>(tot[1]);
    if (rep) {
      rep->rho_mean = stat[0]; rep->rho_std = stat[1]; rep->rho_low = stat[2]; rep->rho_high = stat[3];
      rep->d_mean = stat[4]; rep->d_std = stat[5]; rep->d_merge = stat[6];
    }
  }
  if (rep) {
    rep->n_in = n;
    rep->n_merged = n - kept;
    rep->n_new = nlow;
    rep->n_out = kept + nlow;
  }
  if (kept + nlow > cap)
    return fail(GS_ERR_CAPACITY, "gs_density_control: the output needs " + std::to_string(kept + nlow) +
                                     " Gaussians, the capacity is " + std::to_string(cap));
  return GS_OK;
}

}  // namespace gs
