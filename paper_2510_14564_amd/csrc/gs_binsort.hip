// Tile binning and depth sort.
//
// Paper: Sec. II-A (the Gaussians that reach a pixel are blended in depth
// order) and Sec. IV-C.1 (16x16 pixel tiles share one Gaussian list).  The
// required order of the (tile, Gaussian) entries is (tile, FP32 depth bits,
// Gaussian index).  Instead of radix-sorting K 64-bit keys (about 6 passes over
// K entries), the path
//   1. sorts the N Gaussians by depth bits with a stable LSD radix sort that
//      starts from index order, which yields (depth bits, index) order;
//   2. places every (tile, Gaussian) entry directly at its final position,
//      counting for each tile the earlier depth ranks that cover it (the
//      direct emission below, in two levels: 8 x 8-tile super tiles, then
//      tiles); or, for frames of more tiles than that handles,
//   2'. emits every Gaussian's tiles in rank order at the exclusive prefix
//      sum of its tile counts and stably sorts the K entries by tile id
//      (ceil(log2 T) bits, 1-2 passes).
// Both keep the (depth, index) order inside each tile, so the result equals
// the full sort bit for bit.
#include "gs_internal.h"

namespace gs {

constexpr int kRsThreads = 256;
constexpr int kOsItemsN = 8;    // depth sort of N keys (onesweep): 4096 keys per workgroup of 8 waves
constexpr int kOsThreads = 512;
constexpr int kRsItemsK = 16;   // tile sort of K entries: 4096 keys per block
constexpr int kScanItems = 16;
constexpr int kScanChunk = 256 * kScanItems;

__device__ __forceinline__ uint64_t lanemask_lt() {
  const unsigned lane = __lane_id();
  return (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
}

// Lanes of this wave whose `digit` (nbits wide) equals ours, among `active`:
// per bit, the ballot xor this lane's bit spread over 64 bits marks the lanes
// that differ in that bit; the peers are the valid lanes marked by none.
// Unrolled for the full 8-bit digit (every pass of a 32-bit key).
__device__ __forceinline__ void match_bit(uint32_t digit, int b, uint32_t& lo, uint32_t& hi) {
  // bit b of the digit spread over 32 bits (0 or all ones)
  const uint32_t sb = static_cast<uint32_t>(static_cast<int32_t>(digit << (31 - b)) >> 31);
  const uint64_t m = __ballot(sb != 0u);
  lo |= static_cast<uint32_t>(m) ^ sb;
  hi |= static_cast<uint32_t>(m >> 32) ^ sb;
}
__device__ __forceinline__ uint64_t match_digit(uint32_t digit, int nbits, bool valid) {
  uint32_t lo = 0u, hi = 0u;
  if (nbits == 8) {
#pragma unroll
    for (int b = 0; b < 8; ++b) match_bit(digit, b, lo, hi);
  } else {
    for (int b = 0; b < nbits; ++b) match_bit(digit, b, lo, hi);
  }
  return __ballot(valid) & ~((static_cast<uint64_t>(hi) << 32) | lo);
}

// --------------------------------------------------------------- device scan
// Exclusive prefix sum of uint32 values: per-block sums, one-block scan of the
// sums (which also yields the 64-bit total), then per-block scan + offset.

// Inclusive prefix sum over the 64 lanes on DPP (row shifts, then the row
// broadcasts of lanes 15 and 31): no LDS round trips.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xF, true);
}
__device__ __forceinline__ int wave_incl_scan(int x) {
  x += dpp_i32<0x111, 0xF>(x);   // row_shr:1
  x += dpp_i32<0x112, 0xF>(x);   // row_shr:2
  x += dpp_i32<0x114, 0xF>(x);   // row_shr:4
  x += dpp_i32<0x118, 0xF>(x);   // row_shr:8
  x += dpp_i32<0x142, 0xA>(x);   // row_bcast:15 into rows 1, 3
  x += dpp_i32<0x143, 0xC>(x);   // row_bcast:31 into rows 2, 3
  return x;
}

// Exclusive prefix over a 256-thread workgroup: wave scans on DPP, then the
// four wave totals through LDS (lds >= 4 words; free again on return).
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* lds, uint32_t& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t incl = static_cast<uint32_t>(wave_incl_scan(static_cast<int>(v)));
  if (lane == 63) lds[wave] = incl;
  __syncthreads();
  const uint32_t w0 = lds[0], w1 = lds[1], w2 = lds[2], w3 = lds[3];
  const uint32_t before = (wave > 0 ? w0 : 0u) + (wave > 1 ? w1 : 0u) + (wave > 2 ? w2 : 0u);
  total = ((w0 + w1) + w2) + w3;
  __syncthreads();
  return before + incl - v;
}

// Exclusive prefix over a workgroup of W waves (lds >= W words; free again
// on return), the same as block_exclusive_scan for W = 4.
template <int W>
__device__ __forceinline__ uint32_t block_exclusive_scan_n(uint32_t v, uint32_t* lds, uint32_t& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t incl = static_cast<uint32_t>(wave_incl_scan(static_cast<int>(v)));
  if (lane == 63) lds[wave] = incl;
  __syncthreads();
  uint32_t before = 0u, all = 0u;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const uint32_t x = lds[w];
    before += (w < wave) ? x : 0u;
    all += x;
  }
  total = all;
  __syncthreads();
  return before + incl - v;
}

__global__ __launch_bounds__(256) void k_scan_sums(const uint32_t* __restrict__ in, int64_t n,
                                                   uint32_t* __restrict__ sums) {
  __shared__ uint32_t red[256];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanChunk;
  uint32_t s = 0;
  for (int j = 0; j < kScanItems; ++j) {
    const int64_t idx = base + j * 256 + threadIdx.x;
    if (idx < n) s += in[idx];
  }
  // wave totals (lane 63 of the DPP scan), then the four in a fixed order
  const uint32_t w = static_cast<uint32_t>(__builtin_amdgcn_readlane(wave_incl_scan(static_cast<int>(s)), 63));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x == 0) sums[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// Chunk bounds of the direct emission, derived from the scanned counts (see
// k_scan_apply<true>): with K the total, chunk size E = max(min_entries,
// ceil(K / target)) and count C = min(ceil(K / E), cmax), bounds[c] is the
// first rank whose exclusive offset is >= c E for c < C, and n for
// C <= c <= cmax.  k_dev != NULL: K and the depth sort's look-back flag
// (total[1]) are also copied to k_dev[0], k_dev[1].
struct ChunkArgs {
  uint32_t* bounds;
  int cmax;
  unsigned long long min_entries, target;
  unsigned long long* k_dev;
};

// Per chunk: its offset is the sum of the sums of all earlier chunks, which
// every block adds up itself (a few thousand values at most, read from L2) --
// no separate top-level scan launch.  The last block also writes the 64-bit
// total.  Thread t owns items [16 t, 16 t + 16) of the chunk; whole, 16-byte
// aligned runs move as four 16-byte accesses.
// BOUNDS: instead of the offsets, write the chunk bounds of ChunkArgs.  Every
// block also sums all chunk sums (K); item i, whose offsets span (offs[i],
// offs[i] + cnt[i]], holds the bound of every chunk c >= 1 with c E in that
// span: bounds[c] = i + 1 (the lower bound of c E among the offsets).
template <bool BOUNDS>
__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t* __restrict__ in, int64_t n,
                                                    const uint32_t* __restrict__ sums, uint32_t* __restrict__ out,
                                                    unsigned long long* __restrict__ total, ChunkArgs ca) {
  __shared__ uint32_t lds[256];
  __shared__ unsigned long long red[2][4];
  const int b = blockIdx.x;
  unsigned long long pre = 0, all = 0;
  const int upto = BOUNDS ? static_cast<int>(gridDim.x) : b;
  for (int i = threadIdx.x; i < upto; i += 256) {
    const uint32_t x = sums[i];
    if (i < b) pre += x;
    all += x;
  }
  for (int o = 32; o > 0; o >>= 1) {
    pre += __shfl_xor(pre, o, 64);
    if (BOUNDS) all += __shfl_xor(all, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = pre;
    red[1][threadIdx.x >> 6] = all;
  }
  __syncthreads();
  const unsigned long long offset = red[0][0] + red[0][1] + red[0][2] + red[0][3];
  const int64_t base = static_cast<int64_t>(b) * kScanChunk;
  uint32_t v[kScanItems];
  uint32_t s = 0;
  const int64_t my = base + static_cast<int64_t>(threadIdx.x) * kScanItems;
  const bool vec = my + kScanItems <= n && ((reinterpret_cast<uintptr_t>(in + my) |
                                              (BOUNDS ? 0u : reinterpret_cast<uintptr_t>(out + my))) & 15u) == 0;
  if (vec) {
#pragma unroll
    for (int q = 0; q < kScanItems / 4; ++q) {
      const uint4 w = reinterpret_cast<const uint4*>(in + my)[q];
      v[4 * q] = w.x; v[4 * q + 1] = w.y; v[4 * q + 2] = w.z; v[4 * q + 3] = w.w;
    }
  } else {
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) v[j] = my + j < n ? in[my + j] : 0u;
  }
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) s += v[j];
  uint32_t tot;
  const uint32_t local = block_exclusive_scan(s, lds, tot);
  if constexpr (BOUNDS) {
    const unsigned long long K = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    const unsigned long long E = max(ca.min_entries, (K + ca.target - 1) / ca.target);
    const unsigned long long C = min((K + E - 1) / E, static_cast<unsigned long long>(ca.cmax));
    unsigned long long o = offset + local;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      const unsigned long long hi = o + v[j];
      for (unsigned long long c = o / E + 1; c < C && c * E <= hi; ++c) ca.bounds[c] = static_cast<uint32_t>(my + j + 1);
      o = hi;
    }
    if (b == 0) {
      for (int c = threadIdx.x; c <= ca.cmax; c += 256)
        if (static_cast<unsigned long long>(c) >= C) ca.bounds[c] = static_cast<uint32_t>(n);
        else if (c == 0) ca.bounds[0] = 0u;
      if (ca.k_dev && threadIdx.x == 0) { ca.k_dev[0] = K; ca.k_dev[1] = total[1]; }
    }
  } else {
    uint32_t o[kScanItems];
    uint32_t run = local + static_cast<uint32_t>(offset);
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      o[j] = run;
      run += v[j];
    }
    if (vec) {
#pragma unroll
      for (int q = 0; q < kScanItems / 4; ++q)
        reinterpret_cast<uint4*>(out + my)[q] = make_uint4(o[4 * q], o[4 * q + 1], o[4 * q + 2], o[4 * q + 3]);
    } else {
#pragma unroll
      for (int j = 0; j < kScanItems; ++j)
        if (my + j < n) out[my + j] = o[j];
    }
  }
  if (total && b == static_cast<int>(gridDim.x) - 1 && threadIdx.x == 0) *total = offset + tot;
}

struct ScanWs {
  uint32_t* sums;
  unsigned long long* total;
};

static size_t scan_ws_words(int64_t n) { return static_cast<size_t>(ceil_div(n > 0 ? n : 1, kScanChunk)); }

static gs_status device_exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, ScanWs ws, hipStream_t s) {
  const int nb = static_cast<int>(ceil_div(n > 0 ? n : 1, kScanChunk));
  { TimedLaunch gs_tl("k_scan_sums", s); k_scan_sums<<<nb, 256, 0, s>>>(in, n, ws.sums); }
  { TimedLaunch gs_tl("k_scan_apply<false>", s); k_scan_apply<false><<<nb, 256, 0, s>>>(in, n, ws.sums, out, ws.total, ChunkArgs{}); }
  return check_launch("device_exclusive_scan");
}

// The scan's total and the direct emission's chunk bounds (no offsets).
static gs_status device_chunk_bounds(const uint32_t* in, int64_t n, ScanWs ws, ChunkArgs ca, hipStream_t s) {
  const int nb = static_cast<int>(ceil_div(n > 0 ? n : 1, kScanChunk));
  { TimedLaunch gs_tl("k_scan_sums", s); k_scan_sums<<<nb, 256, 0, s>>>(in, n, ws.sums); }
  { TimedLaunch gs_tl("k_scan_apply<true>", s); k_scan_apply<true><<<nb, 256, 0, s>>>(in, n, ws.sums, nullptr, ws.total, ca); }
  return check_launch("device_chunk_bounds");
}

size_t scan_sums_words(int64_t n) { return scan_ws_words(n); }

gs_status launch_exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* sums,
                                unsigned long long* total, hipStream_t s) {
  return device_exclusive_scan(in, out, n, ScanWs{sums, total}, s);
}

// ---------------------------------------------------------------- radix sort
// One stable LSD pass on (key, value) pairs over `nbits` bits at `shift`.
// Block b owns keys [b*CHUNK, (b+1)*CHUNK); wave w of the block owns the
// contiguous quarter [w*CHUNK/4, (w+1)*CHUNK/4) and walks it 64 keys at a
// time.  A key's rank among equal digits is (keys of earlier waves) + (earlier
// rounds of its wave) + (earlier lanes of its round), so the pass is stable.
// Within a wave the running digit counters need no barrier (a wave's LDS
// operations complete in order); the cross-wave offsets are combined once.

template <int ITEMS>
__global__ __launch_bounds__(kRsThreads) void k_rs_hist(const uint32_t* __restrict__ keys, int64_t count,
                                                        int shift, int nbits, uint32_t* __restrict__ hist,
                                                        int nblocks) {
  constexpr int CHUNK = kRsThreads * ITEMS;
  __shared__ uint32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t mask = (1u << nbits) - 1u;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * CHUNK;
  // all loads first, so that they are in flight together
  uint32_t kk[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const int64_t idx = base + j * kRsThreads + threadIdx.x;
    kk[j] = idx < count ? keys[idx] : 0u;
  }
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const int64_t idx = base + j * kRsThreads + threadIdx.x;
    const bool valid = idx < count;
    const uint32_t d = (kk[j] >> shift) & mask;
    const uint64_t peers = match_digit(d, nbits, valid);
    if (valid && (peers & lanemask_lt()) == 0) atomicAdd(&cnt[d], static_cast<uint32_t>(__popcll(peers)));
  }
  __syncthreads();
  if (threadIdx.x <= mask) hist[static_cast<int64_t>(threadIdx.x) * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

template <int ITEMS>
__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(const uint32_t* __restrict__ keys_in,
                                                           const uint32_t* __restrict__ vals_in,
                                                           uint32_t* __restrict__ keys_out,
                                                           uint32_t* __restrict__ vals_out, int64_t count,
                                                           int shift, int nbits,
                                                           const uint32_t* __restrict__ hist_scan, int nblocks) {
  constexpr int CHUNK = kRsThreads * ITEMS;
  constexpr int PER_WAVE = CHUNK / 4;
  __shared__ uint32_t sk[CHUNK];
  __shared__ uint32_t sv[CHUNK];
  __shared__ uint32_t wrun[4][256];   // per-wave running digit counts
  __shared__ uint32_t dstart[256];    // block-local start of each digit
  __shared__ uint32_t gbase[256];     // global start of each digit for this block
  __shared__ uint32_t scan_tmp[256];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const uint32_t mask = (1u << nbits) - 1u;
  wrun[0][tid] = 0; wrun[1][tid] = 0; wrun[2][tid] = 0; wrun[3][tid] = 0;
  gbase[tid] = (static_cast<uint32_t>(tid) <= mask) ? hist_scan[static_cast<int64_t>(tid) * nblocks + blockIdx.x] : 0u;
  __syncthreads();
  const int64_t base = static_cast<int64_t>(blockIdx.x) * CHUNK + static_cast<int64_t>(wave) * PER_WAVE;
  const uint64_t below = lanemask_lt();
  uint32_t k[ITEMS], v[ITEMS], lr[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const int64_t idx = base + j * 64 + lane;
    const bool valid = idx < count;
    k[j] = valid ? keys_in[idx] : 0u;
    v[j] = valid ? vals_in[idx] : 0u;
  }
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const int64_t idx = base + j * 64 + lane;
    const bool valid = idx < count;
    const uint32_t d = (k[j] >> shift) & mask;
    const uint64_t peers = match_digit(d, nbits, valid);
    const uint32_t before = valid ? wrun[wave][d] : 0u;
    lr[j] = before + static_cast<uint32_t>(__popcll(peers & below));
    if (valid && (peers & below) == 0) wrun[wave][d] = before + static_cast<uint32_t>(__popcll(peers));
  }
  __syncthreads();
  // per digit: offsets of waves 1..3 and the block total, then block-local starts
  const uint32_t c0 = wrun[0][tid], c1 = wrun[1][tid], c2 = wrun[2][tid], c3 = wrun[3][tid];
  uint32_t tot;
  const uint32_t ds = block_exclusive_scan(c0 + c1 + c2 + c3, scan_tmp, tot);
  __syncthreads();
  wrun[0][tid] = ds;
  wrun[1][tid] = ds + c0;
  wrun[2][tid] = ds + c0 + c1;
  wrun[3][tid] = ds + c0 + c1 + c2;
  dstart[tid] = ds;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const int64_t idx = base + j * 64 + lane;
    if (idx < count) {
      const uint32_t d = (k[j] >> shift) & mask;
      const uint32_t pos = wrun[wave][d] + lr[j];
      sk[pos] = k[j];
      sv[pos] = v[j];
    }
  }
  __syncthreads();
  const int64_t bbase = static_cast<int64_t>(blockIdx.x) * CHUNK;
  const int64_t nvalid = min(static_cast<int64_t>(CHUNK), count - bbase);
  for (int p = tid; p < nvalid; p += kRsThreads) {
    const uint32_t key = sk[p];
    const uint32_t d = (key >> shift) & mask;
    const uint32_t g = gbase[d] + (static_cast<uint32_t>(p) - dstart[d]);
    keys_out[g] = key;
    vals_out[g] = sv[p];
  }
}

static gs_status scan_hist(uint32_t* hist, int64_t nh, ScanWs sws, hipStream_t s) {
  ScanWs w = sws;
  w.total = nullptr;
  return device_exclusive_scan(hist, hist, nh, w, s);
}

// Sorts `count` pairs over key bits [0, total_bits) in passes of <= 8 bits.
// Input in (ka, va); the sorted result ends in (ka, va) if the pass count is
// even, else in (kb, vb).  Returns the number of passes.
template <int ITEMS>
static gs_status radix_sort_pairs(uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb, int64_t count,
                                  int total_bits, uint32_t* hist, ScanWs sws, hipStream_t s, int* passes_out) {
  constexpr int CHUNK = kRsThreads * ITEMS;
  int passes = 0;
  if (count > 0) {
    const int nblocks = static_cast<int>(ceil_div(count, CHUNK));
    for (int shift = 0; shift < total_bits; shift += 8) {
      const int nbits = min(8, total_bits - shift);
      const int64_t nh = static_cast<int64_t>(1 << nbits) * nblocks;
      { TimedLaunch gs_tl("k_rs_hist", s); k_rs_hist<ITEMS><<<nblocks, kRsThreads, 0, s>>>(ka, count, shift, nbits, hist, nblocks); }
      gs_status st = scan_hist(hist, nh, sws, s);
      if (st != GS_OK) return st;
      { TimedLaunch gs_tl("k_rs_scatter", s); k_rs_scatter<ITEMS><<<nblocks, kRsThreads, 0, s>>>(ka, va, kb, vb, count, shift, nbits, hist, nblocks); }
      st = check_launch("k_rs_scatter");
      if (st != GS_OK) return st;
      uint32_t* t = ka; ka = kb; kb = t;
      t = va; va = vb; vb = t;
      ++passes;
    }
  }
  *passes_out = passes;
  return GS_OK;
}

// Tile count of a packed rectangle (x0 | x_end << 16, y0 | y_end << 16).
__device__ __forceinline__ uint32_t rect_count(uint2 rc) {
  return ((rc.x >> 16) - (rc.x & 0xFFFFu)) * ((rc.y >> 16) - (rc.y & 0xFFFFu));
}

// The rectangle, in the same packing, of the blocks of 2^shift x 2^shift
// tiles that a tile rectangle touches (empty stays empty; shift 0: itself).
__device__ __forceinline__ uint2 rect_at(uint2 rc, int shift) {
  const uint32_t add = (1u << shift) - 1u;
  const uint32_t x0 = (rc.x & 0xFFFFu) >> shift, xe = ((rc.x >> 16) + add) >> shift;
  const uint32_t y0 = (rc.y & 0xFFFFu) >> shift, ye = ((rc.y >> 16) + add) >> shift;
  return make_uint2(x0 | (xe << 16), y0 | (ye << 16));
}

// ------------------------------------------------------------ onesweep sort
// Stable LSD radix sort of (key, value) pairs in passes of up to 8 bits, one
// sweep per pass:
//   k_os_hist     one read of the keys: the global digit counts of every
//                 pass at once (workgroup counts in LDS, then one atomic per
//                 digit per workgroup); it also clears the pass state below.
//   k_os_scatter  per pass: workgroup v (in the order workgroups start, from
//                 an atomic counter) ranks chunk v of the keys stably, then
//                 learns how many keys of each digit the chunks before it
//                 hold by decoupled look-back: it publishes its own digit
//                 counts, walks back over its predecessors' published words
//                 (a count, or an inclusive prefix that ends the walk) and
//                 publishes its inclusive prefix.  A workgroup waits only on
//                 workgroups that started before it and publish their counts
//                 without waiting, so every wait ends; each spin is bounded
//                 all the same, and a bound that runs out sets an error flag.
// Published words pack a 2-bit state with a 30-bit count and are read and
// written with device-scope atomics, which keep them coherent across XCDs.

constexpr uint32_t kOsEmpty = 0u, kOsAgg = 1u, kOsIncl = 2u;
constexpr uint32_t kOsCountMask = (1u << 30) - 1u;
constexpr int kOsHistBlocks = 256;   // more workgroups queue on the digit counts' atomics
constexpr int kOsMaxPasses = 4;
constexpr uint32_t kOsSpinLimit = 1u << 22;
constexpr int kOsWindow = 8;

__device__ __forceinline__ uint32_t os_load(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void os_store(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ghist[pass][256] must be zero on entry.  Clears state[] (state_words) and
// the per-pass start counters.
__global__ __launch_bounds__(256) void k_os_hist(const uint32_t* __restrict__ keys, int64_t count, int total_bits,
                                                 uint32_t* __restrict__ ghist, uint32_t* __restrict__ state,
                                                 int64_t state_words, uint32_t* __restrict__ counters) {
  __shared__ uint32_t h[kOsMaxPasses][256];
  const int passes = (total_bits + 7) / 8;
  for (int p = 0; p < kOsMaxPasses; ++p) h[p][threadIdx.x] = 0;
  const int64_t gtid = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const int64_t gstride = static_cast<int64_t>(gridDim.x) * 256;
  for (int64_t i = gtid; i < state_words; i += gstride) state[i] = 0u;
  if (gtid < kOsMaxPasses) counters[gtid] = 0u;
  __syncthreads();
  constexpr int U = 8;
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * 256 * U; base < count; base += gstride * U) {
    uint32_t k[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t idx = base + u * 256 + threadIdx.x;
      k[u] = idx < count ? keys[idx] : 0u;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (base + u * 256 + threadIdx.x >= count) continue;
      for (int p = 0; p < passes; ++p) {
        const int nbits = min(8, total_bits - 8 * p);
        atomicAdd(&h[p][(k[u] >> (8 * p)) & ((1u << nbits) - 1u)], 1u);
      }
    }
  }
  __syncthreads();
  for (int p = 0; p < passes; ++p)
    if (h[p][threadIdx.x]) atomicAdd(&ghist[p * 256 + threadIdx.x], h[p][threadIdx.x]);
}

// Pass `pass` of the sort over key bits [0, total_bits).  A pass whose digit
// is the same for every key keeps the order.  The last pass that changes it
// (from the digit counts of every pass, ghist) is the terminal one: it writes
// the values in their final order to vals_final, with each value's rectangle
// and tile count when rect != NULL, and no keys; the passes after it return
// at once.  (All passes trivial: pass 0 is terminal and copies.)
template <int ITEMS, int THREADS>
__global__ __launch_bounds__(THREADS) void k_os_scatter(const uint32_t* __restrict__ keys_in,
                                                           const uint32_t* __restrict__ vals_in,
                                                           uint32_t* __restrict__ keys_out,
                                                           uint32_t* __restrict__ vals_out, int64_t count,
                                                           int pass, int total_bits,
                                                           const uint32_t* __restrict__ ghist,
                                                           uint32_t* __restrict__ state_pass,
                                                           uint32_t* __restrict__ counter, uint32_t* __restrict__ err,
                                                           uint32_t* __restrict__ vals_final,
                                                           const uint2* __restrict__ rect,
                                                           uint2* __restrict__ rect_out,
                                                           uint32_t* __restrict__ cnt_out, int cshift) {
  constexpr int CHUNK = THREADS * ITEMS;
  constexpr int WAVES = THREADS / 64;
  constexpr int PER_WAVE = CHUNK / WAVES;
  static_assert(THREADS >= 256, "one thread per digit");
  __shared__ uint32_t s_vid, s_whole;
  const int passes = (total_bits + 7) / 8;
  const int shift = 8 * pass, nbits = min(8, total_bits - 8 * pass);
  // every pass's digit counts are read at once (one HBM round trip, not one
  // per pass behind a barrier), and the chunk's virtual id is drawn alongside
  uint32_t gh[kOsMaxPasses];
#pragma unroll
  for (int q = 0; q < kOsMaxPasses; ++q) gh[q] = (q < passes && threadIdx.x < 256) ? ghist[q * 256 + threadIdx.x] : 0u;
  if (threadIdx.x == 0) {
    s_whole = 0u;
    s_vid = atomicAdd(counter, 1u);
  }
  __syncthreads();
  // the chunk's keys (whatever the pass turns out to be: a returning or
  // copying workgroup has read a few KB for nothing)
  const uint32_t vid = s_vid;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int64_t base = static_cast<int64_t>(vid) * CHUNK + static_cast<int64_t>(wave) * PER_WAVE;
  uint32_t k[ITEMS], v[ITEMS], lr[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const int64_t idx = base + j * 64 + lane;
    const bool valid = idx < count;
    k[j] = valid ? keys_in[idx] : 0u;
    v[j] = valid ? vals_in[idx] : 0u;
  }
  // bit q of s_whole: some digit of pass q holds every key (the pass keeps the order)
  uint32_t mine = 0u;
#pragma unroll
  for (int q = 0; q < kOsMaxPasses; ++q) {
    const int qb = min(8, total_bits - 8 * q);
    if (q < passes && static_cast<uint32_t>(threadIdx.x) <= ((1u << qb) - 1u) && static_cast<int64_t>(gh[q]) == count)
      mine |= 1u << q;
  }
  if (mine) atomicOr(&s_whole, mine);
  __shared__ uint32_t sk[CHUNK];
  __shared__ uint32_t sv[CHUNK];
  __shared__ uint32_t wrun[WAVES][256];   // per-wave running digit counts
  __shared__ uint32_t dstart[256];    // block-local start of each digit
  __shared__ uint32_t gbase[256];     // global start of each digit for this block
  __shared__ uint32_t scan_tmp[WAVES];
  for (int i = tid; i < WAVES * 256; i += THREADS) (&wrun[0][0])[i] = 0u;
  __syncthreads();
  const uint32_t whole = s_whole;
  int last_changing = 0;
  for (int q = 0; q < passes; ++q)
    if (!((whole >> q) & 1u)) last_changing = q;
  const bool trivial = (whole >> pass) & 1u;
  if (pass > last_changing) return;   // the order is final already
  const bool terminal = pass == last_changing;
  auto emit = [&](int64_t g, uint32_t key, uint32_t val) {
    if (terminal) {
      vals_final[g] = val;
      if (rect) {
        const uint2 rc = rect[val];
        rect_out[g] = rc;
        cnt_out[g] = rect_count(rect_at(rc, cshift));
      }
    } else {
      keys_out[g] = key;
      vals_out[g] = val;
    }
  };
  // every key has the same digit: the pass keeps the order (a copy)
  if (trivial) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * CHUNK + threadIdx.x;
         i < min(count, static_cast<int64_t>(blockIdx.x + 1) * CHUNK); i += THREADS)
      emit(i, keys_in[i], vals_in[i]);
    return;
  }
  const uint32_t mask = (1u << nbits) - 1u;
  const uint64_t below = lanemask_lt();
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const int64_t idx = base + j * 64 + lane;
    const bool valid = idx < count;
    const uint32_t d = (k[j] >> shift) & mask;
    const uint64_t peers = match_digit(d, nbits, valid);
    const uint32_t before = valid ? wrun[wave][d] : 0u;
    lr[j] = before + static_cast<uint32_t>(__popcll(peers & below));
    if (valid && (peers & below) == 0) wrun[wave][d] = before + static_cast<uint32_t>(__popcll(peers));
  }
  __syncthreads();
  // per digit (thread tid < 256): wave offsets and the block's count, then
  // block-local starts
  const bool digit = tid < 256;
  uint32_t cnt = 0u;
  if (digit)
#pragma unroll
    for (int w = 0; w < WAVES; ++w) cnt += wrun[w][tid];
  uint32_t tot;
  const uint32_t ds = block_exclusive_scan_n<WAVES>(cnt, scan_tmp, tot);
  // global digit starts of this pass: exclusive scan of the global counts
  uint32_t ghp = 0u;
#pragma unroll
  for (int q = 0; q < kOsMaxPasses; ++q) ghp = q == pass ? gh[q] : ghp;
  const uint32_t gd = block_exclusive_scan_n<WAVES>(static_cast<uint32_t>(tid) <= mask ? ghp : 0u, scan_tmp, tot);
  // decoupled look-back, one digit per thread
  uint32_t prefix = 0;
  if (static_cast<uint32_t>(tid) <= mask) {
    uint32_t* mine = state_pass + static_cast<int64_t>(vid) * 256 + tid;
    if (vid == 0) {
      os_store(mine, (kOsIncl << 30) | cnt);
    } else {
      os_store(mine, (kOsAgg << 30) | cnt);
      // walk back kOsWindow predecessors at a time (their loads in flight
      // together): add counts until an inclusive prefix; at a predecessor
      // that has not published yet, wait for it and reload from there
      int64_t j = static_cast<int64_t>(vid) - 1;
      uint32_t spins = 0;
      bool found = false;
      while (j >= 0 && !found) {
        uint32_t w[kOsWindow];
#pragma unroll
        for (int u = 0; u < kOsWindow; ++u) w[u] = (j - u >= 0) ? os_load(state_pass + (j - u) * 256 + tid) : 0u;
        int used = 0;
        bool blocked = false;
#pragma unroll
        for (int u = 0; u < kOsWindow; ++u) {
          if (found || blocked || j - u < 0) continue;
          const uint32_t f = w[u] >> 30;
          if (f == kOsEmpty) { blocked = true; continue; }
          prefix += w[u] & kOsCountMask;
          ++used;
          if (f == kOsIncl) found = true;
        }
        j -= used;
        if (blocked && !found) {
          if (++spins > kOsSpinLimit) { atomicOr(err, 1u); break; }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      os_store(mine, (kOsIncl << 30) | ((prefix + cnt) & kOsCountMask));
    }
  }
  if (digit) {
    uint32_t run = ds;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
      const uint32_t c = wrun[w][tid];
      wrun[w][tid] = run;
      run += c;
    }
    dstart[tid] = ds;
    gbase[tid] = gd + prefix;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const int64_t idx = base + j * 64 + lane;
    if (idx < count) {
      const uint32_t d = (k[j] >> shift) & mask;
      const uint32_t pos = wrun[wave][d] + lr[j];
      sk[pos] = k[j];
      sv[pos] = v[j];
    }
  }
  __syncthreads();
  const int64_t bbase = static_cast<int64_t>(vid) * CHUNK;
  const int nvalid = static_cast<int>(min(static_cast<int64_t>(CHUNK), count - bbase));
  if (terminal && rect) {
    // the final order with each value's rectangle: all of the thread's
    // gathers in flight together
    uint32_t g[ITEMS], val[ITEMS];
    uint2 rc[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const int p = tid + j * THREADS;
      if (p < nvalid) {
        const uint32_t d = (sk[p] >> shift) & mask;
        g[j] = gbase[d] + (static_cast<uint32_t>(p) - dstart[d]);
        val[j] = sv[p];
        rc[j] = rect[val[j]];
      }
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      if (tid + j * THREADS < nvalid) {
        vals_final[g[j]] = val[j];
        rect_out[g[j]] = rc[j];
        cnt_out[g[j]] = rect_count(rect_at(rc[j], cshift));
      }
    }
    return;
  }
  for (int p = tid; p < nvalid; p += THREADS) {
    const uint32_t key = sk[p];
    const uint32_t d = (key >> shift) & mask;
    const uint32_t g = gbase[d] + (static_cast<uint32_t>(p) - dstart[d]);
    emit(g, key, sv[p]);
  }
}

struct OsWs {
  uint32_t* ghist;     // [kOsMaxPasses][256]
  uint32_t* state;     // [passes][chunks][256]
  uint32_t* counters;  // [kOsMaxPasses]
  uint32_t* err;       // [1]
};

static size_t os_state_words(int64_t count, int chunk, int passes) {
  return static_cast<size_t>(passes) * 256 * static_cast<size_t>(ceil_div(std::max<int64_t>(count, 1), chunk));
}

// Sorts `count` pairs over key bits [0, total_bits).  Input in (ka, va),
// which the passes use as ping-pong buffers with (kb, vb); the values in
// sorted order end in vals_final (with rect: each value's rectangle in
// rect_out and in cnt_out the count of the blocks of 2^cshift x 2^cshift
// tiles it touches -- its tile count for cshift 0).
// w.ghist must be zero on entry (k_depth_keys clears both sorts' counts).
template <int ITEMS, int THREADS>
static gs_status onesweep_sort_pairs(uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb, int64_t count,
                                     int total_bits, OsWs w, hipStream_t s, uint32_t* vals_final,
                                     const uint2* rect = nullptr, uint2* rect_out = nullptr,
                                     uint32_t* cnt_out = nullptr, int cshift = 0) {
  constexpr int CHUNK = THREADS * ITEMS;
  const int passes = (total_bits + 7) / 8;
  if (count <= 0) return GS_OK;
  const int nblocks = static_cast<int>(ceil_div(count, CHUNK));
  gs_status st;
  const int hb = static_cast<int>(std::min<int64_t>(kOsHistBlocks, ceil_div(count, 256 * 8)));
  { TimedLaunch gs_tl("k_os_hist", s); k_os_hist<<<std::max(hb, 1), 256, 0, s>>>(ka, count, total_bits, w.ghist, w.state,
                                            static_cast<int64_t>(os_state_words(count, CHUNK, passes)), w.counters); }
  if ((st = check_launch("k_os_hist")) != GS_OK) return st;
  for (int p = 0; p < passes; ++p) {
    { TimedLaunch gs_tl("k_os_scatter", s); k_os_scatter<ITEMS, THREADS><<<nblocks, THREADS, 0, s>>>(ka, va, kb, vb, count, p, total_bits, w.ghist,
                                                       w.state + static_cast<size_t>(p) * nblocks * 256,
                                                       w.counters + p, w.err, vals_final, rect, rect_out, cnt_out,
                                                       cshift); }
    if ((st = check_launch("k_os_scatter")) != GS_OK) return st;
    uint32_t* t = ka; ka = kb; kb = t;
    t = va; va = vb; vb = t;
  }
  return GS_OK;
}

static int sort_passes(int bits) { return (bits + 7) / 8; }

// ------------------------------------------------------------- bin kernels

// Depth keys, and each Gaussian's tile rectangle packed into 8 bytes
// (x0 | x_end << 16, y0 | y_end << 16, ends exclusive; all zero when empty) so
// that the later rank-order passes read one small word per Gaussian instead
// of its record and radius.  Also clears `zero_words` words at `zero` (the
// depth sort's digit counts, K and the look-back error flag).
__global__ __launch_bounds__(256) void k_depth_keys(int n, const float* __restrict__ depth,
                                                    const float4* __restrict__ records,
                                                    const int* __restrict__ radius, int tiles_x, int tiles_y,
                                                    uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                    uint2* __restrict__ rect, uint32_t* __restrict__ zero,
                                                    int zero_words) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  for (int z = i; z < zero_words; z += gridDim.x * blockDim.x) zero[z] = 0u;
  if (i >= n) return;
  keys[i] = __float_as_uint(depth[i]);
  vals[i] = static_cast<uint32_t>(i);
  const float4 r0 = records[3 * static_cast<int64_t>(i)];
  int x0, x1, y0, y1;
  const int c = tile_rect(r0.x, r0.y, radius[i], tiles_x, tiles_y, x0, x1, y0, y1);
  rect[i] = c > 0 ? make_uint2(static_cast<uint32_t>(x0) | (static_cast<uint32_t>(x1 + 1) << 16),
                               static_cast<uint32_t>(y0) | (static_cast<uint32_t>(y1 + 1) << 16))
                  : make_uint2(0u, 0u);
}

// Emit: a wave takes 64 consecutive depth ranks and writes all of their
// (tile, Gaussian) entries cooperatively -- lane l writes entries l, l+64, ...
// of the wave's contiguous output range -- so stores are coalesced and a
// Gaussian covering thousands of tiles does not serialise one thread.  Each
// Gaussian's tiles are written row-major over its rectangle.
__global__ __launch_bounds__(256) void k_emit(int n, const uint32_t* __restrict__ order,
                                              const uint32_t* __restrict__ offsets,
                                              const uint2* __restrict__ rect_rank, int tiles_x,
                                              uint32_t* __restrict__ tile_keys, uint32_t* __restrict__ gids) {
  __shared__ uint32_t s_pre[4][65];   // exclusive prefix of entry counts within the wave, plus total
  __shared__ uint32_t s_gid[4][64];
  __shared__ int s_x0[4][64], s_y0[4][64], s_w[4][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = (blockIdx.x * 4 + wave) * 64 + lane;
  uint32_t cnt = 0, gid = 0;
  int x0 = 0, x1 = -1, y0 = 0;
  if (r < n) {
    gid = order[r];
    const uint2 rc = rect_rank[r];
    cnt = rect_count(rc);
    x0 = static_cast<int>(rc.x & 0xFFFFu); x1 = static_cast<int>(rc.x >> 16) - 1;
    y0 = static_cast<int>(rc.y & 0xFFFFu);
  }
  // inclusive scan of cnt over the wave (Hillis-Steele with shuffles)
  uint32_t incl = cnt;
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t t = __shfl_up(incl, d, 64);
    if (lane >= d) incl += t;
  }
  s_pre[wave][lane] = incl - cnt;
  if (lane == 63) s_pre[wave][64] = incl;
  s_gid[wave][lane] = gid;
  s_x0[wave][lane] = x0;
  s_y0[wave][lane] = y0;
  s_w[wave][lane] = x1 - x0 + 1;
  __syncthreads();
  const int r0 = (blockIdx.x * 4 + wave) * 64;
  if (r0 >= n) return;
  const uint32_t total = s_pre[wave][64];
  const uint32_t base = offsets[r0];
  for (uint32_t p = lane; p < total; p += 64) {
    // owner: the last k with s_pre[k] <= p (binary search over 64 prefixes)
    int lo = 0, hi = 63;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_pre[wave][mid] <= p) lo = mid; else hi = mid - 1;
    }
    const uint32_t j = p - s_pre[wave][lo];
    const uint32_t w = static_cast<uint32_t>(s_w[wave][lo]);
    // row = j / w without an integer division: the float quotient is within
    // one of the exact one for j, w < 2^24 (tiles of a rectangle), corrected
    // by one integer step
    uint32_t row = static_cast<uint32_t>(static_cast<float>(j) * __builtin_amdgcn_rcpf(static_cast<float>(w)));
    if (row * w > j) --row;
    else if ((row + 1) * w <= j) ++row;
    const uint32_t col = j - row * w;
    tile_keys[base + p] = static_cast<uint32_t>((s_y0[wave][lo] + static_cast<int>(row)) * tiles_x +
                                                s_x0[wave][lo] + static_cast<int>(col));
    gids[base + p] = s_gid[wave][lo];
  }
}

// ranges[t] = [lower_bound(t), lower_bound(t + 1)) over the sorted tile ids.
__global__ __launch_bounds__(256) void k_ranges(int ntiles, const uint32_t* __restrict__ tiles, uint32_t K,
                                                uint2* __restrict__ ranges) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntiles) return;
  auto lb = [&](uint32_t key) {
    uint32_t lo = 0, hi = K;
    while (lo < hi) {
      const uint32_t mid = lo + ((hi - lo) >> 1);
      if (tiles[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
  };
  ranges[t] = make_uint2(lb(static_cast<uint32_t>(t)), lb(static_cast<uint32_t>(t + 1)));
}

// ----------------------------------------------------------- direct emission
// The tile sort without sorting.  After the depth sort the entries of tile t
// are, in order, the depth ranks whose rectangle contains t.  Two levels,
// with super tiles of 8 x 8 tiles.
// Coarse: the ranks are cut into C chunks of about E coarse entries each
// (chunk c = ranks [R_c, R_c+1); a rank has one coarse entry per super tile
// its rectangle touches).
//  1. k_chunk_count: per chunk, the coarse entries of every super tile, from
//     a 2D difference array of the chunk's super-tile rectangles in LDS (four
//     LDS atomics per Gaussian, then prefix sums along rows and columns) --
//     table[c][s]; it also adds up the tile counts (K).
//  2. k_chunk_colscan: per super tile, the exclusive prefix over chunks (in
//     place) and the total; k_coarse_parts: the super tiles' starts in the
//     coarse list and the cut of each super tile's run into parts of at most
//     kPart entries (numbered over the super tiles in turn).
//  3. k_emit_coarse: one workgroup per chunk walks its ranks 256 at a time.
//     Rank 64 w + l of a group comes before rank 64 w' + l' on a super tile
//     that both rectangles contain iff (w, l) < (w', l'); with per-wave 64-bit
//     masks col[w][x] (lanes whose rectangle spans column x) and row[w][y],
//     the number of the group's ranks before rank 64 w + l on (x, y) is
//     sum_{w' < w} popc(col[w'][x] & row[w'][y]) + popc(col[w][x] & row[w][y]
//     & lanes below l).  So each entry computes its final position from the
//     super tile's position at the group start.  A coarse entry holds the
//     Gaussian and its rectangle within the super tile.
// Fine: per part (a run of one super tile's coarse entries, in rank order),
//  4. k_fine_count: the entries of each of the super tile's 64 tiles;
//     k_fine_scan: per super tile, their exclusive prefix over its parts and
//     the tile totals; k_tile_starts: the tiles' starts (the ranges).
//  5. k_fine_emit: a wave takes 64 coarse entries, one per lane.  The entries
//     covering one of the 64 tiles are the 64-bit mask col[x] & row[y] of the
//     wave, so the tile's entries go out in one store: lane l at the tile's
//     position plus the count of the mask's lanes below l.  The waves of a
//     workgroup take consecutive runs of 64 and offset each tile by the
//     earlier waves' counts.
// A tile's stores are consecutive addresses from one workgroup, so a line
// fills in L2 before it leaves; entries written straight from the chunks to
// the tiles land as four-byte pieces scattered over the whole list, and lines
// leave L2 partly written, several times over.
// Same result as a stable sort by tile of the rank-ordered emission, i.e. the
// order (tile, depth bits, index).  Used for frames of at most
// kDirectMaxTiles tiles.
constexpr int kSuperShift = 3;            // super tiles of 8 x 8 tiles
constexpr int kSuper = 1 << kSuperShift;
constexpr int kDirectChunks = 512;        // chunks at most
constexpr int64_t kDirectMinEntries = 4096;
constexpr size_t kLdsBudget = 65536;      // bytes of LDS per workgroup
constexpr size_t kEmitStaticLds = 11776;  // k_emit_coarse's fixed arrays, rounded up
constexpr int kPart = 1024;               // coarse entries per part of the fine passes
constexpr int kFineThreads = 256;
constexpr int kFineWaves = kFineThreads / 64;
constexpr int kPartSteps = kPart / kFineThreads;
constexpr int kFineGrid = 2048;           // workgroups of the fine passes at most (each loops over parts)
constexpr int kDirectMaxTiles = 16384;    // tiles at most (one workgroup writes the tile starts)

static int super_dim(int tiles) { return (tiles + kSuper - 1) >> kSuperShift; }

// LDS of the coarse emission over an sx x sy grid of super tiles: masks
// col[4][sx], row[4][sy] (u64), then pos[sx sy] (u32) and delta[sx sy] (u16).
static size_t emit_dyn_lds(int sx, int sy) {
  const size_t nt = static_cast<size_t>(sx) * sy;
  return 32 * static_cast<size_t>(sx + sy) + 4 * nt + 2 * ((nt + 1) / 2 * 2);
}
static bool direct_ok(int tiles_x, int tiles_y) {
  const int sx = super_dim(tiles_x), sy = super_dim(tiles_y);
  return static_cast<size_t>(tiles_x) * tiles_y <= static_cast<size_t>(kDirectMaxTiles) &&
         4 * static_cast<size_t>(sx + 1) * (sy + 1) <= kLdsBudget &&
         emit_dyn_lds(sx, sy) + kEmitStaticLds <= kLdsBudget;
}
static int64_t direct_max_chunks(int64_t cap) {
  return std::max<int64_t>(1, std::min<int64_t>(kDirectChunks, ceil_div(std::max<int64_t>(cap, 1), kDirectMinEntries)));
}
// parts at most: every super tile's run of at most `cap` coarse entries in total
static int64_t direct_max_parts(int64_t cap, int ns) { return ceil_div(std::max<int64_t>(cap, 1), kPart) + ns; }

// In-place inclusive prefix sums of `len` ints at p[0], p[stride], ... by one wave.
__device__ __forceinline__ void wave_prefix_lds(int* p, int len, int stride, int lane) {
  int carry = 0;
  for (int b = 0; b < len; b += 64) {
    const int i = b + lane;
    const int v = wave_incl_scan(i < len ? p[i * stride] : 0);
    if (i < len) p[i * stride] = v + carry;
    carry += __builtin_amdgcn_readlane(v, 63);
  }
}

constexpr int kDirectThreads = 1024;
constexpr int kDirectWaves = kDirectThreads / 64;

// Per chunk: table[c][s] over the sx x sy super tiles, and the chunk's tile
// counts added to *kfine.
__global__ __launch_bounds__(kDirectThreads) void k_chunk_count(const uint32_t* __restrict__ bounds,
                                                                const uint2* __restrict__ rect_rank, int sx, int sy,
                                                                uint32_t* __restrict__ table,
                                                                unsigned long long* __restrict__ kfine) {
  extern __shared__ int s_diff[];   // (sy + 1) rows of (sx + 1)
  __shared__ unsigned long long s_k[kDirectWaves];
  const int c = blockIdx.x, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int pitch = sx + 1, cells = pitch * (sy + 1);
  for (int i = tid; i < cells; i += kDirectThreads) s_diff[i] = 0;
  __syncthreads();
  const uint32_t r1 = bounds[c + 1];
  unsigned long long fine = 0;
  for (uint32_t r = bounds[c] + tid; r < r1; r += kDirectThreads) {
    const uint2 rc = rect_rank[r];
    fine += rect_count(rc);
    const uint2 sr = rect_at(rc, kSuperShift);
    if (rect_count(sr) == 0) continue;
    const int x0 = static_cast<int>(sr.x & 0xFFFFu), xe = static_cast<int>(sr.x >> 16);
    const int y0 = static_cast<int>(sr.y & 0xFFFFu), ye = static_cast<int>(sr.y >> 16);
    atomicAdd(&s_diff[y0 * pitch + x0], 1);
    atomicAdd(&s_diff[y0 * pitch + xe], -1);
    atomicAdd(&s_diff[ye * pitch + x0], -1);
    atomicAdd(&s_diff[ye * pitch + xe], 1);
  }
  for (int o = 32; o > 0; o >>= 1) fine += __shfl_xor(fine, o, 64);
  if (lane == 0) s_k[wave] = fine;
  __syncthreads();
  if (tid == 0) {
    unsigned long long k = 0;
    for (int w = 0; w < kDirectWaves; ++w) k += s_k[w];
    if (k) atomicAdd(kfine, k);
  }
  for (int y = wave; y < sy; y += kDirectWaves) wave_prefix_lds(s_diff + y * pitch, sx, 1, lane);
  __syncthreads();
  for (int x = wave; x < sx; x += kDirectWaves) wave_prefix_lds(s_diff + x, sy, pitch, lane);
  __syncthreads();
  uint32_t* const out = table + static_cast<size_t>(c) * sx * sy;
  for (int y = wave; y < sy; y += kDirectWaves)
    for (int x = lane; x < sx; x += 64) out[y * sx + x] = static_cast<uint32_t>(s_diff[y * pitch + x]);
}

// One workgroup (16 waves) per 64 columns (tiles or super tiles); wave w owns
// a contiguous range of at most kDirectChunks / 16 chunks, whose counts it
// holds in registers (one read of the table, all loads in flight at once).
// table[c][t] becomes the entries of t in chunks before c; total[t] is t's
// count.
constexpr int kColPer = kDirectChunks / 16;
__global__ __launch_bounds__(1024) void k_chunk_colscan(int C, int ntiles, uint32_t* __restrict__ table,
                                                        uint32_t* __restrict__ total) {
  __shared__ uint32_t s_part[16][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int t = blockIdx.x * 64 + lane;
  const int per = (C + 15) / 16;   // at most kColPer (C <= kDirectChunks)
  const int c0 = min(C, wave * per), c1 = min(C, c0 + per);
  uint32_t v[kColPer];
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kColPer; ++k) {
    v[k] = (t < ntiles && c0 + k < c1) ? table[static_cast<size_t>(c0 + k) * ntiles + t] : 0u;
    sum += v[k];
  }
  s_part[wave][lane] = sum;
  __syncthreads();
  uint32_t run = 0, all = 0;
  for (int w = 0; w < 16; ++w) {
    const uint32_t x = s_part[w][lane];
    run += (w < wave) ? x : 0u;
    all += x;
  }
  if (t >= ntiles) return;
  if (wave == 0) total[t] = all;
#pragma unroll
  for (int k = 0; k < kColPer; ++k) {
    if (c0 + k < c1) table[static_cast<size_t>(c0 + k) * ntiles + t] = run;
    run += v[k];
  }
}

// Exclusive prefix of one 64-bit value per thread over a workgroup of
// THREADS threads (s_w: THREADS / 64 words of LDS, free again on return);
// `all` is the sum.
template <int THREADS>
__device__ __forceinline__ unsigned long long block_exclusive_u64(unsigned long long v, unsigned long long* s_w,
                                                                  unsigned long long& all) {
  constexpr int W = THREADS / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  unsigned long long incl = v;
  for (int d = 1; d < 64; d <<= 1) {
    const unsigned long long u = __shfl_up(incl, d, 64);
    if (lane >= d) incl += u;
  }
  if (lane == 63) s_w[wave] = incl;
  __syncthreads();
  unsigned long long before = incl - v;
  all = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    all += s_w[w];
    before += (w < wave) ? s_w[w] : 0ull;
  }
  __syncthreads();
  return before;
}

// start[t] = exclusive prefix of total over the tiles, ranges[t] = (start,
// start + total), by one workgroup.  K = *kfine (the sum of the tile counts)
// goes to rb[0] and, if given, k_dev[0]; *fits = whether the entries fit.  If
// they do not fit in `capacity`, every range is written empty instead, so
// that work queued on these lists before the caller learns of the overflow
// (the no-wait call) reads nothing past the buffers.
struct StartArgs {
  int ntiles;
  uint32_t* start;
  uint2* ranges;
  unsigned long long capacity;
  const unsigned long long* kfine;
  unsigned long long* rb;
  unsigned long long* k_dev;
  uint32_t* fits;
};
constexpr int kStartRegs = kDirectMaxTiles / 1024;   // a thread's totals, all loads in flight at once
__global__ __launch_bounds__(1024) void k_tile_starts(const uint32_t* __restrict__ total, StartArgs a) {
  __shared__ unsigned long long s_w[16];
  // the tile totals, then the tile starts: read and written tile by tile
  // across the lanes (coalesced), scanned in runs of consecutive tiles
  __shared__ uint32_t s_t[kDirectMaxTiles];
  const int tid = threadIdx.x;
  for (int t = tid; t < a.ntiles; t += 1024) s_t[t] = total[t];
  __syncthreads();
  const int per = (a.ntiles + 1023) / 1024;   // at most kStartRegs: direct_ok bounds the tiles
  const int t0 = min(a.ntiles, tid * per), t1 = min(a.ntiles, t0 + per);
  uint32_t v[kStartRegs];
  unsigned long long sum = 0;
#pragma unroll
  for (int k = 0; k < kStartRegs; ++k) {
    v[k] = t0 + k < t1 ? s_t[t0 + k] : 0u;
    sum += v[k];
  }
  unsigned long long all;
  unsigned long long run = block_exclusive_u64<1024>(sum, s_w, all);
  const unsigned long long K = *a.kfine;
  // positions are 32-bit: a total beyond that does not fit either
  const bool fits = K <= min(a.capacity, 0xFFFFFFFFull);
  if (tid == 0) {
    a.rb[0] = K;
    if (a.k_dev) a.k_dev[0] = K;
    *a.fits = fits ? 1u : 0u;
  }
  __syncthreads();   // every thread has read its totals
#pragma unroll
  for (int k = 0; k < kStartRegs; ++k) {
    if (t0 + k < t1) s_t[t0 + k] = static_cast<uint32_t>(run);
    run += v[k];
  }
  __syncthreads();
  // tile t ends where tile t + 1 starts (the last one at the total)
  for (int t = tid; t < a.ntiles; t += 1024) {
    const uint32_t st = s_t[t];
    const uint32_t en = t + 1 < a.ntiles ? s_t[t + 1] : static_cast<uint32_t>(all);
    a.start[t] = st;
    a.ranges[t] = fits ? make_uint2(st, en) : make_uint2(0u, 0u);
  }
}

// Super tile s's run of the coarse list starts at start[s] (exclusive prefix
// of the totals) and is cut into parts of kPart entries, numbered over the
// super tiles in turn: parts pbase[s] .. pbase[s+1]-1 (pbase[ns]: all parts).
// A coarse list longer than its buffer (capacity) gives no parts: K is at
// least as large, so the frame is reported as not fitting.
__global__ __launch_bounds__(1024) void k_coarse_parts(int ns, const uint32_t* __restrict__ ctotal,
                                                       uint32_t* __restrict__ cstart, unsigned long long capacity,
                                                       uint32_t* __restrict__ pbase) {
  __shared__ unsigned long long s_w[16];
  const int tid = threadIdx.x;
  const int per = (ns + 1023) / 1024;
  const int t0 = min(ns, tid * per), t1 = min(ns, t0 + per);
  unsigned long long sum = 0, psum = 0;
  for (int t = t0; t < t1; ++t) {
    const uint32_t v = ctotal[t];
    sum += v;
    psum += (v + kPart - 1) / kPart;
  }
  unsigned long long all, pall;
  unsigned long long run = block_exclusive_u64<1024>(sum, s_w, all);
  unsigned long long prun = block_exclusive_u64<1024>(psum, s_w, pall);
  const bool fits = all <= min(capacity, 0xFFFFFFFFull);
  for (int t = t0; t < t1; ++t) {
    const uint32_t v = ctotal[t];
    cstart[t] = static_cast<uint32_t>(run);
    pbase[t] = fits ? static_cast<uint32_t>(prun) : 0u;
    run += v;
    prun += (v + kPart - 1) / kPart;
  }
  if (tid == 0) pbase[ns] = fits ? static_cast<uint32_t>(pall) : 0u;
}

// Inclusive max over the 64 lanes on DPP (row shifts, then the row broadcasts
// of lanes 15 and 31); lanes shifted in from outside a row read 0.
__device__ __forceinline__ uint32_t wave_incl_max(uint32_t x) {
  x = max(x, static_cast<uint32_t>(dpp_i32<0x111, 0xF>(static_cast<int>(x))));   // row_shr:1
  x = max(x, static_cast<uint32_t>(dpp_i32<0x112, 0xF>(static_cast<int>(x))));   // row_shr:2
  x = max(x, static_cast<uint32_t>(dpp_i32<0x114, 0xF>(static_cast<int>(x))));   // row_shr:4
  x = max(x, static_cast<uint32_t>(dpp_i32<0x118, 0xF>(static_cast<int>(x))));   // row_shr:8
  x = max(x, static_cast<uint32_t>(dpp_i32<0x142, 0xA>(static_cast<int>(x))));   // row_bcast:15 into rows 1, 3
  x = max(x, static_cast<uint32_t>(dpp_i32<0x143, 0xC>(static_cast<int>(x))));   // row_bcast:31 into rows 2, 3
  return x;
}

// Owner of entry e0 + lane among the ranks of one rank-wave (offsets
// pre[0..64]): the last rank with a nonzero count whose offset is <= the
// entry.  Lane k looks at rank k: the run's first entry belongs to the
// highest such rank at or before e0 (a ballot), and each rank starting inside
// the run marks its first entry's lane in the wave's 64-word scratch; an
// inclusive max over the lanes then hands every entry its rank -- three LDS
// accesses and a DPP scan instead of a six-step dependent binary search.
__device__ __forceinline__ int run_owner(const uint32_t* __restrict__ pre, uint32_t e0, uint32_t* __restrict__ mark,
                                         int lane) {
  const uint32_t pk = pre[lane], pk1 = pre[lane + 1];
  const bool nz = pk1 > pk;
  const uint64_t before = __ballot(nz && pk <= e0);   // nonzero: entry e0 exists
  const uint32_t k0 = 63u - static_cast<uint32_t>(__clzll(before));
  mark[lane] = 0u;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  if (nz && pk > e0 && pk < e0 + 64u) mark[pk - e0] = static_cast<uint32_t>(lane) + 1u;
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  uint32_t v = mark[lane];
  if (lane == 0) v = k0 + 1u;
  return static_cast<int>(wave_incl_max(v)) - 1;
}

// Placement of coarse entry e of rank-wave rw (uniform over the wave) of the
// current group (offsets pre[0..64], total pre[64]), owned by rank lo of the
// rank-wave: the entry goes to its super tile's position at the group start
// plus the group's earlier ranks on that super tile; the group's last entry
// on a super tile stores the group's count there.  s_rect holds the ranks'
// super-tile rectangles, s_frect their tile rectangles.
__device__ __forceinline__ void place_entry(int rw, uint32_t e, int lo, const uint32_t* __restrict__ pre,
                                            const uint2* __restrict__ s_rect, const uint2* __restrict__ s_frect,
                                            const uint32_t* __restrict__ s_magic,
                                            const uint32_t* __restrict__ s_gid,
                                            const unsigned long long* __restrict__ s_dyn,
                                            const uint32_t* __restrict__ s_pos, uint16_t* __restrict__ s_delta,
                                            int edge, int tiles_x, unsigned long long* __restrict__ coarse,
                                            uint32_t capacity) {
  if (e >= pre[64]) return;
  const int i = rw * 64 + lo;
  const uint2 q = s_rect[i];
  const uint32_t j = e - pre[lo];
  const uint32_t qx0 = q.x & 0xFFFFu, w = (q.x >> 16) - qx0;
  // row = j / w as a multiply-high by the rank's magic ceil(2^32 / w) (0 for
  // w = 1): exact for j, w < 2^16, which the tables' LDS bound guarantees
  const uint32_t mg = s_magic[i];
  const uint32_t rr = __umulhi(j, mg) + (mg == 0u ? j : 0u);
  const int tx = static_cast<int>(qx0 + (j - rr * w));
  const int ty = static_cast<int>((q.y & 0xFFFFu) + rr);
  const int t = ty * tiles_x + tx;
  // the group's ranks on the tile, per rank-wave; earlier ones: whole earlier
  // rank-waves, then the lanes below lo of this one; later ones decide "last"
  unsigned long long m[4];
#pragma unroll
  for (int w2 = 0; w2 < 4; ++w2) m[w2] = s_dyn[w2 * edge + tx] & s_dyn[w2 * edge + tiles_x + ty];
  const unsigned long long below = (1ull << lo) - 1ull, above = ~(below | (1ull << lo));
  uint32_t within;
  unsigned long long later;
  switch (rw) {
    case 0:
      within = __popcll(m[0] & below);
      later = (m[0] & above) | m[1] | m[2] | m[3];
      break;
    case 1:
      within = __popcll(m[0]) + __popcll(m[1] & below);
      later = (m[1] & above) | m[2] | m[3];
      break;
    case 2:
      within = __popcll(m[0]) + __popcll(m[1]) + __popcll(m[2] & below);
      later = (m[2] & above) | m[3];
      break;
    default:
      within = __popcll(m[0]) + __popcll(m[1]) + __popcll(m[2]) + __popcll(m[3] & below);
      later = m[3] & above;
      break;
  }
  const uint32_t p = s_pos[t] + within;
  if (p < capacity) {
    // the rank's tile rectangle clipped to super tile (tx, ty), in its frame
    const uint2 f = s_frect[i];
    const uint32_t bx = static_cast<uint32_t>(tx) << kSuperShift, by = static_cast<uint32_t>(ty) << kSuperShift;
    const uint32_t lx0 = max(f.x & 0xFFFFu, bx) - bx, lxe = min(f.x >> 16, bx + kSuper) - bx;
    const uint32_t ly0 = max(f.y & 0xFFFFu, by) - by, lye = min(f.y >> 16, by + kSuper) - by;
    const uint32_t lr = lx0 | (lxe << 4) | (ly0 << 8) | (lye << 12);
    coarse[p] = static_cast<unsigned long long>(s_gid[i]) | (static_cast<unsigned long long>(lr) << 32);
  }
  if (later == 0ull) s_delta[t] = static_cast<uint16_t>(within + 1u);   // at most 256
}

// A workgroup barrier that orders LDS only: the waves' outstanding global
// stores need not drain before it (nothing in the workgroup reads them).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Coarse emission over the sx x sy super tiles (tiles_x, tiles_y below).
// Groups of 256 ranks.  Waves 0-3 hold the group's ranks (64 each, a
// rank-wave), loaded while the group before was placed, and build their
// coverage masks; then the group's runs of 64 entries (rank-wave 0's, then
// 1's, ...) are dealt to waves 4-15 in turn, so that a rank-wave with many
// entries does not hold up the group, while waves 0-3 load the next group
// (they store nothing to global memory, so their loads wait for no stores).  An entry
// finds its rank from the 64 entry offsets of its rank-wave (run_owner), its
// super tile from the rank's rectangle, and its position as the super tile's
// position at the start of the group plus the count of the group's earlier
// ranks on it.  The entry of the super tile's last rank in the group also
// writes the group's count into delta[t], which one pass over the super
// tiles adds to the positions once every entry of the group is placed.
// two workgroups per CU (8 waves per SIMD): at most 64 VGPRs
__global__ __launch_bounds__(kDirectThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_emit_coarse(const uint32_t* __restrict__ bounds,
                                                                const uint32_t* __restrict__ order,
                                                                const uint2* __restrict__ rect_rank,
                                                                const uint32_t* __restrict__ table,
                                                                const uint32_t* __restrict__ start, int tiles_x,
                                                                int tiles_y, unsigned long long* __restrict__ coarse,
                                                                uint32_t capacity) {
  // dynamic: col[4][tiles_x] row[4][tiles_y] (u64), then pos[ntiles] (u32), delta[ntiles] (u16)
  extern __shared__ unsigned long long s_dyn[];
  __shared__ uint32_t s_pre[4][65];   // per rank-wave: exclusive entry offsets, then the total
  __shared__ uint32_t s_gid[256];
  __shared__ uint2 s_rect[256];
  __shared__ uint2 s_frect[256];
  __shared__ uint32_t s_magic[256];   // ceil(2^32 / rectangle width), 0 for width 1
  __shared__ uint32_t s_mark[kDirectWaves][64];   // per wave: run_owner's scratch
  const int ntiles = tiles_x * tiles_y;
  const int edge = tiles_x + tiles_y;
  uint32_t* const s_pos = reinterpret_cast<uint32_t*>(s_dyn + 4 * edge);
  uint16_t* const s_delta = reinterpret_cast<uint16_t*>(s_pos + ntiles);
  const int c = blockIdx.x, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wave_u = __builtin_amdgcn_readfirstlane(wave);
  const uint32_t R0 = bounds[c], R1 = bounds[c + 1];
  if (R0 >= R1) return;
  const uint32_t* const tab = table + static_cast<size_t>(c) * ntiles;
  for (int t = tid; t < ntiles; t += kDirectThreads) {
    s_pos[t] = start[t] + tab[t];
    s_delta[t] = 0;
  }
  // the next group's ranks, loaded at a clamped index with no condition (so
  // that no branch hides the count of loads in flight: the first use waits
  // for these only) and masked at that use
  uint2 nfr = make_uint2(0u, 0u);
  uint32_t ngid = 0u;
  if (wave < 4) {
    const uint32_t rl = min(R0 + static_cast<uint32_t>(tid), R1 - 1u);
    nfr = rect_rank[rl];
    ngid = order[rl];
  }
  for (uint32_t r0 = R0; r0 < R1; r0 += 256) {
    lds_barrier();   // positions updated, masks of the previous group no longer read
    if (wave < 4) {
      const bool valid = r0 + static_cast<uint32_t>(tid) < R1;
      const uint2 fr = valid ? nfr : make_uint2(0u, 0u);   // (0, 0) past the chunk: no entries
      const uint32_t gid = valid ? ngid : 0u;
      const uint32_t rl = min(r0 + 256u + static_cast<uint32_t>(tid), R1 - 1u);
      nfr = rect_rank[rl];
      ngid = order[rl];
      const uint2 rc = rect_at(fr, kSuperShift);
      const uint32_t cnt = rect_count(rc);
      s_rect[tid] = rc;
      s_frect[tid] = fr;
      s_gid[tid] = gid;
      const uint32_t wd = (rc.x >> 16) - (rc.x & 0xFFFFu);
      s_magic[tid] = wd >= 2u ? 0xFFFFFFFFu / wd + 1u : 0u;
      uint32_t incl = cnt;
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(incl, d, 64);
        if (lane >= d) incl += t;
      }
      s_pre[wave][lane] = incl - cnt;
      if (lane == 63) s_pre[wave][64] = incl;
      // this wave's coverage masks: zero, then set -- per lane over its own
      // columns and rows, or by ballots over the wave's joint extent,
      // whichever takes fewer steps
      unsigned long long* const col = s_dyn + wave * edge;
      unsigned long long* const row = col + tiles_x;
      for (int i = lane; i < edge; i += 64) col[i] = 0ull;
      const int x0 = static_cast<int>(rc.x & 0xFFFFu), xe = static_cast<int>(rc.x >> 16);
      const int y0 = static_cast<int>(rc.y & 0xFFFFu), ye = static_cast<int>(rc.y >> 16);
      const bool has = cnt > 0;
      int own = has ? (xe - x0) + (ye - y0) : 0;
      int xmin = has ? x0 : tiles_x, xmax = has ? xe : 0, ymin = has ? y0 : tiles_y, ymax = has ? ye : 0;
      for (int o = 32; o > 0; o >>= 1) {
        own = max(own, __shfl_xor(own, o, 64));
        xmin = min(xmin, __shfl_xor(xmin, o, 64));
        xmax = max(xmax, __shfl_xor(xmax, o, 64));
        ymin = min(ymin, __shfl_xor(ymin, o, 64));
        ymax = max(ymax, __shfl_xor(ymax, o, 64));
      }
      const unsigned long long bit = 1ull << lane;
      if (own <= max(xmax - xmin, 0) + max(ymax - ymin, 0)) {
        if (has) {
          for (int x = x0; x < xe; ++x) atomicOr(&col[x], bit);
          for (int y = y0; y < ye; ++y) atomicOr(&row[y], bit);
        }
      } else {
        for (int x = xmin; x < xmax; ++x) {
          const unsigned long long m = __ballot(has && x0 <= x && x < xe);
          if (lane == 0) col[x] = m;
        }
        for (int y = ymin; y < ymax; ++y) {
          const unsigned long long m = __ballot(has && y0 <= y && y < ye);
          if (lane == 0) row[y] = m;
        }
      }
    }
    lds_barrier();
    // place the group's entries: the runs of 64 entries of rank-waves 0..3 in
    // turn, dealt to waves 4-15 round-robin (a run's rank-wave is uniform
    // over the wave)
    if (wave_u >= 4) {
      const uint32_t c1 = __builtin_amdgcn_readfirstlane((s_pre[0][64] + 63u) >> 6);
      const uint32_t c2 = c1 + __builtin_amdgcn_readfirstlane((s_pre[1][64] + 63u) >> 6);
      const uint32_t c3 = c2 + __builtin_amdgcn_readfirstlane((s_pre[2][64] + 63u) >> 6);
      const uint32_t nrun = c3 + __builtin_amdgcn_readfirstlane((s_pre[3][64] + 63u) >> 6);
      for (uint32_t run = static_cast<uint32_t>(wave_u - 4); run < nrun; run += kDirectWaves - 4) {
        const int rw = run < c1 ? 0 : (run < c2 ? 1 : (run < c3 ? 2 : 3));
        const uint32_t first = run < c1 ? 0u : (run < c2 ? c1 : (run < c3 ? c2 : c3));
        const uint32_t e0 = (run - first) * 64u;
        const int lo = run_owner(s_pre[rw], e0, s_mark[wave_u], lane);
        place_entry(rw, e0 + lane, lo, s_pre[rw], s_rect, s_frect, s_magic, s_gid, s_dyn, s_pos, s_delta, edge,
                    tiles_x, coarse, capacity);
      }
    }
    lds_barrier();
    for (int t = tid; t < ntiles; t += kDirectThreads) {
      const uint32_t d = s_delta[t];
      if (d) { s_pos[t] += d; s_delta[t] = 0; }
    }
  }
}

// Fine passes.  A coarse entry packs the Gaussian (low word) and its
// rectangle within the super tile (high word: x0 | x_end << 4 | y0 << 8 |
// y_end << 12, ends exclusive, all in 0..8).  For a wave's 64 entries (lane e
// holds entry e, 0 for none) col[x] is the mask of entries spanning column x
// of the super tile and row[y] of those spanning row y: the entries on tile
// (x, y) are col[x] & row[y].
struct FineMasks {
  uint64_t col[kSuper], row[kSuper];
};
// (Each mask is the AND of two compare ballots: a ballot of the combined
// bool would first turn it into an integer and back.)
__device__ __forceinline__ void fine_masks(uint32_t lr, FineMasks& m) {
  const uint32_t x0 = lr & 15u, xe = (lr >> 4) & 15u, y0 = (lr >> 8) & 15u, ye = (lr >> 12) & 15u;
#pragma unroll
  for (int k = 0; k < kSuper; ++k) {
    const uint32_t u = static_cast<uint32_t>(k);
    m.col[k] = __builtin_amdgcn_ballot_w64(x0 <= u) & __builtin_amdgcn_ballot_w64(u < xe);
    m.row[k] = __builtin_amdgcn_ballot_w64(y0 <= u) & __builtin_amdgcn_ballot_w64(u < ye);
  }
}
// Lane t's tile (t & 7, t >> 3): the mask of the wave's entries covering it.
__device__ __forceinline__ uint64_t fine_tile_mask(const FineMasks& m, int lane) {
  uint64_t c = m.col[0], r = m.row[0];
#pragma unroll
  for (int k = 1; k < kSuper; ++k) {
    c = (lane & (kSuper - 1)) == k ? m.col[k] : c;
    r = (lane >> kSuperShift) == k ? m.row[k] : r;
  }
  return c & r;
}

// The fine passes' part p: its super tile (the last s with pbase[s] <= p,
// from the part bases in LDS) and its coarse entries [lo, hi).
struct Part {
  uint32_t s, lo, hi;
};
__device__ __forceinline__ Part find_part(const uint32_t* __restrict__ s_pb, int ns, uint32_t p,
                                          const uint32_t* __restrict__ cstart, const uint32_t* __restrict__ ctotal) {
  int a = 0, b = ns - 1;
  while (a < b) {
    const int mid = (a + b + 1) >> 1;
    if (s_pb[mid] <= p) a = mid; else b = mid - 1;
  }
  const uint32_t s = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(a));
  const uint32_t base = cstart[s], lo = base + (p - s_pb[s]) * static_cast<uint32_t>(kPart);
  return Part{s, lo, min(lo + static_cast<uint32_t>(kPart), base + ctotal[s])};
}

// A part's coarse entries, kPartSteps per thread: step j of wave w holds
// entries lo + 256 j + 64 w + lane (0 past hi), all loads in flight at once.
__device__ __forceinline__ void load_part(const unsigned long long* __restrict__ coarse, const Part& pt, int wave,
                                          int lane, unsigned long long (&v)[kPartSteps]) {
#pragma unroll
  for (int j = 0; j < kPartSteps; ++j) {
    const uint32_t e = pt.lo + static_cast<uint32_t>(j * kFineThreads + wave * 64 + lane);
    v[j] = e < pt.hi ? coarse[e] : 0ull;
  }
}

// Per part p: ftab[p][t] = the entries of its super tile's tile t in the
// part.  The workgroups loop over the parts.
__global__ __launch_bounds__(kFineThreads) void k_fine_count(const uint32_t* __restrict__ pbase, int ns,
                                                             const uint32_t* __restrict__ cstart,
                                                             const uint32_t* __restrict__ ctotal,
                                                             const unsigned long long* __restrict__ coarse,
                                                             uint32_t* __restrict__ ftab) {
  extern __shared__ uint32_t s_pb[];   // pbase[0..ns]
  __shared__ uint32_t s_sum[kFineWaves][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i = threadIdx.x; i <= ns; i += kFineThreads) s_pb[i] = pbase[i];
  __syncthreads();
  const uint32_t np = s_pb[ns];
  for (uint32_t p = blockIdx.x; p < np; p += gridDim.x) {
    const Part pt = find_part(s_pb, ns, p, cstart, ctotal);
    unsigned long long v[kPartSteps];
    load_part(coarse, pt, wave, lane, v);
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < kPartSteps; ++j) {
      FineMasks m;
      fine_masks(static_cast<uint32_t>(v[j] >> 32), m);
      acc += static_cast<uint32_t>(__popcll(fine_tile_mask(m, lane)));
    }
    s_sum[wave][lane] = acc;
    __syncthreads();
    if (wave == 0) {
      uint32_t t = 0;
#pragma unroll
      for (int w = 0; w < kFineWaves; ++w) t += s_sum[w][lane];
      ftab[static_cast<size_t>(p) * 64 + lane] = t;
    }
    __syncthreads();
  }
}

// Per super tile s (one workgroup): the counts ftab[p][t] of its parts become
// exclusive prefixes over the parts, and each tile's total goes to total[]
// (lanes of tiles outside the frame write nothing).  Wave w takes a quarter
// of the parts, lane t the tile; the rows are read kScanBatch at a time, all
// loads in flight together.
constexpr int kScanBatch = 8;
__global__ __launch_bounds__(256) void k_fine_scan(const uint32_t* __restrict__ pbase, uint32_t* __restrict__ ftab,
                                                   int sx, int tiles_x, int tiles_y, uint32_t* __restrict__ total) {
  __shared__ uint32_t s_sum[4][64];
  const int s = blockIdx.x, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t p0 = pbase[s], p1 = pbase[s + 1];
  const uint32_t per = (p1 - p0 + 3u) / 4u;
  const uint32_t a = min(p1, p0 + static_cast<uint32_t>(wave) * per), b = min(p1, a + per);
  uint32_t* const col = ftab + lane;
  uint32_t sum = 0;
  for (uint32_t p = a; p < b; p += kScanBatch) {
    uint32_t x[kScanBatch];
#pragma unroll
    for (int k = 0; k < kScanBatch; ++k) x[k] = p + k < b ? col[static_cast<size_t>(p + k) * 64] : 0u;
#pragma unroll
    for (int k = 0; k < kScanBatch; ++k) sum += x[k];
  }
  s_sum[wave][lane] = sum;
  __syncthreads();
  uint32_t run = 0, all = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const uint32_t x = s_sum[w][lane];
    run += (w < wave) ? x : 0u;
    all += x;
  }
  for (uint32_t p = a; p < b; p += kScanBatch) {
    uint32_t x[kScanBatch];
#pragma unroll
    for (int k = 0; k < kScanBatch; ++k) x[k] = p + k < b ? col[static_cast<size_t>(p + k) * 64] : 0u;
#pragma unroll
    for (int k = 0; k < kScanBatch; ++k) {
      if (p + k < b) col[static_cast<size_t>(p + k) * 64] = run;
      run += x[k];
    }
  }
  if (wave == 0) {
    const int tx = (s % sx) * kSuper + (lane & (kSuper - 1)), ty = (s / sx) * kSuper + (lane >> kSuperShift);
    if (tx < tiles_x && ty < tiles_y) total[ty * tiles_x + tx] = all;
  }
}

// Per part p: the point_list entries of its coarse entries.  Lane t of every
// wave keeps tile t's next position (pos); per step of 256 entries each wave
// counts its entries per tile, the counts of the earlier waves give its
// offsets, and then the 64 tiles go out in turn, one store each (exec = the
// tile's mask).  Nothing is written unless every entry fits (*fits, from
// k_tile_starts): then every position is below K <= capacity.
__global__ __launch_bounds__(kFineThreads) void k_fine_emit(const uint32_t* __restrict__ pbase, int ns,
                                                            const uint32_t* __restrict__ cstart,
                                                            const uint32_t* __restrict__ ctotal,
                                                            const unsigned long long* __restrict__ coarse,
                                                            const uint32_t* __restrict__ ftab,
                                                            const uint32_t* __restrict__ start, int sx, int tiles_x,
                                                            int tiles_y, const uint32_t* __restrict__ fits,
                                                            uint32_t* __restrict__ point_list) {
  extern __shared__ uint32_t s_pb[];   // pbase[0..ns]
  __shared__ uint32_t s_cnt[2][kFineWaves][64];   // two steps in flight: one barrier per step
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (*fits == 0u) return;
  for (int i = threadIdx.x; i <= ns; i += kFineThreads) s_pb[i] = pbase[i];
  __syncthreads();
  const uint32_t np = s_pb[ns];
  int buf = 0;
  for (uint32_t p = blockIdx.x; p < np; p += gridDim.x) {
    const Part pt = find_part(s_pb, ns, p, cstart, ctotal);
    unsigned long long v[kPartSteps];
    load_part(coarse, pt, wave, lane, v);
    const int tx = static_cast<int>(pt.s % static_cast<uint32_t>(sx)) * kSuper + (lane & (kSuper - 1));
    const int ty = static_cast<int>(pt.s / static_cast<uint32_t>(sx)) * kSuper + (lane >> kSuperShift);
    uint32_t pos = (tx < tiles_x && ty < tiles_y) ? start[ty * tiles_x + tx] + ftab[static_cast<size_t>(p) * 64 + lane]
                                                  : 0u;
    const int steps = static_cast<int>((pt.hi - pt.lo + kFineThreads - 1) / kFineThreads);
#pragma unroll 1
    for (int j = 0; j < steps; ++j) {
      const unsigned long long e = v[0];
#pragma unroll
      for (int k = 0; k + 1 < kPartSteps; ++k) v[k] = v[k + 1];
      const uint32_t gid = static_cast<uint32_t>(e);
      FineMasks m;
      fine_masks(static_cast<uint32_t>(e >> 32), m);
      s_cnt[buf][wave][lane] = static_cast<uint32_t>(__popcll(fine_tile_mask(m, lane)));
      lds_barrier();
      uint32_t before = pos, all = 0;
#pragma unroll
      for (int w = 0; w < kFineWaves; ++w) {
        const uint32_t c = s_cnt[buf][w][lane];
        before += (w < wave) ? c : 0u;
        all += c;
      }
      pos += all;
      buf ^= 1;
#pragma unroll
      for (int t = 0; t < 64; ++t) {
        const uint64_t M = m.col[t & (kSuper - 1)] & m.row[t >> kSuperShift];
        if (M == 0ull) continue;
        const uint32_t bt = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(before), t));
        if (__builtin_amdgcn_inverse_ballot_w64(M))
          point_list[bt + __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(M >> 32),
                                                    __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(M), 0u))] = gid;
      }
    }
  }
}

static int bits_for(int64_t values) {  // bits needed to represent 0..values-1
  int b = 0;
  while ((int64_t(1) << b) < values) ++b;
  return b < 1 ? 1 : b;
}

struct BinWs {
  uint32_t *dk0, *dv0, *dk1, *dv1, *order, *cnt, *offs;
  uint2 *rect, *rect_rank;
  uint32_t *ek0, *ek1, *ev1;      // radix tile sort (no direct emission)
  uint32_t* hist;
  ScanWs scan;
  OsWs os;                        // depth sort state
  uint32_t* zero;                 // its digit counts, K, the error flag and kfine, cleared by k_depth_keys
  unsigned long long* readback;   // [0] K, [1] the error flag
  unsigned long long* kfine;      // direct emission: the tile counts' sum
  // direct emission: chunk bounds, chunk x super-tile table, super-tile
  // totals and starts, tile totals and starts, the parts, per part x tile
  // counts, and the coarse list
  uint32_t *bounds, *table, *ctotal, *cstart, *total, *start;
  uint32_t *pbase, *ftab, *fits;
  unsigned long long* coarse;
};

constexpr int kZeroWords = kOsMaxPasses * 256 + 6;   // digit counts, K, error flag, kfine

static BinWs carve_bin(void* ws, int64_t n, int64_t cap, int tiles_x, int tiles_y, size_t* used) {
  Carver c(ws);
  BinWs b{};
  const size_t N = static_cast<size_t>(n > 0 ? n : 1), C = static_cast<size_t>(cap > 0 ? cap : 1);
  const bool direct = direct_ok(tiles_x, tiles_y);
  b.dk0 = c.take<uint32_t>(N); b.dv0 = c.take<uint32_t>(N);
  b.dk1 = c.take<uint32_t>(N); b.dv1 = c.take<uint32_t>(N);
  b.order = c.take<uint32_t>(N);
  b.cnt = c.take<uint32_t>(N); b.offs = c.take<uint32_t>(N);
  b.rect = c.take<uint2>(N); b.rect_rank = c.take<uint2>(N);
  if (direct) {
    b.scan.sums = c.take<uint32_t>(scan_ws_words(static_cast<int64_t>(N)));
  } else {
    b.ek0 = c.take<uint32_t>(C); b.ek1 = c.take<uint32_t>(C); b.ev1 = c.take<uint32_t>(C);
    const size_t hist_words = 256 * static_cast<size_t>(ceil_div(std::max<int64_t>(cap, 1), kRsThreads * kRsItemsK));
    const int64_t maxn = std::max<int64_t>(std::max<int64_t>(n, cap), 1);
    b.hist = c.take<uint32_t>(hist_words);
    b.scan.sums = c.take<uint32_t>(scan_ws_words(std::max<int64_t>(static_cast<int64_t>(hist_words), maxn)));
  }
  // cleared by k_depth_keys: the onesweep digit counts, then K, the error flag and kfine
  b.zero = c.take<uint32_t>(kZeroWords);
  b.readback = reinterpret_cast<unsigned long long*>(b.zero + kOsMaxPasses * 256);
  b.kfine = b.readback + 2;
  b.scan.total = b.readback;
  b.os.ghist = b.zero;
  b.os.err = reinterpret_cast<uint32_t*>(b.readback + 1);
  b.os.state = c.take<uint32_t>(os_state_words(n, kOsThreads * kOsItemsN, kOsMaxPasses));
  b.os.counters = c.take<uint32_t>(kOsMaxPasses);
  if (direct) {
    const size_t nt = static_cast<size_t>(tiles_x) * tiles_y;
    const int ns = super_dim(tiles_x) * super_dim(tiles_y);
    const size_t chunks = static_cast<size_t>(direct_max_chunks(cap));
    const size_t parts = static_cast<size_t>(direct_max_parts(cap, ns));
    b.bounds = c.take<uint32_t>(chunks + 1);
    b.table = c.take<uint32_t>(chunks * ns);
    b.ctotal = c.take<uint32_t>(ns);
    b.cstart = c.take<uint32_t>(ns);
    b.total = c.take<uint32_t>(nt);
    b.start = c.take<uint32_t>(nt);
    b.pbase = c.take<uint32_t>(ns + 1);
    b.fits = c.take<uint32_t>(1);
    b.ftab = c.take<uint32_t>(parts * 64);
    b.coarse = c.take<unsigned long long>(C);
  }
  *used = c.off + 256;
  return b;
}

size_t binsort_workspace(int64_t n, int64_t capacity, int tiles_x, int tiles_y) {
  size_t used = 0;
  carve_bin(nullptr, n, capacity, tiles_x, tiles_y, &used);
  return used;
}

bool binsort_direct(int tiles_x, int tiles_y) { return direct_ok(tiles_x, tiles_y); }

__global__ void k_put_zero_k(unsigned long long* __restrict__ k_dev) {
  if (threadIdx.x < 2) k_dev[threadIdx.x] = 0ull;
}

gs_status run_bin_sort(int64_t n64, const gs_projected& proj, const DevCam& cam, void* ws, size_t ws_bytes,
                       uint32_t* point_list, int64_t capacity, uint32_t* ranges, int64_t* k_out,
                       unsigned long long* k_dev, hipStream_t s) {
  const int n = static_cast<int>(n64);
  const int ntiles = cam.tiles_x * cam.tiles_y;
  size_t need = 0;
  BinWs b = carve_bin(ws, n64, capacity, cam.tiles_x, cam.tiles_y, &need);
  if (ws_bytes < need) return fail(GS_ERR_INVALID_ARG, "gs_bin_sort: workspace too small");
  gs_status st;
  int64_t K = 0;
  if (n > 0) {
    const unsigned g = static_cast<unsigned>(ceil_div(n, 256));
    { TimedLaunch gs_tl("k_depth_keys", s); k_depth_keys<<<g, 256, 0, s>>>(n, proj.depth, reinterpret_cast<const float4*>(proj.records), proj.radius,
                                   cam.tiles_x, cam.tiles_y, b.dk0, b.dv0, b.rect, b.zero, kZeroWords); }
    if ((st = check_launch("k_depth_keys")) != GS_OK) return st;
    // the terminal pass also gathers each rank's rectangle and its count of
    // super tiles (direct emission) or tiles
    if ((st = onesweep_sort_pairs<kOsItemsN, kOsThreads>(b.dk0, b.dv0, b.dk1, b.dv1, n, 32, b.os, s, b.order, b.rect,
                                             b.rect_rank, b.cnt, b.table ? kSuperShift : 0)) != GS_OK)
      return st;
    const uint32_t* order = b.order;
    unsigned long long rb[2] = {0ull, 0ull};
    if (b.table) {
      // direct emission, sized on the device from the scanned coarse total:
      // no host wait between the depth sort and the placement; K (and the
      // look-back flag) are read once at the end
      const int tx = cam.tiles_x, ty = cam.tiles_y;
      const int sx = super_dim(tx), sy = super_dim(ty), ns = sx * sy;
      const int cmax = static_cast<int>(direct_max_chunks(capacity));
      const unsigned fgrid = static_cast<unsigned>(std::min<int64_t>(direct_max_parts(capacity, ns), kFineGrid));
      const uint32_t cap32 = static_cast<uint32_t>(std::min<int64_t>(capacity, UINT32_MAX));
      if ((st = device_chunk_bounds(b.cnt, n, b.scan,
                                    ChunkArgs{b.bounds, cmax, static_cast<unsigned long long>(kDirectMinEntries),
                                              static_cast<unsigned long long>(kDirectChunks), k_dev},
                                    s)) != GS_OK)
        return st;
      { TimedLaunch gs_tl("k_chunk_count", s); k_chunk_count<<<cmax, kDirectThreads, sizeof(int) * (sx + 1) * (sy + 1), s>>>(
          b.bounds, b.rect_rank, sx, sy, b.table, b.kfine); }
      if ((st = check_launch("k_chunk_count")) != GS_OK) return st;
      { TimedLaunch gs_tl("k_chunk_colscan", s); k_chunk_colscan<<<static_cast<unsigned>(ceil_div(ns, 64)), 1024, 0, s>>>(cmax, ns, b.table, b.ctotal); }
      if ((st = check_launch("k_chunk_colscan")) != GS_OK) return st;
      { TimedLaunch gs_tl("k_coarse_parts", s); k_coarse_parts<<<1, 1024, 0, s>>>(ns, b.ctotal, b.cstart, static_cast<unsigned long long>(capacity),
                                                                                  b.pbase); }
      if ((st = check_launch("k_coarse_parts")) != GS_OK) return st;
      { TimedLaunch gs_tl("k_emit_coarse", s); k_emit_coarse<<<cmax, kDirectThreads, emit_dyn_lds(sx, sy), s>>>(
          b.bounds, order, b.rect_rank, b.table, b.cstart, sx, sy, b.coarse, cap32); }
      if ((st = check_launch("k_emit_coarse")) != GS_OK) return st;
      const size_t pb_lds = sizeof(uint32_t) * (static_cast<size_t>(ns) + 1);
      { TimedLaunch gs_tl("k_fine_count", s); k_fine_count<<<fgrid, kFineThreads, pb_lds, s>>>(b.pbase, ns, b.cstart, b.ctotal, b.coarse, b.ftab); }
      if ((st = check_launch("k_fine_count")) != GS_OK) return st;
      { TimedLaunch gs_tl("k_fine_scan", s); k_fine_scan<<<ns, 256, 0, s>>>(b.pbase, b.ftab, sx, tx, ty, b.total); }
      if ((st = check_launch("k_fine_scan")) != GS_OK) return st;
      const StartArgs sa{ntiles, b.start, reinterpret_cast<uint2*>(ranges), static_cast<unsigned long long>(capacity),
                         b.kfine, b.readback, k_dev, b.fits};
      { TimedLaunch gs_tl("k_tile_starts", s); k_tile_starts<<<1, 1024, 0, s>>>(b.total, sa); }
      if ((st = check_launch("k_tile_starts")) != GS_OK) return st;
      { TimedLaunch gs_tl("k_fine_emit", s); k_fine_emit<<<fgrid, kFineThreads, pb_lds, s>>>(
          b.pbase, ns, b.cstart, b.ctotal, b.coarse, b.ftab, b.start, sx, tx, ty, b.fits, point_list); }
      if ((st = check_launch("k_fine_emit")) != GS_OK) return st;
      if (k_dev) return GS_OK;   // the caller checks K and the flag later
    } else if ((st = device_exclusive_scan(b.cnt, b.offs, n, b.scan, s)) != GS_OK) {
      return st;
    }
    if ((st = check_hip(hipMemcpyAsync(rb, b.readback, sizeof(rb), hipMemcpyDeviceToHost, s),
                        "hipMemcpyAsync(K)")) != GS_OK) return st;
    if ((st = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize")) != GS_OK) return st;
    if (static_cast<uint32_t>(rb[1]) != 0u)
      return fail(GS_ERR_HIP, "gs_bin_sort: depth sort look-back did not complete (spin limit)");
    K = static_cast<int64_t>(rb[0]);
    *k_out = K;
    if (K >= (int64_t(1) << 32)) return fail(GS_ERR_UNSUPPORTED, "gs_bin_sort: more than 2^32 entries");
    if (K > capacity) return fail(GS_ERR_CAPACITY, "gs_bin_sort: capacity too small");
    if (b.table) return GS_OK;
    if (K > 0) {
      const int tbits = bits_for(ntiles);
      const int tp = sort_passes(tbits);
      // choose the emit target so that the last pass lands in point_list
      uint32_t* ka = b.ek0;
      uint32_t* va = (tp % 2 == 0) ? point_list : b.ev1;
      uint32_t* kb = b.ek1;
      uint32_t* vb = (tp % 2 == 0) ? b.ev1 : point_list;
      { TimedLaunch gs_tl("k_emit", s); k_emit<<<static_cast<unsigned>(ceil_div(n, 256)), 256, 0, s>>>(
          n, order, b.offs, b.rect_rank, cam.tiles_x, ka, va); }
      if ((st = check_launch("k_emit")) != GS_OK) return st;
      int p2 = 0;
      if ((st = radix_sort_pairs<kRsItemsK>(ka, va, kb, vb, K, tbits, b.hist, b.scan, s, &p2)) != GS_OK) return st;
      const uint32_t* sorted_tiles = (p2 % 2 == 0) ? ka : kb;
      { TimedLaunch gs_tl("k_ranges", s); k_ranges<<<static_cast<unsigned>(ceil_div(ntiles, 256)), 256, 0, s>>>(
          ntiles, sorted_tiles, static_cast<uint32_t>(K), reinterpret_cast<uint2*>(ranges)); }
      return check_launch("k_ranges");
    }
  } else {
    if (k_out) *k_out = 0;
    if (k_dev) {
      { TimedLaunch gs_tl("k_put_zero_k", s); k_put_zero_k<<<1, 64, 0, s>>>(k_dev); }
      if ((st = check_launch("k_put_zero_k")) != GS_OK) return st;
    }
  }
  // K == 0: every tile is empty
  if ((st = check_hip(hipMemsetAsync(ranges, 0, sizeof(uint32_t) * 2 * static_cast<size_t>(ntiles), s),
                      "hipMemsetAsync(ranges)")) != GS_OK) return st;
  return GS_OK;
}

}  // namespace gs
