// Learned colour decoder on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16).
//
// Not part of the paper's method: an optional replacement for the SH colour
// read of the projection (Sec. I / Sec. II-A, colour from SH coefficients).
// Per sample, x = [z (16 latent values); Y_0..15(d)] (the real SH encoding of
// the unit view direction), h1 = ReLU(W1 x + b1), h2 = ReLU(W2 h1 + b2),
// c = sigmoid(W3 h2 + b3); W and z are BF16, every product is accumulated in
// FP32, and the view encoding and hidden activations enter the products as a
// hi + lo pair of BF16 values (about 2^-17 relative), so the colour matches the
// BF16-weight definition to near FP32 accuracy.
//
// A wave evaluates 16 samples at a time.  In the 16x16x32 MFMA, lane l holds
// A[l % 16][8 (l / 16) + e], B[8 (l / 16) + e][l % 16] (e = 0..7) and
// D[4 (l / 16) + i][l % 16] (i = 0..3).  Samples run along the 16 columns, so
// after a layer lane l holds hidden units 16 b + 4 (l / 16) + i of sample
// l % 16.  Read back as the next layer's B operand, slot e of lane l then
// carries hidden unit hid(c, l / 16, e) = 32 c + 16 (e / 4) + 4 (l / 16) + e % 4
// of k-chunk c; the packed weights permute their input columns the same way,
// so activations never leave registers between layers.
#include "gs_internal.h"
#include "gs_sh.h"

namespace gs {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kMlpIn = 32, kMlpH = 64, kMlpOut = 3;
constexpr int P_W1 = 0, P_B1 = 2048, P_W2 = 2112, P_B2 = 6208, P_W3 = 6272, P_B3 = 6464;

// Packed operand image: kOps tiles of 64 lanes x 8 BF16 values, then the
// biases in FP32 (b1[64], b2[64], b3[3]).
//   0..3   W1 row-block b                       (forward, layer 1)
//   4..11  W2 row-block b, k-chunk c (4+2b+c)    (forward, layer 2, permuted k)
//   12..13 W3 (rows 3..15 zero), k-chunk c       (forward, layer 3, permuted k)
//   14..17 W3^T row-block b (k = output unit)    (backward, dL/dh2)
//   18..25 W2^T row-block b, k-chunk c (18+2b+c) (backward, dL/dh1, permuted k)
//   26..29 W1^T row-block b, k-chunk c (26+2b+c) (backward, dL/dx, permuted k)
constexpr int kOps = 30;
constexpr int kOpW1 = 0, kOpW2 = 4, kOpW3 = 12, kOpW3T = 14, kOpW2T = 18, kOpW1T = 26;
constexpr int kBiasFloats = 131;

__host__ __device__ constexpr int hid(int c, int g, int e) { return 32 * c + 16 * (e >> 2) + 4 * g + (e & 3); }

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(static_cast<uint32_t>(b) << 16); }

__device__ __forceinline__ floatx4 mfma(const uint4& a, const bf16x8& b, const floatx4& c) {
  bf16x8 av;
  __builtin_memcpy(&av, &a, sizeof(av));
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b, c, 0, 0, 0);
}

__global__ __launch_bounds__(64) void k_mlp_pack(const uint16_t* __restrict__ P, uint4* __restrict__ ops,
                                                 float* __restrict__ bias) {
  const int op = blockIdx.x, l = threadIdx.x, g = l >> 4, r = l & 15;
  uint16_t v[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    uint16_t x = 0;
    if (op < kOpW2) {
      x = P[P_W1 + (16 * op + r) * kMlpIn + 8 * g + e];
    } else if (op < kOpW3) {
      const int b = (op - kOpW2) >> 1, c = (op - kOpW2) & 1;
      x = P[P_W2 + (16 * b + r) * kMlpH + hid(c, g, e)];
    } else if (op < kOpW3T) {
      const int c = op - kOpW3;
      x = (r < kMlpOut) ? P[P_W3 + r * kMlpH + hid(c, g, e)] : 0;
    } else if (op < kOpW2T) {
      const int b = op - kOpW3T;
      x = (g == 0 && e < kMlpOut) ? P[P_W3 + e * kMlpH + 16 * b + r] : 0;
    } else if (op < kOpW1T) {
      const int b = (op - kOpW2T) >> 1, c = (op - kOpW2T) & 1;
      x = P[P_W2 + hid(c, g, e) * kMlpH + 16 * b + r];
    } else {
      const int b = (op - kOpW1T) >> 1, c = (op - kOpW1T) & 1;
      x = P[P_W1 + hid(c, g, e) * kMlpIn + 16 * b + r];
    }
    v[e] = x;
  }
  uint4 w;
  w.x = v[0] | (static_cast<uint32_t>(v[1]) << 16);
  w.y = v[2] | (static_cast<uint32_t>(v[3]) << 16);
  w.z = v[4] | (static_cast<uint32_t>(v[5]) << 16);
  w.w = v[6] | (static_cast<uint32_t>(v[7]) << 16);
  ops[op * 64 + l] = w;
  if (op == 0) {
    bias[l] = bf2f(P[P_B1 + l]);
    bias[64 + l] = bf2f(P[P_B2 + l]);
    if (l < kMlpOut) bias[128 + l] = bf2f(P[P_B3 + l]);
  }
}

struct MlpShared {
  uint4 ops[kOps * 64];
  float bias[kBiasFloats + 1];
};

__device__ __forceinline__ void load_packed(MlpShared& sh, const uint4* __restrict__ ops,
                                            const float* __restrict__ bias) {
  for (int i = threadIdx.x; i < kOps * 64; i += blockDim.x) sh.ops[i] = ops[i];
  for (int i = threadIdx.x; i < kBiasFloats; i += blockDim.x) sh.bias[i] = bias[i];
}

// A value v carried as two BF16 operands, hi = bf16(v) and lo = bf16(v - hi):
// hi + lo equals v to about 2^-17 relative, so products with the (exactly
// BF16) weights keep activations and the view encoding at close to FP32
// accuracy for twice the matrix-core work, which is not this kernel's bound.
struct Split8 {
  bf16x8 hi, lo;
};

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));

// Two values split at once: one packed conversion for both hi parts, one for
// both lo parts (round to nearest even, as a single conversion would).
struct Split2 {
  bf16x2 hi, lo;
};
__device__ __forceinline__ Split2 split2(float a, float b) {
  const floatx2 v = {a, b};
  Split2 p;
  p.hi = __builtin_convertvector(v, bf16x2);
  p.lo = __builtin_convertvector(v - __builtin_convertvector(p.hi, floatx2), bf16x2);
  return p;
}

// slots e, e + 1 (e even) of s
__device__ __forceinline__ void split_put2(Split8& s, int e, float a, float b) {
  const Split2 p = split2(a, b);
  s.hi[e] = p.hi[0]; s.hi[e + 1] = p.hi[1];
  s.lo[e] = p.lo[0]; s.lo[e + 1] = p.lo[1];
}

// Read a D-layout pre-activation (4 row-blocks, bias included) back as the
// split B operands of the next layer, after the ReLU.
__device__ __forceinline__ void relu_to_b(const floatx4 h[4], Split8& B0, Split8& B1) {
#pragma unroll
  for (int e = 0; e < 8; e += 2) {
    const int b0 = e >> 2, i = e & 3;
    split_put2(B0, e, fmaxf(h[b0][i], 0.0f), fmaxf(h[b0][i + 1], 0.0f));
    split_put2(B1, e, fmaxf(h[2 + b0][i], 0.0f), fmaxf(h[2 + b0][i + 1], 0.0f));
  }
}

// The biases of a hidden layer in the D layout of row-block b: lane (g, r)
// holds rows 4 g .. 4 g + 3, i.e. units 16 b + 4 g + i -- the accumulator a
// layer's products start from, so the pre-activation needs no separate add.
__device__ __forceinline__ floatx4 bias_d(const float* bias, int b, int g) {
  return *reinterpret_cast<const floatx4*>(bias + 16 * b + 4 * g);
}

// Layer-1 B operand of lane (g, sample s): latent values 8g..8g+7 (g < 2,
// exact BF16, lo = 0) or the SH encoding values 8(g-2)..8(g-2)+7 of the view
// direction (g >= 2).
__device__ __forceinline__ Split8 input_operand(int g, bool valid, const uint4& zslice, const float d[3]) {
  Split8 X;
  if (g < 2) {
    const uint4 raw = valid ? zslice : make_uint4(0, 0, 0, 0);
    __builtin_memcpy(&X.hi, &raw, sizeof(X.hi));
#pragma unroll
    for (int e = 0; e < 8; ++e) X.lo[e] = static_cast<__bf16>(0.0f);
  } else {
    float Y[16];
    sh_basis(3, d[0], d[1], d[2], Y);
    // static indices (a lane-dependent index into Y would become a select chain)
    const bool upper = g == 3;
#pragma unroll
    for (int e = 0; e < 8; e += 2)
      split_put2(X, e, valid ? (upper ? Y[8 + e] : Y[e]) : 0.0f, valid ? (upper ? Y[9 + e] : Y[e + 1]) : 0.0f);
  }
  return X;
}

struct MlpFwdState {
  floatx4 h1[4], h2[4], o;
  Split8 X, B0, B1, C0, C1;
};

__device__ __forceinline__ floatx4 mfma2(const uint4& a, const Split8& b, const floatx4& c) {
  return mfma(a, b.lo, mfma(a, b.hi, c));
}

// h1, h2: pre-activations (biases included); B, C: the split ReLU outputs.
__device__ __forceinline__ void mlp_forward_group(const MlpShared& sh, int lane, MlpFwdState& st) {
  const int g = lane >> 4;
  const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int b = 0; b < 4; ++b) st.h1[b] = mfma2(sh.ops[(kOpW1 + b) * 64 + lane], st.X, bias_d(sh.bias, b, g));
  relu_to_b(st.h1, st.B0, st.B1);
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    floatx4 acc = mfma2(sh.ops[(kOpW2 + 2 * b) * 64 + lane], st.B0, bias_d(sh.bias + 64, b, g));
    st.h2[b] = mfma2(sh.ops[(kOpW2 + 2 * b + 1) * 64 + lane], st.B1, acc);
  }
  relu_to_b(st.h2, st.C0, st.C1);
  floatx4 acc = mfma2(sh.ops[kOpW3 * 64 + lane], st.C0, zero);
  st.o = mfma2(sh.ops[(kOpW3 + 1) * 64 + lane], st.C1, acc);
}

// The hardware reciprocal (1 ulp) instead of a correctly rounded division:
// the colour's error budget is set by the BF16 products, far above it.
__device__ __forceinline__ float sigmoidf(float x) { return __builtin_amdgcn_rcpf(1.0f + __expf(-x)); }

// Inputs of one lane's sample.  The kernels load them one group ahead, so
// their latency hides behind the current group's arithmetic (a wave runs
// many groups in turn and few waves share a SIMD).
struct SampleIn {
  float a[3];       // unit direction (MODE 0) or the Gaussian's mean (MODE 1)
  float c[3];       // backward: dL/dc or the distillation target (quarter 0)
  uint4 z;          // latent values 8 g .. 8 g + 7 (quarters 0, 1)
  float m[3];       // MODE 1 backward: dL/dmean so far (the geometry's share)
  bool in;          // s < S (and, MODE 1, the Gaussian is live)
};

// dL_dc: channel i of sample s at dL_dc[(c0 + i) cs + s ss] -- MODE 0 [S][3]
// (c0 0, cs 1, ss 3); MODE 1 g2d[9][S] (c0 6, cs S, ss 1) or accumulator rows
// [S][kAccStride] (c0 6, cs 1, ss kAccStride).
template <int MODE, bool BWD>
__device__ __forceinline__ SampleIn load_sample(int64_t s64, int S, int per, int g, const uint16_t* __restrict__ latents,
                                                const float* __restrict__ dirs, const float* __restrict__ means,
                                                const int* __restrict__ radius, const float* __restrict__ dL_dc,
                                                const float* __restrict__ dmean = nullptr, int64_t cs = 1,
                                                int64_t ss = 3) {
  SampleIn x;
  x.a[0] = 0.f; x.a[1] = 0.f; x.a[2] = 1.f;
  x.c[0] = x.c[1] = x.c[2] = 0.f;
  x.m[0] = x.m[1] = x.m[2] = 0.f;
  x.z = make_uint4(0, 0, 0, 0);
  // look-ahead indices run past S (in 64-bit, so they cannot wrap)
  x.in = s64 >= 0 && s64 < S;
  if (!x.in) return x;
  const int s = static_cast<int>(s64);
  if (MODE == 0) {
    x.a[0] = dirs[3 * static_cast<int64_t>(s)];
    x.a[1] = dirs[3 * static_cast<int64_t>(s) + 1];
    x.a[2] = dirs[3 * static_cast<int64_t>(s) + 2];
  } else {
    x.in = radius[s] > 0;
    x.a[0] = means[s]; x.a[1] = means[S + s]; x.a[2] = means[2 * S + s];
  }
  if (g < 2) x.z = *reinterpret_cast<const uint4*>(latents + static_cast<int64_t>(s / per) * 16 + 8 * g);
  if (BWD && g == 0) {
#pragma unroll
    for (int i = 0; i < kMlpOut; ++i) {
      x.c[i] = dL_dc[(MODE == 1 ? 6 + i : i) * cs + s * ss];
      if (MODE == 1 && dmean && x.in) x.m[i] = dmean[static_cast<int64_t>(i) * S + s];
    }
  }
  return x;
}

// Unit view direction of a loaded sample (MODE 1: from the mean and camera).
template <int MODE>
__device__ __forceinline__ void sample_dir(const SampleIn& x, const DevCam& cam, float d[3], float& len) {
  len = 1.f;
  if (MODE == 0) {
    d[0] = x.a[0]; d[1] = x.a[1]; d[2] = x.a[2];
  } else if (x.in) {
    view_dir(x.a, cam, d, len);
  } else {
    d[0] = 0.f; d[1] = 0.f; d[2] = 1.f;
  }
}

// MODE 0: samples s < S with unit directions dirs[s][3], latent s / per,
//         colours out[s][3].
// MODE 1: sample s = Gaussian s of the projection; direction from its centre
//         and the camera; colours written into the record of every live
//         Gaussian (radius > 0).
template <int MODE>
__global__ __launch_bounds__(256) void k_mlp_fwd(int S, int per, const uint16_t* __restrict__ latents,
                                                 const float* __restrict__ dirs, const float* __restrict__ means,
                                                 const int* __restrict__ radius, DevCam cam,
                                                 const uint4* __restrict__ ops, const float* __restrict__ bias,
                                                 float* __restrict__ out, float* __restrict__ records) {
  __shared__ MlpShared sh;
  load_packed(sh, ops, bias);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
  const int stride = gridDim.x * 4;
  int grp = blockIdx.x * 4 + wave;
  SampleIn cur = load_sample<MODE, false>(static_cast<int64_t>(grp) * 16 + r, S, per, g, latents, dirs, means, radius,
                                          nullptr);
  for (; static_cast<int64_t>(grp) * 16 < S; grp += stride) {
    const int s = grp * 16 + r;
    const SampleIn nxt = load_sample<MODE, false>((static_cast<int64_t>(grp) + stride) * 16 + r, S, per, g, latents,
                                                  dirs, means, radius, nullptr);
    const bool valid = cur.in;
    float d[3], len;
    sample_dir<MODE>(cur, cam, d, len);
    MlpFwdState st;
    st.X = input_operand(g, valid, cur.z, d);
    mlp_forward_group(sh, lane, st);
    cur = nxt;
    if (g == 0 && valid) {
#pragma unroll
      for (int i = 0; i < kMlpOut; ++i) {
        float c = sigmoidf(st.o[i] + sh.bias[128 + i]);
        c = isfinite(c) ? c : 0.0f;
        if (MODE == 0) out[3 * s + i] = c;
        else records[12 * static_cast<int64_t>(s) + 6 + i] = c;
      }
    }
  }
}

// At least four groups of 16 per wave; about three workgroups per CU at most
// (each copies the 31 KB operand image to LDS once).
static unsigned mlp_grid(int64_t S) {
  return static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>(ceil_div(S, 256), 768)));
}

gs_status launch_mlp_pack(const uint16_t* params, void* packed, hipStream_t s) {
  uint4* ops = static_cast<uint4*>(packed);
  float* bias = reinterpret_cast<float*>(ops + kOps * 64);
  { TimedLaunch gs_tl("k_mlp_pack", s); k_mlp_pack<<<kOps, 64, 0, s>>>(params, ops, bias); }
  return check_launch("k_mlp_pack");
}

static const uint4* packed_ops(const void* p) { return static_cast<const uint4*>(p); }
static const float* packed_bias(const void* p) {
  return reinterpret_cast<const float*>(static_cast<const uint4*>(p) + kOps * 64);
}

gs_status launch_mlp_fwd(int64_t S, int per, const uint16_t* latents, const float* dirs, const void* packed,
                         float* rgb, hipStream_t s) {
  if (S == 0) return GS_OK;
  DevCam dummy{};
  { TimedLaunch gs_tl("k_mlp_fwd<0>", s); k_mlp_fwd<0><<<mlp_grid(S), 256, 0, s>>>(static_cast<int>(S), per, latents, dirs, nullptr, nullptr, dummy,
                                           packed_ops(packed), packed_bias(packed), rgb, nullptr); }
  return check_launch("k_mlp_fwd");
}

gs_status launch_mlp_render(int64_t n, const uint16_t* latents, const float* means, const int* radius,
                            const DevCam& cam, const void* packed, float* records, hipStream_t s) {
  if (n == 0) return GS_OK;
  { TimedLaunch gs_tl("k_mlp_fwd<1>", s); k_mlp_fwd<1><<<mlp_grid(n), 256, 0, s>>>(static_cast<int>(n), 1, latents, nullptr, means, radius, cam,
                                           packed_ops(packed), packed_bias(packed), nullptr, records); }
  return check_launch("k_mlp_render");
}

size_t mlp_packed_bytes() { return kOps * 64 * sizeof(uint4) + kBiasFloats * sizeof(float); }


// ------------------------------------------------------------------ backward
//
// A wave takes groups of 16 samples in the forward's lane layout, recomputes
// the forward (keeping the pre-activations for the ReLU masks) and runs
//   g3 = dL/dc * c (1 - c)            (quarter-0 lanes, rows 0..2)
//   g2 = (W3^T g3) [a2 > 0],  g1 = (W2^T g2) [a1 > 0],  dx = W1^T g1
// with the packed transposed weights as A operands, so every gradient lands in
// the D layout like the activations.  dx rows 0..15 are dL/dz, rows 16..31
// dL/dY (the SH encoding), which the basis gradient carries to the direction.
// The gradients entering the transposed products are hi + lo BF16 pairs as in
// the forward.  Weight gradients contract over samples: each group's
// activations and gradients go to LDS transposed ([unit][sample], hi and lo
// planes) and
//   dW1 += g1 x^T,  dW2 += g2 h1^T,  dW3 += g3 h2^T
// run as hi.hi + lo.hi + hi.lo (the lo.lo term, about 2^-18 relative, is
// dropped) on two 16x16x32 products whose K runs over the group's 16 samples
// twice: [g_hi | g_lo] x [h_hi | h_hi], then [g_hi | g_lo] x [h_lo | 0] (for the
// latent inputs, whose lo part is zero, the first alone).  Sums stay
// in registers for the wave's whole share and are written once as a partial
// vector; a fixed-order two-stage sum over waves makes the result
// deterministic for a given sample count.

constexpr int kPartStride = GS_MLP_PARAMS + 1;  // parameters, then the loss
constexpr int kBwdWavesMax = 1024;
constexpr int kReduceChunk = 64;                 // waves per first-stage block

// Transposed staging of one group ([unit][sample]); plane 0 holds the BF16
// value (hi), plane 1 the BF16 rounding of the remainder (lo).  Rows are
// padded to kRow = 20 values (10 banks): the four quarters of a wave, which
// write rows 4 apart, then land on disjoint LDS banks, and row starts stay
// 8-byte aligned for the operand reads.
constexpr int kRow = 20;
struct alignas(16) MlpStage {
  __bf16 x[2][32][kRow];
  __bf16 h1[2][64][kRow];
  __bf16 h2[2][64][kRow];
  __bf16 g1[2][64][kRow];
  __bf16 g2[2][64][kRow];
  __bf16 g3[2][16][kRow];
};

// unit u of sample r: slot e of a split operand
__device__ __forceinline__ void stage_put(__bf16 (*plane)[64][kRow], int u, int r, const Split8& v, int e) {
  plane[0][u][r] = v.hi[e];
  plane[1][u][r] = v.lo[e];
}

// A 16x16x32 operand over a group's staged samples: lane (g, r) takes row
// `row`, samples 8 (g & 1) .. 8 (g & 1) + 7 of plane p (K slots 8 g .. 8 g + 7:
// samples 0..15, then 0..15 again).
template <int ROWS>
__device__ __forceinline__ bf16x8 stage_read8(const __bf16 (*plane)[ROWS][kRow], int p, int row, int g) {
  bf16x8 v;
  __builtin_memcpy(&v, &plane[p][row][8 * (g & 1)], sizeof(v));
  return v;
}
// [hi | lo] along K (the gradient side), [hi | hi], and [lo | 0]
template <int ROWS>
__device__ __forceinline__ bf16x8 stage_hilo(const __bf16 (*plane)[ROWS][kRow], int row, int g) {
  return stage_read8<ROWS>(plane, g >> 1, row, g);
}
template <int ROWS>
__device__ __forceinline__ bf16x8 stage_lo0(const __bf16 (*plane)[ROWS][kRow], int row, int g) {
  bf16x8 v = stage_read8<ROWS>(plane, 1, row, g);
  return g < 2 ? v : bf16x8{};
}

__device__ __forceinline__ floatx4 mfma32(const bf16x8& a, const bf16x8& b, const floatx4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// D-layout gradients (4 row-blocks) as the split B operands of the next product.
__device__ __forceinline__ void grad_to_b(const floatx4 h[4], Split8& B0, Split8& B1) {
#pragma unroll
  for (int e = 0; e < 8; e += 2) {
    split_put2(B0, e, h[e >> 2][e & 3], h[e >> 2][(e & 3) + 1]);
    split_put2(B1, e, h[2 + (e >> 2)][e & 3], h[2 + (e >> 2)][(e & 3) + 1]);
  }
}

// Sum over the 16 lanes of each DPP row (the 16 samples of one quarter); every
// lane of the row gets the sum.  Fixed order, so deterministic.
__device__ __forceinline__ float row_sum16(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));   // quad 1,0,3,2
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));   // quad 2,3,0,1
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x124, 0xF, 0xF, false));  // row_ror 4
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x128, 0xF, 0xF, false));  // row_ror 8
  return v;
}

struct MlpGrads {
  floatx4 dW1[4][2], dW2[4][4], dW3[4];
  float db1[16], db2[16], db3[3], loss;
};

// One group: forward, loss gradient, backward, weight-gradient update.
// Returns dL/dz (dxz) and dL/dY (dxe) of this lane's sample in the D layout.
template <int MODE>
__device__ __forceinline__ void mlp_bwd_group(const MlpShared& sh, MlpStage& sg, MlpGrads& G, int lane,
                                              const SampleIn& x, const float d[3], bool loss_mode, float scale,
                                              floatx4& dxz, floatx4& dxe) {
  const int g = lane >> 4, r = lane & 15;
  const bool valid = x.in;
  const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
  MlpFwdState st;
  st.X = input_operand(g, valid, x.z, d);
  mlp_forward_group(sh, lane, st);
  floatx4 g3 = zero;
  if (g == 0 && valid) {
#pragma unroll
    for (int i = 0; i < kMlpOut; ++i) {
      const float c = sigmoidf(st.o[i] + sh.bias[128 + i]);
      float gc;
      if (MODE == 0 && loss_mode) {
        const float e = c - x.c[i];
        G.loss += scale * e * e;
        gc = 2.0f * scale * e;
      } else {
        gc = x.c[i];
      }
      g3[i] = gc * c * (1.0f - c);
      G.db3[i] += g3[i];
    }
  }
  Split8 Bg3;
#pragma unroll
  for (int e = 0; e < 8; e += 2)
    split_put2(Bg3, e, (g == 0 && e < 4) ? g3[e & 3] : 0.0f, (g == 0 && e < 4) ? g3[(e & 3) + 1] : 0.0f);
  floatx4 g2[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const floatx4 t = mfma2(sh.ops[(kOpW3T + b) * 64 + lane], Bg3, zero);
#pragma unroll
    for (int i = 0; i < 4; ++i) g2[b][i] = (st.h2[b][i] > 0.0f) ? t[i] : 0.0f;
  }
  Split8 G0, G1;
  grad_to_b(g2, G0, G1);
  floatx4 g1[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    floatx4 t = mfma2(sh.ops[(kOpW2T + 2 * b) * 64 + lane], G0, zero);
    t = mfma2(sh.ops[(kOpW2T + 2 * b + 1) * 64 + lane], G1, t);
#pragma unroll
    for (int i = 0; i < 4; ++i) g1[b][i] = (st.h1[b][i] > 0.0f) ? t[i] : 0.0f;
  }
  Split8 H0, H1;
  grad_to_b(g1, H0, H1);
  dxz = mfma2(sh.ops[(kOpW1T + 0) * 64 + lane], H0, zero);
  dxz = mfma2(sh.ops[(kOpW1T + 1) * 64 + lane], H1, dxz);
  dxe = mfma2(sh.ops[(kOpW1T + 2) * 64 + lane], H0, zero);
  dxe = mfma2(sh.ops[(kOpW1T + 3) * 64 + lane], H1, dxe);

  // transposed staging for the weight gradients: the split operands the
  // products above used (slot e of B_c carries unit hid(c, g, e))
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int u = hid(c, g, e);
      stage_put(sg.h1, u, r, c ? st.B1 : st.B0, e);
      stage_put(sg.h2, u, r, c ? st.C1 : st.C0, e);
      stage_put(sg.g1, u, r, c ? H1 : H0, e);
      stage_put(sg.g2, u, r, c ? G1 : G0, e);
    }
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      G.db1[4 * b + i] += g1[b][i];
      G.db2[4 * b + i] += g2[b][i];
    }
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    sg.x[0][8 * g + e][r] = st.X.hi[e];
    sg.x[1][8 * g + e][r] = st.X.lo[e];
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float v = g == 0 ? g3[i] : 0.0f;
    const __bf16 h = static_cast<__bf16>(v);
    sg.g3[0][4 * g + i][r] = h;
    sg.g3[1][4 * g + i][r] = static_cast<__bf16>(v - static_cast<float>(h));
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  bf16x8 bH1[4], bH1l[4], bH2[4], bH2l[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    bH1[b] = stage_read8<64>(sg.h1, 0, 16 * b + r, g);
    bH1l[b] = stage_lo0<64>(sg.h1, 16 * b + r, g);
    bH2[b] = stage_read8<64>(sg.h2, 0, 16 * b + r, g);
    bH2l[b] = stage_lo0<64>(sg.h2, 16 * b + r, g);
  }
  const bf16x8 bX0 = stage_read8<32>(sg.x, 0, r, g);
  const bf16x8 bX1 = stage_read8<32>(sg.x, 0, 16 + r, g), bX1l = stage_lo0<32>(sg.x, 16 + r, g);
  const bf16x8 aG3 = stage_hilo<16>(sg.g3, r, g);
#pragma unroll
  for (int bo = 0; bo < 4; ++bo) {
    const bf16x8 aG2 = stage_hilo<64>(sg.g2, 16 * bo + r, g);
    const bf16x8 aG1 = stage_hilo<64>(sg.g1, 16 * bo + r, g);
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) G.dW2[bo][bi] = mfma32(aG2, bH1l[bi], mfma32(aG2, bH1[bi], G.dW2[bo][bi]));
    G.dW1[bo][0] = mfma32(aG1, bX0, G.dW1[bo][0]);
    G.dW1[bo][1] = mfma32(aG1, bX1l, mfma32(aG1, bX1, G.dW1[bo][1]));
    G.dW3[bo] = mfma32(aG3, bH2l[bo], mfma32(aG3, bH2[bo], G.dW3[bo]));
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// MODE 0: sample s has direction dirs[s] and latent s / per (per a power of
//         two); dL/dc from dL_dc[S][3], or, with target != NULL, from the
//         distillation loss scale * |c - target|^2 (accumulated into the
//         partial's last slot).  dlat[S / per][16] is overwritten.
// MODE 1: sample s = Gaussian s of the projection (per = 1), dL/dc from rows
//         6..8 of g2d[9][S] or entries 6..8 of the accumulator rows (cs, ss:
//         see load_sample); dlat[s] and the direction's share of dL/dmean are
//         written for live Gaussians (dmean is added to), zeros elsewhere.
template <int MODE>
__global__ __launch_bounds__(256) void k_mlp_bwd(int S, int per, const uint16_t* __restrict__ latents,
                                                 const float* __restrict__ dirs, const float* __restrict__ means,
                                                 const int* __restrict__ radius, DevCam cam,
                                                 const uint4* __restrict__ ops, const float* __restrict__ bias,
                                                 const float* __restrict__ dL_dc, const float* __restrict__ target,
                                                 float scale, float* __restrict__ dlat, float* __restrict__ dmean,
                                                 float* __restrict__ partial, int64_t cs, int64_t ss) {
  __shared__ MlpShared sh;
  __shared__ MlpStage stage[4];
  load_packed(sh, ops, bias);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
  MlpStage& sg = stage[wave];
  const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
  MlpGrads G;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    G.dW1[a][0] = zero; G.dW1[a][1] = zero; G.dW3[a] = zero;
#pragma unroll
    for (int b = 0; b < 4; ++b) G.dW2[a][b] = zero;
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) { G.db1[k] = 0.f; G.db2[k] = 0.f; }
  G.db3[0] = G.db3[1] = G.db3[2] = 0.f;
  G.loss = 0.f;

  const int wave_id = blockIdx.x * 4 + wave, nwaves = gridDim.x * 4;
  const int ngroups = (S + 15) / 16;
  // per >= 16: a wave owns whole latents (per / 16 consecutive groups each)
  const int gpl = per >= 16 ? per / 16 : 1;
  const int nunits = ngroups / gpl;
  const bool loss_mode = (MODE == 0) && target != nullptr;
  const float* cin = (MODE == 0 && loss_mode) ? target : dL_dc;
  // groups of this wave in order: units wave_id, wave_id + nwaves, ..., each
  // unit's gpl groups in turn; the next group's inputs are loaded ahead
  auto group_of = [&](int unit, int q) { return (static_cast<int64_t>(unit) * gpl + q) * 16 + r; };
  SampleIn cur = load_sample<MODE, true>(group_of(wave_id, 0), wave_id < nunits ? S : 0, per, g, latents, dirs,
                                         means, radius, cin, dmean, cs, ss);
  for (int unit = wave_id; unit < nunits; unit += nwaves) {
    floatx4 zacc = zero;
    for (int q = 0; q < gpl; ++q) {
      const int s = static_cast<int>(group_of(unit, q));
      const int nunit = (q + 1 < gpl) ? unit : unit + nwaves;
      const int nq = (q + 1 < gpl) ? q + 1 : 0;
      const SampleIn nxt = load_sample<MODE, true>(group_of(nunit, nq), nunit < nunits ? S : 0, per, g, latents,
                                                   dirs, means, radius, cin, dmean, cs, ss);
      const bool valid = cur.in;
      float d[3], len;
      sample_dir<MODE>(cur, cam, d, len);
      floatx4 dxz, dxe;
      mlp_bwd_group<MODE>(sh, sg, G, lane, cur, d, loss_mode, scale, dxz, dxe);
      if (per >= 16) {
#pragma unroll
        for (int i = 0; i < 4; ++i) zacc[i] += row_sum16(dxz[i]);
      } else if (s < S) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float v = dxz[i];
          for (int w = 1; w < per; w <<= 1) v += __shfl_xor(v, w, 16);
          if ((r & (per - 1)) == 0) dlat[static_cast<int64_t>(s / per) * 16 + 4 * g + i] = valid ? v : 0.0f;
        }
      }
      if (MODE == 1) {
        // dL/dd = sum_j dL/dY_j grad Y_j(d); this lane holds j = 4g + i
        float w16[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) w16[j] = ((j >> 2) == g) ? dxe[j & 3] : 0.0f;
        float gd[3];
        sh_basis_vjp(3, d[0], d[1], d[2], w16, gd[0], gd[1], gd[2]);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          gd[k] += __shfl_xor(gd[k], 16, 64);
          gd[k] += __shfl_xor(gd[k], 32, 64);
        }
        if (g == 0 && valid) {
          // d = v / |v| with v = mean - centre:  dL/dv = (dL/dd - d (d . dL/dd)) / |v|
          const float dd = d[0] * gd[0] + d[1] * gd[1] + d[2] * gd[2];
          const float il = __builtin_amdgcn_rcpf(len);
#pragma unroll
          for (int k = 0; k < 3; ++k) dmean[static_cast<int64_t>(k) * S + s] = cur.m[k] + (gd[k] - d[k] * dd) * il;
        }
      }
      cur = nxt;
    }
    if (per >= 16 && r == 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) dlat[static_cast<int64_t>(unit) * 16 + 4 * g + i] = zacc[i];
    }
  }

  // partial vector of this wave (D layout: row 4g + i of a 16-row block, column r)
  float* out = partial + static_cast<int64_t>(wave_id) * kPartStride;
#pragma unroll
  for (int bo = 0; bo < 4; ++bo)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int o = 16 * bo + 4 * g + i;
#pragma unroll
      for (int bi = 0; bi < 4; ++bi) out[P_W2 + o * kMlpH + 16 * bi + r] = G.dW2[bo][bi][i];
      out[P_W1 + o * kMlpIn + r] = G.dW1[bo][0][i];
      out[P_W1 + o * kMlpIn + 16 + r] = G.dW1[bo][1][i];
    }
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int o = 4 * g + i;
      if (o < kMlpOut) out[P_W3 + o * kMlpH + 16 * bi + r] = G.dW3[bi][i];
    }
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float s1 = row_sum16(G.db1[4 * b + i]);
      const float s2 = row_sum16(G.db2[4 * b + i]);
      if (r == 0) {
        out[P_B1 + 16 * b + 4 * g + i] = s1;
        out[P_B2 + 16 * b + 4 * g + i] = s2;
      }
    }
#pragma unroll
  for (int i = 0; i < kMlpOut; ++i) {
    const float s3 = row_sum16(G.db3[i]);
    if (lane == 0) out[P_B3 + i] = s3;
  }
  const float sl = row_sum16(G.loss);
  if (lane == 0) out[GS_MLP_PARAMS] = sl;
}

// First stage: block (x, y) sums waves [64 y, 64 y + 64) of 64 parameters,
// four interleaved sub-sums per parameter combined in a fixed order.
__global__ __launch_bounds__(256) void k_mlp_reduce1(const float* __restrict__ partial, int nwaves,
                                                     float* __restrict__ stage2) {
  __shared__ float part[4][64];
  const int p = blockIdx.x * 64 + (threadIdx.x & 63), q = threadIdx.x >> 6;
  const int w0 = blockIdx.y * kReduceChunk, w1 = min(nwaves, w0 + kReduceChunk);
  float acc = 0.f;
  if (p < kPartStride)
    for (int w = w0 + q; w < w1; w += 4) acc += partial[static_cast<int64_t>(w) * kPartStride + p];
  part[q][threadIdx.x & 63] = acc;
  __syncthreads();
  if (q == 0 && p < kPartStride) {
    const int t = threadIdx.x;
    stage2[static_cast<int64_t>(blockIdx.y) * kPartStride + p] = ((part[0][t] + part[1][t]) + part[2][t]) + part[3][t];
  }
}

__global__ __launch_bounds__(256) void k_mlp_reduce2(const float* __restrict__ stage2, int nchunks,
                                                     float* __restrict__ dparams, float* __restrict__ loss) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= kPartStride) return;
  float acc = 0.f;
  for (int c = 0; c < nchunks; ++c) acc += stage2[static_cast<int64_t>(c) * kPartStride + p];
  if (p < GS_MLP_PARAMS) dparams[p] = acc;
  else if (loss) *loss = acc;
}

// Waves of the backward for S samples: about 8 groups of 16 per wave, a
// multiple of 4 (one block), at most kBwdWavesMax.
static int mlp_bwd_waves(int64_t S, int per) {
  const int64_t groups = std::max<int64_t>(1, ceil_div(S, 16));
  const int64_t units = per >= 16 ? std::max<int64_t>(1, groups / (per / 16)) : groups;
  int64_t w = ceil_div(units, 8);
  w = std::min<int64_t>(kBwdWavesMax, std::max<int64_t>(4, ceil_div(w, 4) * 4));
  return static_cast<int>(w);
}

size_t mlp_bwd_workspace(int64_t S, int per) {
  const int w = mlp_bwd_waves(S, per);
  const int chunks = static_cast<int>(ceil_div(w, kReduceChunk));
  return static_cast<size_t>(w + chunks) * kPartStride * sizeof(float);
}

static gs_status reduce_partials(float* ws, int nwaves, float* dparams, float* loss, hipStream_t s) {
  const int chunks = static_cast<int>(ceil_div(nwaves, kReduceChunk));
  float* stage2 = ws + static_cast<size_t>(nwaves) * kPartStride;
  { TimedLaunch gs_tl("k_mlp_reduce1", s); k_mlp_reduce1<<<dim3(static_cast<unsigned>(ceil_div(kPartStride, 64)), chunks), 256, 0, s>>>(ws, nwaves, stage2); }
  { TimedLaunch gs_tl("k_mlp_reduce2", s); k_mlp_reduce2<<<static_cast<unsigned>(ceil_div(kPartStride, 256)), 256, 0, s>>>(stage2, chunks, dparams, loss); }
  return check_launch("k_mlp_reduce");
}

gs_status launch_mlp_bwd(int64_t S, int per, const uint16_t* latents, const float* dirs, const void* packed,
                         const float* dL_drgb, const float* target, float scale, float* dlat, float* dparams,
                         float* loss, void* ws, hipStream_t s) {
  const int waves = mlp_bwd_waves(S, per);
  DevCam dummy{};
  { TimedLaunch gs_tl("k_mlp_bwd<0>", s); k_mlp_bwd<0><<<waves / 4, 256, 0, s>>>(static_cast<int>(S), per, latents, dirs, nullptr, nullptr, dummy,
                                         packed_ops(packed), packed_bias(packed), dL_drgb, target, scale, dlat,
                                         nullptr, static_cast<float*>(ws), 1, 3); }
  gs_status st = check_launch("k_mlp_bwd");
  if (st != GS_OK) return st;
  return reduce_partials(static_cast<float*>(ws), waves, dparams, loss, s);
}

gs_status launch_mlp_render_bwd(int64_t n, const uint16_t* latents, const float* means, const int* radius,
                                const DevCam& cam, const void* packed, const float* g2d, bool rows, float* dlat,
                                float* dmeans, float* dparams, void* ws, hipStream_t s) {
  const int waves = mlp_bwd_waves(n, 1);
  const int64_t cs = rows ? 1 : n, ss = rows ? kAccStride : 1;
  { TimedLaunch gs_tl("k_mlp_bwd<1>", s); k_mlp_bwd<1><<<waves / 4, 256, 0, s>>>(static_cast<int>(n), 1, latents, nullptr, means, radius, cam,
                                         packed_ops(packed), packed_bias(packed), g2d, nullptr, 0.0f, dlat, dmeans,
                                         static_cast<float*>(ws), cs, ss); }
  gs_status st = check_launch("k_mlp_render_bwd");
  if (st != GS_OK) return st;
  return reduce_partials(static_cast<float*>(ws), waves, dparams, nullptr, s);
}

// ------------------------------------------------------------------ training support

// SH colour of Gaussian s / per at direction dirs[s] (the projection's colour
// rule at an arbitrary direction), optionally clamped to [0, 1].
__global__ __launch_bounds__(256) void k_sh_colour(int S, int per, int n, int deg, const float* __restrict__ sh,
                                                   const float* __restrict__ dirs, int clamp01,
                                                   float* __restrict__ out) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= S) return;
  const int i = s / per;
  float Y[16];
  sh_basis(deg, dirs[3 * s], dirs[3 * s + 1], dirs[3 * s + 2], Y);
  const int nc = (deg + 1) * (deg + 1);
  for (int c = 0; c < 3; ++c) {
    float acc = 0.f;
    for (int j = 0; j < nc; ++j) acc += Y[j] * sh[(static_cast<int64_t>(j) * 3 + c) * n + i];
    float v = fmaxf(acc + 0.5f, 0.0f);
    if (clamp01) v = fminf(v, 1.0f);
    out[3 * static_cast<int64_t>(s) + c] = v;
  }
}

gs_status launch_sh_colour(int64_t S, int per, int64_t n, int deg, const float* sh, const float* dirs, int clamp01,
                           float* out, hipStream_t s) {
  if (S == 0) return GS_OK;
  { TimedLaunch gs_tl("k_sh_colour", s); k_sh_colour<<<static_cast<unsigned>(ceil_div(S, 256)), 256, 0, s>>>(static_cast<int>(S), per, static_cast<int>(n),
                                                                      deg, sh, dirs, clamp01, out); }
  return check_launch("k_sh_colour");
}

// Adam (bias-corrected), FP32 master parameters, optional BF16 copy rounded to
// nearest even for the forward.
__global__ __launch_bounds__(256) void k_adam(int64_t n, float* __restrict__ p, const float* __restrict__ grad,
                                              float* __restrict__ m, float* __restrict__ v,
                                              uint16_t* __restrict__ pb, float lr, float b1, float b2, float eps,
                                              float bc1, float bc2) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = grad[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  p[i] = pi;
  if (pb) {
    const __bf16 h = static_cast<__bf16>(pi);
    uint16_t bits;
    __builtin_memcpy(&bits, &h, sizeof(bits));
    pb[i] = bits;
  }
}

gs_status launch_adam(int64_t n, float* p, const float* g, float* m, float* v, uint16_t* pb, float lr, float b1,
                      float b2, float eps, float bc1, float bc2, hipStream_t s) {
  if (n == 0) return GS_OK;
  { TimedLaunch gs_tl("k_adam", s); k_adam<<<static_cast<unsigned>(ceil_div(n, 256)), 256, 0, s>>>(n, p, g, m, v, pb, lr, b1, b2, eps, bc1, bc2); }
  return check_launch("k_adam");
}

}  // namespace gs
