// Photometric L1 loss of a rendered image against a target, and its gradient.
// The loss is a device scalar: per-block partial sums, then one block sums the
// partials in a fixed order (deterministic).
#include "gs_internal.h"

#include <mutex>

namespace gs {

constexpr int kL1Blocks = GS_L1_PARTIALS;

// Sum over a 256-thread workgroup in a fixed order: DPP within each 16-lane
// row, the rows of a wave through readlane, then the four waves via LDS
// (red >= 4 floats).  The result is valid in thread 0.
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float block_sum256(float v, float* red) {
  v += dpp_f32<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_f32<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_f32<0x124>(v);   // row_ror:4
  v += dpp_f32<0x128>(v);   // row_ror:8
  // readlane moves 32-bit words: the float's bits, not its value
  auto lane_f = [&](int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)); };
  const float w = (lane_f(0) + lane_f(16)) + (lane_f(32) + lane_f(48));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
  __syncthreads();
  return ((red[0] + red[1]) + red[2]) + red[3];
}


__global__ __launch_bounds__(256) void k_l1_partial(const float* __restrict__ img, const float* __restrict__ tgt,
                                                    int64_t count, float inv_count, float* __restrict__ grad,
                                                    float* __restrict__ partial) {
  __shared__ float red[4];
  auto sgn = [&](float d) { return d > 0.0f ? inv_count : (d < 0.0f ? -inv_count : 0.0f); };
  float s = 0.0f;
  const int64_t t0 = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
  // 16-byte accesses when all three arrays allow them (four values per step),
  // then the remaining count % 4 values
  const bool vec = ((reinterpret_cast<uintptr_t>(img) | reinterpret_cast<uintptr_t>(tgt) |
                     reinterpret_cast<uintptr_t>(grad)) & 15u) == 0;
  int64_t done = 0;
  if (vec) {
    const int64_t n4 = count / 4;
    for (int64_t i = t0; i < n4; i += stride) {
      const float4 a = reinterpret_cast<const float4*>(img)[i];
      const float4 b = reinterpret_cast<const float4*>(tgt)[i];
      const float d0 = a.x - b.x, d1 = a.y - b.y, d2 = a.z - b.z, d3 = a.w - b.w;
      s += fabsf(d0);
      s += fabsf(d1);
      s += fabsf(d2);
      s += fabsf(d3);
      if (grad) reinterpret_cast<float4*>(grad)[i] = make_float4(sgn(d0), sgn(d1), sgn(d2), sgn(d3));
    }
    done = 4 * n4;
  }
  for (int64_t i = done + t0; i < count; i += stride) {
    const float d = img[i] - tgt[i];
    s += fabsf(d);
    if (grad) grad[i] = sgn(d);
  }
  const float total = block_sum256(s, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void k_l1_final(const float* __restrict__ partial, int nb, float inv_count,
                                                  float* __restrict__ loss) {
  __shared__ float red[4];
  float s = 0.0f;
  for (int i = threadIdx.x; i < nb; i += 256) s += partial[i];
  const float total = block_sum256(s, red);
  if (threadIdx.x == 0) *loss = total * inv_count;
}

gs_status launch_l1(const float* img, const float* target, int64_t count, float* loss, float* grad,
                    float* partials, hipStream_t s) {
  const int nb = static_cast<int>(std::min<int64_t>(kL1Blocks, ceil_div(count, 256)));
  const float inv = 1.0f / static_cast<float>(count);
  { TimedLaunch gs_tl("k_l1_partial", s); k_l1_partial<<<nb, 256, 0, s>>>(img, target, count, inv, grad, partials); }
  { TimedLaunch gs_tl("k_l1_final", s); k_l1_final<<<1, 256, 0, s>>>(partials, nb, inv, loss); }
  return check_launch("k_l1");
}


// ------------------------------------------------- no-allocation variant
// Partial sums of gs_l1_loss_static live in this file-scope device array
// (one copy per GPU, alive until the process ends).  Host code never passes
// the array's name to a kernel: the name is a host-side stand-in, and the
// device address of each GPU's copy is looked up once per device.
static __device__ __align__(256) float scratch[GS_L1_STATIC_PARTIALS];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of the current device's scratch array (looked up on the
// first call on each device, with that device current).
gs_status static_scratch(float** out) {
  int dev = -1;
  gs_status st = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (st != GS_OK) return st;
  if (dev < 0 || dev >= kMaxDevices) return fail(GS_ERR_UNSUPPORTED, "gs_l1_loss_static: device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    st = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (st != GS_OK) return st;
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[dev];
  return GS_OK;
}

}  // namespace gs
