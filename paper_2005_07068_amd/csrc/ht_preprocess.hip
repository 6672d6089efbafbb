// Observation preprocessing (section II.B): RGB-D frame -> O = (O_s, O_d) by skin colour and
// depth segmentation, in exact integer arithmetic (the rule is stated in handtrack.h).
//
// Two launches: per-block minima of the defined depths of skin pixels, then every block
// reduces those few minima itself (no atomics, no memset: graph-capturable) and writes the
// outputs.  The work is a few bytes per pixel and bound by launch latency at 640x480.

#include "ht_device.h"

namespace ht {

namespace {

constexpr int kPixPerThread = 4;

__device__ __forceinline__ bool is_skin(const uint8_t* __restrict__ rgb, int i,
                                        const ht_seg_params& p) {
  const int r = rgb[3 * i], g = rgb[3 * i + 1], b = rgb[3 * i + 2];
  // BT.601 chroma, 8-bit fixed point; >> on a negative int is an arithmetic (floor) shift
  const int cb = 128 + ((-43 * r - 85 * g + 128 * b + 128) >> 8);
  const int cr = 128 + ((128 * r - 107 * g - 21 * b + 128) >> 8);
  return cb >= p.cb_lo && cb <= p.cb_hi && cr >= p.cr_lo && cr <= p.cr_hi;
}

__device__ __forceinline__ int block_min(int v, int* s_red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
  if (lane == 0) s_red[wv] = v;
  __syncthreads();
  int m = s_red[0];
  for (int q = 1; q < kWavesPerBlock; ++q) m = min(m, s_red[q]);
  __syncthreads();
  return m;
}

__global__ __launch_bounds__(kBlock) void seg_min_kernel(int n, const uint8_t* __restrict__ rgb,
                                                         const uint16_t* __restrict__ depth,
                                                         ht_seg_params p,
                                                         int* __restrict__ partial) {
  __shared__ int s_red[kWavesPerBlock];
  int m = INT_MAX;
  const int stride = gridDim.x * kBlock;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const int d = depth[i];
    if (d > 0 && is_skin(rgb, i, p)) m = min(m, d);
  }
  m = block_min(m, s_red);
  if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

__global__ __launch_bounds__(kBlock) void seg_apply_kernel(int n, int n_partial,
                                                           const uint8_t* __restrict__ rgb,
                                                           const uint16_t* __restrict__ depth,
                                                           ht_seg_params p,
                                                           const int* __restrict__ partial,
                                                           uint16_t* __restrict__ depth_out,
                                                           uint8_t* __restrict__ skin_out) {
  __shared__ int s_red[kWavesPerBlock];
  int m = INT_MAX;
  for (int q = threadIdx.x; q < n_partial; q += kBlock) m = min(m, partial[q]);
  const int z0 = block_min(m, s_red);
  const bool any = z0 != INT_MAX;
  const int z1 = any ? z0 + p.band_mm : -1;
  const int bg = (int)p.bg_depth_mm;
  const int stride = gridDim.x * kBlock;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const int d = depth[i];
    const bool band = any && d > 0 && d >= z0 && d <= z1;
    depth_out[i] = (uint16_t)(band ? d : (d > 0 ? bg : 0));
    skin_out[i] = (uint8_t)(band && is_skin(rgb, i, p) ? 1 : 0);
  }
}

}  // namespace

int preprocess_partials(int W, int H) {
  const long long n = (long long)W * H;
  const long long blocks = (n + (long long)kBlock * kPixPerThread - 1) / ((long long)kBlock * kPixPerThread);
  return (int)std::min<long long>(std::max<long long>(blocks, 1), 1024);
}

hipError_t launch_preprocess(int W, int H, const uint8_t* rgb, const uint16_t* depth,
                             const ht_seg_params& p, int* partial, uint16_t* depth_out,
                             uint8_t* skin_out, hipStream_t s) {
  const int n = W * H;
  const int nb = preprocess_partials(W, H);
  hipLaunchKernelGGL(seg_min_kernel, dim3(nb), dim3(kBlock), 0, s, n, rgb, depth, p, partial);
  hipLaunchKernelGGL(seg_apply_kernel, dim3(nb), dim3(kBlock), 0, s, n, nb, rgb, depth, p,
                     partial, depth_out, skin_out);
  return hipGetLastError();
}

}  // namespace ht
