// Evaluation kernels: observation packing, forward kinematics prologue, work scheduling,
// persistent ray cast + Eq. 4 cost terms + reduction (with the optional adjoint), finalize.
//
// Work decomposition: an 8x8 pixel tile is one wavefront (64 lanes, one pixel each).  The
// primitives of a particle are culled per tile by their conservative screen boxes with a
// ballot; tiles that no primitive touches render the background, whose cost terms are
// summed once per observation, so only touched tiles are visited.  A work item is a run of
// `tiles_per_item` touched-rectangle tiles of one particle; persistent workgroups of four
// wavefronts dequeue items, stage the particle's primitive table in LDS and write one
// partial per item, which the finalize kernel combines in item order (deterministic).  The
// clamped depth sum is accumulated in FP64: its FP32 per-pixel terms are multiples of
// 2^-15 mm (depths of at least 256 mm), so the sum is exact and the cost does not depend on
// how the tiles were split into items.
#include <float.h>
#include <math.h>

#include "ht_device.h"

namespace ht {

// ------------------------------------------------------------------------------------
// small helpers

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// A pointer read from memory (a FrameSlot field) is generic to the compiler, and generic
// loads count against the LDS counter too, so every LDS wait would also wait for them; these
// buffers are device memory, so their loads are issued as global loads.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* global_ptr(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
// Wavefront total on the vector unit: DPP moves within each 16-lane row (quad permutations,
// then row rotations by 4 and 8), then the four row sums read from lanes 0, 16, 32, 48 and
// added in a fixed order.  Deterministic; the result is wave-uniform.  (__shfl_xor lowers to
// ds_bpermute, an LDS round trip per step.)
template <int CTRL>
__device__ __forceinline__ int dpp(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}
__device__ __forceinline__ float wave_total(float v) {
  v += __int_as_float(dpp<0xB1>(__float_as_int(v)));    // quad_perm [1, 0, 3, 2]
  v += __int_as_float(dpp<0x4E>(__float_as_int(v)));    // quad_perm [2, 3, 0, 1]
  v += __int_as_float(dpp<0x124>(__float_as_int(v)));   // row_ror:4
  v += __int_as_float(dpp<0x128>(__float_as_int(v)));   // row_ror:8
  const int b = __float_as_int(v);
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(b, 0));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(b, 16));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(b, 32));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(b, 48));
  return (r0 + r1) + (r2 + r3);
}
// Row total: after the same four DPP steps every lane holds the sum over its 16-lane row.
__device__ __forceinline__ float row_total(float v) {
  v += __int_as_float(dpp<0xB1>(__float_as_int(v)));
  v += __int_as_float(dpp<0x4E>(__float_as_int(v)));
  v += __int_as_float(dpp<0x124>(__float_as_int(v)));
  v += __int_as_float(dpp<0x128>(__float_as_int(v)));
  return v;
}
__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
  int x = (int)v;
  x |= dpp<0xB1>(x);
  x |= dpp<0x4E>(x);
  x |= dpp<0x124>(x);
  x |= dpp<0x128>(x);
  return (uint32_t)(__builtin_amdgcn_readlane(x, 0) | __builtin_amdgcn_readlane(x, 16) |
                    __builtin_amdgcn_readlane(x, 32) | __builtin_amdgcn_readlane(x, 48));
}
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

// C = A * B for 3x4 affine transforms (row-major, implicit last row 0 0 0 1).
__device__ inline void mul34(const double* A, const double* B, double* C) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      double v = A[i * 4 + 0] * B[0 * 4 + j] + A[i * 4 + 1] * B[1 * 4 + j] +
                 A[i * 4 + 2] * B[2 * 4 + j];
      if (j == 3) v += A[i * 4 + 3];
      C[i * 4 + j] = v;
    }
  }
}

// T <- T * Rot(axis, angle) (Rodrigues) given sin and cos of the angle; rotation part only.
__device__ inline void post_rotate(double* T, const double* a, double s, double c) {
  const double C = 1.0 - c;
  const double R[9] = {c + a[0] * a[0] * C, a[0] * a[1] * C - a[2] * s, a[0] * a[2] * C + a[1] * s,
                       a[1] * a[0] * C + a[2] * s, c + a[1] * a[1] * C, a[1] * a[2] * C - a[0] * s,
                       a[2] * a[0] * C - a[1] * s, a[2] * a[1] * C + a[0] * s, c + a[2] * a[2] * C};
  double out[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      out[i * 3 + j] = T[i * 4 + 0] * R[0 * 3 + j] + T[i * 4 + 1] * R[1 * 3 + j] +
                       T[i * 4 + 2] * R[2 * 3 + j];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) T[i * 4 + j] = out[i * 3 + j];
}

__device__ __forceinline__ void split(double x, float& hi, float& lo) {
  hi = (float)x;
  lo = (float)(x - (double)hi);
}

// ------------------------------------------------------------------------------------
// observation packing: one wavefront per tile

__global__ __launch_bounds__(kBlock) void pack_kernel(const uint16_t* __restrict__ depth,
                                                      const uint8_t* __restrict__ skin, int W,
                                                      int H, int TW, int TH,
                                                      uint32_t* __restrict__ words,
                                                      float* __restrict__ tile_td,
                                                      int* __restrict__ tile_skin, float bg) {
  const int lane = threadIdx.x & (kWave - 1);
  const int tile = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (tile >= TW * TH) return;
  const int tx = tile % TW, ty = tile / TW;
  const int u = tx * kTile + (lane & 7), v = ty * kTile + (lane >> 3);
  uint32_t w = 0;
  float td = 0.0f;
  int sk = 0;
  if (u < W && v < H) {
    const uint32_t d = depth[(size_t)v * W + u];
    const int s = skin[(size_t)v * W + u] != 0;
    w = d | (s ? kSkinBit : 0u) | kValidBit;
    const float rbg = bg > 0.0f ? bg : 0.0f;
    td = fminf(fabsf((float)d - rbg), kDClamp);
    sk = s;
  }
  words[(size_t)tile * kTilePx + lane] = w;
  td = wave_sum(td);
  sk = wave_sum(sk);
  if (lane == 0) {
    tile_td[tile] = td;
    tile_skin[tile] = sk;
  }
}

// Whole-ROI background sums in a fixed order (one workgroup).
__global__ __launch_bounds__(kBlock) void total_kernel(const float* __restrict__ tile_td,
                                                       const int* __restrict__ tile_skin,
                                                       int n_tiles, double* __restrict__ out) {
  __shared__ double s_td[kBlock];
  __shared__ double s_sk[kBlock];
  double td = 0.0, sk = 0.0;
  for (int i = threadIdx.x; i < n_tiles; i += kBlock) {
    td += (double)tile_td[i];
    sk += (double)tile_skin[i];
  }
  s_td[threadIdx.x] = td;
  s_sk[threadIdx.x] = sk;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s_td[threadIdx.x] += s_td[threadIdx.x + o];
      s_sk[threadIdx.x] += s_sk[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = s_td[0];
    out[1] = s_sk[0];
  }
}

hipError_t launch_pack_observation(const uint16_t* depth, const uint8_t* skin, int W, int H,
                                   int TW, int TH, uint32_t* words, float* tile_td,
                                   int* tile_skin, double* totals, float bg, hipStream_t s) {
  const int n_tiles = TW * TH;
  hipLaunchKernelGGL(pack_kernel, dim3((n_tiles + kWavesPerBlock - 1) / kWavesPerBlock),
                     dim3(kBlock), 0, s, depth, skin, W, H, TW, TH, words, tile_td, tile_skin,
                     bg);
  hipLaunchKernelGGL(total_kernel, dim3(1), dim3(kBlock), 0, s, tile_td, tile_skin, n_tiles,
                     totals);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// work list, built by one workgroup (kSchedBlock threads, kSchedSmall for launches of at most
// kSchedSmall particles, whose barriers then wait on 4 wavefronts instead of 16).  The tiles
// per work item are
// chosen from the launch's actual tile count: about kItemsPerGroup items per persistent
// workgroup (more, smaller items measured slower: each item stages its particle's tables),
// a multiple of the wavefronts per workgroup, at least kFloorTilesFwd (kFloorTilesGrad for
// a gradient) and at most the configured tiles_per_item (itself >= kMinTilesPerItem, which
// sizes the workspace).  An exclusive scan of the per-particle item counts then gives the
// item -> particle map, and the dequeue counter is reset here (no memset: graph-capturable).

constexpr int kItemsPerGroup = 1;

// Inclusive scan over the workgroup; every thread gets its own prefix and the total: a scan
// within each wavefront by lane shifts, then the wavefront totals through LDS (two barriers
// instead of two per doubling step).
// The same for a pair: v is scanned, w only totalled, through the same two barriers.
template <int NW>
__device__ int block_scan2(int2* s_sum, int v, int w, int* total_v, int* total_w) {
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int u = __shfl_up(v, o);
    if (lane >= o) v += u;
    w += __shfl_xor(w, o);
  }
  if (lane == kWave - 1) s_sum[wv] = make_int2(v, w);
  __syncthreads();
  int before = 0, all = 0, all_w = 0;
#pragma unroll
  for (int q = 0; q < NW; ++q) {
    const int2 t = s_sum[q];
    before += q < wv ? t.x : 0;
    all += t.x;
    all_w += t.y;
  }
  __syncthreads();
  *total_v = all;
  *total_w = all_w;
  return v + before;
}

template <int NW>
__device__ int block_scan(int* s_sum, int v, int* total) {
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int u = __shfl_up(v, o);
    if (lane >= o) v += u;
  }
  if (lane == kWave - 1) s_sum[wv] = v;
  __syncthreads();
  int before = 0, all = 0;
#pragma unroll
  for (int q = 0; q < NW; ++q) {
    const int w = s_sum[q];
    before += q < wv ? w : 0;
    all += w;
  }
  __syncthreads();
  *total = all;
  return v + before;
}

// Each thread of the work-list kernel loads kSchedBatch tile counts at a time, so that their
// latencies overlap (the counts were written by every XCD, so each load misses this L2).
constexpr int kSchedBatch = 8;
constexpr int kSchedBlock = 1024;    // threads of the work-list kernel (its only workgroup)
constexpr int kSchedSmall = 256;     // ... for launches of at most this many particles
constexpr int kSchedWindow = 8192;   // items staged in LDS per round (32 KB)

// Workspace particle holding the kinematics of evaluated particle r (itself, or its source
// from the previous evaluation).
__device__ __forceinline__ int src_of(const EvalArgs& a, int r) {
  return a.src ? (r / a.n_particles) * a.src_stride + a.src[r] : r;
}

// Tile counts of particles i0 .. i0 + kSchedBatch - 1 (zero from e on).  The loads are
// unconditional, their indices clamped to the last particle, so all of them are in flight at
// once (a guarded load per particle compiled into a wait per particle).
__device__ __forceinline__ void load_tiles(const EvalArgs& a, const Workspace& ws, int i0, int e,
                                           int (&v)[kSchedBatch]) {
  const int last = a.n_frames * a.n_particles - 1;
  int r[kSchedBatch];
#pragma unroll
  for (int j = 0; j < kSchedBatch; ++j) r[j] = min(i0 + j, last);
  if (a.src) {   // one branch for the batch (src_of per particle branched per load)
    int q[kSchedBatch];
#pragma unroll
    for (int j = 0; j < kSchedBatch; ++j) q[j] = a.src[r[j]];
#pragma unroll
    for (int j = 0; j < kSchedBatch; ++j) r[j] = (r[j] / a.n_particles) * a.src_stride + q[j];
  }
#pragma unroll
  for (int j = 0; j < kSchedBatch; ++j) v[j] = ws.tiles[r[j]];
  // past the chunk: not counted and no tiles (-1, as a skipped particle)
#pragma unroll
  for (int j = 0; j < kSchedBatch; ++j) v[j] = i0 + j < e ? v[j] : -1;
}

// The tile counts of batch i0 of a thread whose particles start at b: the first batch (every
// batch of launches up to BLOCK * kSchedBatch particles) is kept in registers from the
// first pass, later ones are loaded again.
__device__ __forceinline__ void batch_tiles(const EvalArgs& a, const Workspace& ws, int i0, int b,
                                            int e, const int (&v0)[kSchedBatch],
                                            int (&v)[kSchedBatch]) {
  if (i0 == b) {
#pragma unroll
    for (int j = 0; j < kSchedBatch; ++j) v[j] = v0[j];
  } else {
    load_tiles(a, ws, i0, e, v);
  }
}

template <int BLOCK>
__device__ void schedule_items(const EvalArgs& a, int n_total, const Workspace& ws) {
  constexpr int kNW = BLOCK / kWave;
  __shared__ int s_sum[kNW];
  const int t = threadIdx.x;
  const int chunk = (n_total + BLOCK - 1) / BLOCK;
  const int b = min(t * chunk, n_total), e = min(b + chunk, n_total);
  int v0[kSchedBatch];
  load_tiles(a, ws, b, e, v0);
  // tiles to visit, and particles evaluated (not skipped), of this thread's chunk; a skipped
  // particle has tile count -1 and no work items
  int tiles = 0, evaluated = 0;
  for (int i0 = b; i0 < e; i0 += kSchedBatch) {
    int v[kSchedBatch];
    batch_tiles(a, ws, i0, b, e, v0, v);
#pragma unroll
    for (int j = 0; j < kSchedBatch; ++j) {
      tiles += max(v[j], 0);
      evaluated += v[j] >= 0 ? 1 : 0;
    }
  }
  __shared__ int2 s_sum2[kNW];
  int total_tiles, total_evaluated;
  block_scan2<kNW>(s_sum2, tiles, evaluated, &total_tiles, &total_evaluated);
  const long long target = (long long)a.grid * kItemsPerGroup;
  long long tq = ((long long)total_tiles + target - 1) / target;
  tq = (tq + kWavesPerBlock - 1) / kWavesPerBlock * kWavesPerBlock;
  // a gradient item also writes and its finalize re-reads a wrench per segment: longer items
  const long long lo = a.grad ? (long long)kFloorTilesGrad : (long long)kFloorTilesFwd;
  const int tpi = (int)max(min(lo, (long long)a.tiles_per_item), min(tq, (long long)a.tiles_per_item));

  int local = 0;
  for (int i0 = b; i0 < e; i0 += kSchedBatch) {
    int v[kSchedBatch];
    batch_tiles(a, ws, i0, b, e, v0, v);
#pragma unroll
    for (int j = 0; j < kSchedBatch; ++j) local += (max(v[j], 0) + tpi - 1) / tpi;
  }
  int total_items;
  const int incl = block_scan<kNW>(s_sum, local, &total_items);
  const int my_b = incl - local, my_e = incl;   // this thread's items, contiguous
  // item offsets: staged in LDS (then stored coalesced) when they fit
  __shared__ int s_map[kSchedWindow];
  const bool staged = n_total <= kSchedWindow;
  int off = my_b;
  for (int i0 = b; i0 < e; i0 += kSchedBatch) {
    int v[kSchedBatch];
    batch_tiles(a, ws, i0, b, e, v0, v);
#pragma unroll
    for (int j = 0; j < kSchedBatch; ++j) {
      if (i0 + j >= e) break;
      if (staged) s_map[i0 + j] = off;
      else ws.item_off[i0 + j] = off;
      off += (max(v[j], 0) + tpi - 1) / tpi;
    }
  }
  if (staged) {
    __syncthreads();
    for (int i = t; i < n_total; i += BLOCK) ws.item_off[i] = s_map[i];
    __syncthreads();
  }
  // the item -> particle map, staged in LDS one window at a time so that the global stores
  // are coalesced (each thread's items are contiguous, so its own stores would touch one
  // cache line per lane)
  for (int w0 = 0; w0 < total_items; w0 += kSchedWindow) {
    const int w1 = min(w0 + kSchedWindow, total_items);
    if (my_b < w1 && my_e > w0) {
      int o = my_b;
      for (int i0 = b; i0 < e && o < w1; i0 += kSchedBatch) {
        int v[kSchedBatch];
        batch_tiles(a, ws, i0, b, e, v0, v);
#pragma unroll
        for (int j = 0; j < kSchedBatch; ++j) {
          if (i0 + j >= e) break;
          const int n = (max(v[j], 0) + tpi - 1) / tpi;
          const int q0 = max(o, w0), q1 = min(o + n, w1);
          for (int q = q0; q < q1; ++q) s_map[q - w0] = i0 + j;
          o += n;
        }
      }
    }
    __syncthreads();
    for (int q = w0 + t; q < w1; q += BLOCK) ws.item_map[q] = s_map[q - w0];
    __syncthreads();
  }
  if (t == 0) {
    if (a.eval_count) atomicAdd(&a.eval_count[a.grad ? 1 : 0], (unsigned long long)total_evaluated);
    ws.item_off[n_total] = total_items;
    ws.counters[0] = 0;
    ws.counters[1] = total_items;
    ws.counters[2] = tpi;
    // a gradient launch with at most about two items per persistent workgroup has nothing to
    // even out its items' different costs (and its tiles are the heavier ones), so each
    // particle's items take interleaved tiles of about equal work; elsewhere runs of
    // consecutive tiles measured faster (the dequeue balances larger launches)
    ws.counters[3] = a.grad && total_items <= 2 * a.grid ? 1 : 0;
  }
}

// Image extent of a capsule (segment q0-q1, radius r) as the hull of its two end spheres'
// extents: the planes x = a z through the camera that touch a sphere with centre (X, Y, Z),
// Z > r, have a = (X Z -/+ r sqrt(X^2 + Z^2 - r^2)) / (Z^2 - r^2), and likewise in y.  The
// capsule's support along a plane normal is the larger of its end spheres', so no interior
// point lies outside.  Writes pixel coordinates (u0, u1, v0, v1), padded by a quarter pixel
// for the FP32 rounding; returns false when a sphere reaches the camera plane.  The culling
// geometry takes the hardware reciprocal and square root (errors of about 1e-7 relative,
// 1e-4 pixel at most, far inside the pads; the quotients' range-safe sequences made the
// primitive set-up a long chain of latencies).
__device__ bool capsule_extent(const double* q0, const double* q1, double r,
                               const FrameSlot& fs, float* e) {
  float amin = INFINITY, amax = -INFINITY, bmin = INFINITY, bmax = -INFINITY;
  const float rr = (float)r;
  for (int j = 0; j < 2; ++j) {
    const double* q = j ? q1 : q0;
    const float X = (float)q[0], Y = (float)q[1], Z = (float)q[2];
    if (!(Z > 1.001f * rr + 1.0f)) return false;
    const float den = (Z - rr) * (Z + rr);
    const float inv = fast_rcp(den);
    const float hx = rr * fast_sqrt(fmaf(X, X, den)), hy = rr * fast_sqrt(fmaf(Y, Y, den));
    const float xz = X * Z, yz = Y * Z;
    amin = fminf(amin, (xz - hx) * inv);
    amax = fmaxf(amax, (xz + hx) * inv);
    bmin = fminf(bmin, (yz - hy) * inv);
    bmax = fmaxf(bmax, (yz + hy) * inv);
  }
  e[0] = fmaf(fs.fx, amin, fs.cx) - 0.25f;
  e[1] = fmaf(fs.fx, amax, fs.cx) + 0.25f;
  e[2] = fmaf(fs.fy, bmin, fs.cy) - 0.25f;
  e[3] = fmaf(fs.fy, bmax, fs.cy) + 0.25f;
  return true;
}

// Bounding disc of the image of a sphere (centre q, radius r, q.z > r): the image is an
// ellipse whose major axis points away from the principal point and spans the normalised
// radii tan(theta - alpha) .. tan(theta + alpha), theta being the angle of q from the optical
// axis and sin(alpha) = r / |q|.  Its centre and semi-major axis, in pixels (the larger focal
// length for the radius), give a disc that contains it.
__device__ void sphere_image_disc(const double* q, double r, const FrameSlot& fs, float* D,
                                  float& rho) {
  const float X = (float)q[0], Y = (float)q[1], Z = (float)q[2], R = (float)r;
  const float rad = fast_sqrt(fmaf(X, X, Y * Y));
  const float inv_n = __builtin_amdgcn_rsqf(fmaf(rad, rad, Z * Z));
  const float st = rad * inv_n, ct = Z * inv_n, sa = R * inv_n;
  const float ca = fast_sqrt(fmaxf(0.0f, 1.0f - sa * sa));
  const float tp = fmaf(st, ca, ct * sa) * fast_rcp(fmaf(ct, ca, -st * sa));   // tan(theta + alpha)
  const float tm = fmaf(st, ca, -ct * sa) * fast_rcp(fmaf(ct, ca, st * sa));   // tan(theta - alpha)
  const float m = 0.5f * (tp + tm), h = 0.5f * (tp - tm);
  const float ir = fast_rcp(rad);
  const float ex = rad > 0.0f ? X * ir : 1.0f, ey = rad > 0.0f ? Y * ir : 0.0f;
  D[0] = fmaf(fs.fx, m * ex, fs.cx);
  D[1] = fmaf(fs.fy, m * ey, fs.cy);
  rho = h * fmaxf(fs.fx, fs.fy);
}

// Farthest pixel centre of an 8x8 tile from the tile's centre: 3.5 sqrt(2) pixels.
constexpr float kTileHalfDiag = 4.9498f;

// ------------------------------------------------------------------------------------
// forward kinematics prologue: one wavefront per particle (FP64 inside)

// One primitive's model data (in type order: slot o holds primitive prim_order[o]).
struct PrimIn {
  int k, seg, type, root;
  double frame[12];
  double size[3];
  double inv2[3];
};

__device__ __forceinline__ void load_prim(const DevModel* __restrict__ G, int o, PrimIn& q) {
  const int k = G->prim_order[o];
  q.k = k;
  q.seg = G->prim_seg[k];
  q.type = G->prim_type[k];
  q.root = G->prim_root[k];
  for (int i = 0; i < 12; ++i) q.frame[i] = G->prim_frame[k][i];
  for (int i = 0; i < 3; ++i) {
    q.size[i] = G->prim_size[k][i];
    q.inv2[i] = G->prim_inv2[k][i];
  }
}

// WPP wavefronts per particle: 1, or 2 for models of more than 64 primitives, whose set-up then
// takes one round on each of the two wavefronts instead of two rounds on one (the second
// wavefront waits for the first one's trigonometry and chains at the barriers, and sets up
// primitives 64..127; the first writes the record).
template <int WPP>
__global__ __launch_bounds__(kBlock, 4) void fk_kernel(EvalArgs a, Workspace ws) {
  __shared__ double s_T[kWavesPerBlock][HT_MAX_SEG][12];
  __shared__ double s_h[kWavesPerBlock][HT_MAX_DOF];
  __shared__ double s_sin[kWavesPerBlock][HT_MAX_DOF], s_cos[kWavesPerBlock][HT_MAX_DOF];
  // the wavefront index as a scalar, so that everything per particle below is wave-uniform
  // (scalar instructions and branches)
  const int lane = threadIdx.x & (kWave - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  constexpr int kPpb = kWavesPerBlock / WPP;     // particles per workgroup
  const int pb = w / WPP, h = w % WPP;           // particle in the workgroup, its wavefront
  const int n_total = a.n_frames * a.n_particles;
  const int p = blockIdx.x * kPpb + pb;
  const bool active = p < n_total;
  const int n_dof = a.n_dof, n_seg = a.n_seg, n_prim = a.n_prim;
  const DevModel* __restrict__ G = a.model;
  // Every load that depends on the particle alone is issued first, together and with clamped
  // indices (a load behind a branch, or issued after another whose result is awaited, adds a
  // memory latency to this latency-bound kernel): this lane's pose parameter, the frame's
  // slot and stop flag, the candidate's active flag and this lane's collision pair.
  const int pc = min(p, n_total - 1);
  const int f = pc / a.n_particles;
  const float x_lane = a.poses[(size_t)pc * n_dof + min(lane, n_dof - 1)];
  const int slot_raw = a.frame_slots[f];
  const int stop_raw = a.frame_stop ? a.frame_stop[f] : 0;
  const int act_raw = a.active ? a.active[pc / a.active_div] : 1;
  const int kc_i = max(lane - (kWave - HT_MAX_KC), 0);
  const int kc_a = G->kc_a[kc_i], kc_b = G->kc_b[kc_i];
  // the kinematic tables (everything before the primitive tables), staged by one coalesced
  // copy with all its loads in flight at once: the tree walk would otherwise wait on long
  // chains of dependent global loads.  The primitive tables are read from global memory by the
  // lane that sets a primitive up, issued here so that their latency overlaps the
  // trigonometry and the tree walk.
  constexpr int kSegBytes = ((int)offsetof(DevModel, prim_type) + 15) / 16 * 16;
  static_assert(kSegBytes <= (int)sizeof(DevModel), "copy stays inside the model");
  __shared__ __align__(16) unsigned char s_model[kSegBytes];
  {
    constexpr int kN = kSegBytes / 16, kIt = (kN + kBlock - 1) / kBlock;
    const uint4* src4 = reinterpret_cast<const uint4*>(a.model);
    uint4* dst4 = reinterpret_cast<uint4*>(s_model);
    uint4 v[kIt];
#pragma unroll
    for (int j = 0; j < kIt; ++j) v[j] = src4[min((int)threadIdx.x + j * kBlock, kN - 1)];
#pragma unroll
    for (int j = 0; j < kIt; ++j)
      if ((int)threadIdx.x + j * kBlock < kN) dst4[threadIdx.x + j * kBlock] = v[j];
  }
  // only the members before prim_type may be read through M
  const DevModel& M = *reinterpret_cast<const DevModel*>(s_model);
  __shared__ int s_fin[kWavesPerBlock];
  PrimIn pin0;
  if (active && lane + h * kWave < n_prim) load_prim(G, lane + h * kWave, pin0);

  // every angle's sine and cosine at once (one lane per pose parameter, n_dof <= 64), so the
  // tree walk below is trigonometry-free
  static_assert(HT_MAX_DOF <= kWave, "one lane per pose parameter");
  bool finite = true;
  if (active && h == 0 && lane < n_dof) {
    const float x = x_lane;
    s_h[pb][lane] = (double)x;
    finite = isfinite(x);
    double sv = 0.0, cv = 1.0;
    if (finite) sincos((double)x, &sv, &cv);
    s_sin[pb][lane] = sv;
    s_cos[pb][lane] = cv;
  }
  finite = __ballot(!finite) == 0ull;
  if (h == 0 && lane == 0) s_fin[pb] = finite ? 1 : 0;
  const int slot = active ? slot_raw : -1;
  const bool slot_ok = active && slot >= 0 && slot < HT_MAX_SLOTS && a.slots[slot].set;
  if (active && !slot_ok && h == 0 && lane == 0 && a.dev_errors)
    atomicOr(a.dev_errors, HT_DEVERR_UNSET_SLOT);
  // a particle of a stopped frame (tracking stop rule), or a candidate of a refined particle
  // that has stopped refining, is neither cast nor written
  const bool skip = active && (stop_raw != 0 || act_raw == 0);
  __syncthreads();
  // the first wavefront's finiteness test, for every wavefront of the particle
  if (WPP > 1) finite = __builtin_amdgcn_readfirstlane(s_fin[pb]) != 0;
  const bool valid = slot_ok && finite && !skip;
  // the slot's background sums, needed only by the record written at the end: loaded after
  // the barrier as global loads (which no barrier waits for), so that their two dependent
  // latencies overlap the tree walk
  double bg_td = 0.0, bg_or = 0.0;
  if (slot_ok && h == 0) {
    const double* tot = a.slots[slot].totals;
    bg_td = global_ptr(tot)[0];
    bg_or = global_ptr(tot)[1];
  }

  // segment transforms, T_s = W L_root ... L_parent(s) L_s with L_s = Off_s Rot(a1, q1)
  // Rot(a2, q2) and W the wrist of s's tree: every lane forms its own L_s once and stages it
  // in LDS, then multiplies its ancestors' staged transforms right to left (the tree is
  // shallow: palm and three phalanges), so no joint rotation is computed twice.
  __shared__ double s_L[kWavesPerBlock][HT_MAX_SEG][12];
  const bool seg_lane = valid && h == 0 && lane < n_seg;
  if (seg_lane) {
    double Lm[12];
    for (int i = 0; i < 12; ++i) Lm[i] = M.seg_off[lane][i];
    for (int j = 0; j < 2; ++j) {
      const int dof = M.seg_dof[lane][j];
      if (dof >= 0) post_rotate(Lm, M.seg_axis[lane][j], s_sin[pb][dof], s_cos[pb][dof]);
    }
    for (int i = 0; i < 12; ++i) s_L[pb][lane][i] = Lm[i];
  }
  __syncthreads();
  if (seg_lane) {
    double P[12];
    for (int i = 0; i < 12; ++i) P[i] = s_L[pb][lane][i];
    int q = M.seg_parent[lane], root = lane;
    while (q >= 0) {
      double Q[12];
      mul34(s_L[pb][q], P, Q);
      for (int i = 0; i < 12; ++i) P[i] = Q[i];
      root = q;
      q = M.seg_parent[q];
    }
    // wrist: Trans(x, y, z) Rz(tz) Ry(ty) Rx(tx)
    const int b = M.seg_root_dof[root];
    const double* hq = &s_h[pb][b];
    const double sx = s_sin[pb][b + 3], cx = s_cos[pb][b + 3];
    const double sy = s_sin[pb][b + 4], cy = s_cos[pb][b + 4];
    const double sz = s_sin[pb][b + 5], cz = s_cos[pb][b + 5];
    const double Rzy[9] = {cz * cy, -sz, cz * sy, sz * cy, cz, sz * sy, -sy, 0.0, cy};
    double W0[12];
    W0[0] = Rzy[0];
    W0[1] = Rzy[1] * cx + Rzy[2] * sx;
    W0[2] = -Rzy[1] * sx + Rzy[2] * cx;
    W0[3] = hq[0];
    W0[4] = Rzy[3];
    W0[5] = Rzy[4] * cx + Rzy[5] * sx;
    W0[6] = -Rzy[4] * sx + Rzy[5] * cx;
    W0[7] = hq[1];
    W0[8] = Rzy[6];
    W0[9] = Rzy[7] * cx + Rzy[8] * sx;
    W0[10] = -Rzy[7] * sx + Rzy[8] * cx;
    W0[11] = hq[2];
    if (root == lane) {
      // wrist dofs: translations along camera axes; rotations about Rz Ry e_x, Rz e_y, e_z
      // through the wrist position
      float* df = ws.dof_frame + ((size_t)p * n_dof + b) * 8;
      for (int i = 0; i < 3; ++i) {
        float* f = df + i * 8;
        f[0] = 1.0f;
        f[1] = i == 0;
        f[2] = i == 1;
        f[3] = i == 2;
        f[4] = f[5] = f[6] = f[7] = 0.0f;
      }
      const double ax[3][3] = {{W0[0], W0[4], W0[8]}, {-sz, cz, 0.0}, {0.0, 0.0, 1.0}};
      for (int i = 0; i < 3; ++i) {
        float* f = df + (3 + i) * 8;
        f[0] = 0.0f;
        f[1] = (float)ax[i][0];
        f[2] = (float)ax[i][1];
        f[3] = (float)ax[i][2];
        f[4] = (float)hq[0];
        f[5] = (float)hq[1];
        f[6] = (float)hq[2];
        f[7] = 0.0f;
      }
    }
    double T[12];
    mul34(W0, P, T);
    for (int i = 0; i < 12; ++i) s_T[pb][lane][i] = T[i];
    // joint axes in the camera frame: the second joint's axis is R_s a2; the first's is
    // R_s Rot(a2, q2)^T a1 (each rotation leaves its own axis fixed); both pass through the
    // segment origin
    const int dof1 = M.seg_dof[lane][0], dof2 = M.seg_dof[lane][1];
    for (int j = 0; j < 2; ++j) {
      const int dof = j ? dof2 : dof1;
      if (dof < 0) continue;
      double v[3] = {M.seg_axis[lane][j][0], M.seg_axis[lane][j][1], M.seg_axis[lane][j][2]};
      if (j == 0 && dof2 >= 0) {
        // Rot(a2, q2)^T v = c v - s (a2 x v) + (1 - c)(a2 . v) a2
        const double* a2 = M.seg_axis[lane][1];
        const double sn = s_sin[pb][dof2], cs = s_cos[pb][dof2];
        const double dt = (1.0 - cs) * (a2[0] * v[0] + a2[1] * v[1] + a2[2] * v[2]);
        const double cr[3] = {a2[1] * v[2] - a2[2] * v[1], a2[2] * v[0] - a2[0] * v[2],
                              a2[0] * v[1] - a2[1] * v[0]};
        for (int i = 0; i < 3; ++i) v[i] = cs * v[i] - sn * cr[i] + dt * a2[i];
      }
      float* f = ws.dof_frame + ((size_t)p * n_dof + dof) * 8;
      f[0] = 0.0f;
      for (int i = 0; i < 3; ++i) {
        f[1 + i] = (float)(T[i * 4 + 0] * v[0] + T[i * 4 + 1] * v[1] + T[i * 4 + 2] * v[2]);
        f[4 + i] = (float)T[i * 4 + 3];
      }
      f[7] = 0.0f;
    }
    float* so = ws.seg_org + ((size_t)p * n_seg + lane) * 4;
    so[0] = (float)T[3];
    so[1] = (float)T[7];
    so[2] = (float)T[11];
    so[3] = 0.0f;
  }
  // collision terms of Eq. 5, one per spare lane (summed in order below)
  __shared__ double s_kc[kWavesPerBlock][HT_MAX_KC];
  // (every pair slot is written, zero past the model's pairs, so the record below sums all of
  // them without a branch per slot)
  if (valid && h == 0 && lane >= kWave - HT_MAX_KC) {
    const int i = lane - (kWave - HT_MAX_KC);
    double v = 0.0;
    if (i < M.n_kc) v = fmax(-(s_h[pb][kc_a] - s_h[pb][kc_b]), 0.0);
    s_kc[pb][i] = v;
  }
  __syncthreads();

  // primitive records and screen boxes, in type order (a wave's lanes then take at most two
  // of the three set-up paths per round); per-tree unions of the primitive boxes (u0, v0 minima; u1, v1 maxima), accumulated with
  // LDS atomics (cheaper than sixteen wave reductions)
  __shared__ int s_rect[kWavesPerBlock][kMaxRects][4];
  if (h == 0 && lane < kMaxRects * 4)
    s_rect[pb][lane >> 2][lane & 3] = (lane & 1) ? INT_MIN : INT_MAX;
  __syncthreads();
  if (valid) {
    const FrameSlot fs = a.slots[slot];
    for (int o = lane + h * kWave; o < n_prim; o += kWave * WPP) {
      PrimIn pin;
      if (o == lane + h * kWave) pin = pin0;
      else load_prim(G, o, pin);
      const int k = pin.k;
      const int s = pin.seg;
      double F[12];
      mul34(s_T[pb][s], pin.frame, F);
      const double* sz = pin.size;
      const int typ = pin.type;
      float rec[kRec];
      for (int i = 0; i < kRec; ++i) rec[i] = 0.0f;
      const double c[3] = {F[3], F[7], F[11]};
      const double* T = s_T[pb][s];
      split(c[0], rec[0], rec[4]);
      split(c[1], rec[1], rec[5]);
      split(c[2], rec[2], rec[6]);
      rec[12] = (float)(c[0] - T[3]);
      rec[13] = (float)(c[1] - T[7]);
      rec[14] = (float)(c[2] - T[11]);
      rec[15] = __int_as_float(s);
      // the frame's columns are unit vectors to FP64 rounding, so the axis needs no
      // normalisation
      const double u[3] = {F[2], F[6], F[10]};
      // terms of the ray tests that do not depend on the pixel are formed here once, as the
      // same FP32 operations the tests would perform (so the tests' results are unchanged):
      // products with the ray's z component sz
      if (typ == HT_SPHERE) {
        rec[3] = (float)(sz[0] * sz[0]);
        rec[7] = fs.sz * rec[2];
      } else if (typ == HT_CYLINDER || typ == HT_CONE) {
        // circular cylinder (radius r0) or truncated cone (radius r0 at s = 0, r1 at s = L)
        const double r0 = sz[0], L = sz[1], r1 = typ == HT_CONE ? sz[2] : sz[0];
        rec[3] = typ == HT_CONE ? (float)r0 : (float)(r0 * r0);
        rec[7] = (float)L;
        rec[8] = (float)u[0];
        rec[9] = (float)u[1];
        rec[10] = (float)u[2];
        rec[11] = typ == HT_CONE ? (float)((r1 - r0) / L)
                                 : (float)(c[0] * u[0] + c[1] * u[1] + c[2] * u[2]);
        if (typ == HT_CYLINDER) {
          // sz uz, then the part of the cap centre perpendicular to the axis (q = c - (c.u) u:
          // q_z sz, q_x, q_y), whose product with d is the side reference's numerator
          const double cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
          rec[16] = fs.sz * rec[10];
          rec[17] = fs.sz * (float)(c[2] - cu * u[2]);
          rec[18] = (float)(c[0] - cu * u[0]);
          rec[19] = (float)(c[1] - cu * u[1]);
        }
      } else {
        // ellipsoid: Q = R diag(1/s^2) R^T with R the rotation part of F; elliptic cylinder:
        // the same without the axis term, Q = ex ex^T / a^2 + ey ey^T / b^2
        const bool ecyl = typ == HT_ECYLINDER;
        const double inv[3] = {pin.inv2[0], ecyl ? pin.inv2[2] : pin.inv2[1],
                               ecyl ? 0.0 : pin.inv2[2]};
        double Q[6] = {0, 0, 0, 0, 0, 0};
        for (int j = 0; j < 3; ++j) {
          const double r0 = F[0 * 4 + j], r1 = F[1 * 4 + j], r2 = F[2 * 4 + j];
          Q[0] += inv[j] * r0 * r0;
          Q[1] += inv[j] * r0 * r1;
          Q[2] += inv[j] * r0 * r2;
          Q[3] += inv[j] * r1 * r1;
          Q[4] += inv[j] * r1 * r2;
          Q[5] += inv[j] * r2 * r2;
        }
        rec[3] = (float)Q[0];
        rec[7] = (float)Q[1];
        rec[8] = (float)Q[2];
        rec[9] = (float)Q[3];
        rec[10] = (float)Q[4];
        rec[11] = (float)Q[5];
        if (ecyl) {
          rec[16] = (float)u[0];
          rec[17] = (float)u[1];
          rec[18] = (float)u[2];
          rec[19] = (float)sz[1];
        } else {
          rec[16] = rec[8] * fs.sz;
          rec[17] = rec[10] * fs.sz;
          rec[18] = rec[11] * fs.sz;
        }
      }
      float4* dst = reinterpret_cast<float4*>(ws.recs + ((size_t)p * n_prim + k) * kRec);
      for (int i = 0; i < kRec / 4; ++i)
        dst[i] = make_float4(rec[4 * i], rec[4 * i + 1], rec[4 * i + 2], rec[4 * i + 3]);

      // conservative pixel box of an axis-aligned 3D box of the solid, in FP32 (its rounding,
      // about 1e-4 mm, is covered by a quarter-pixel pad)
      float lo3[3], hi3[3];
      {
        const float cf[3] = {(float)c[0], (float)c[1], (float)c[2]};
        const float uf[3] = {(float)u[0], (float)u[1], (float)u[2]};
        const float s0 = (float)sz[0], s1 = (float)sz[1], s2 = (float)sz[2];
        if (typ == HT_SPHERE) {
          for (int i = 0; i < 3; ++i) {
            lo3[i] = cf[i] - s0;
            hi3[i] = cf[i] + s0;
          }
        } else if (typ == HT_CYLINDER || typ == HT_CONE) {
          // the solid is the convex hull of its two cap discs
          const float r1 = typ == HT_CONE ? s2 : s0;
          for (int i = 0; i < 3; ++i) {
            const float sn = fast_sqrt(fmaxf(0.0f, 1.0f - uf[i] * uf[i]));
            const float c1 = fmaf(s1, uf[i], cf[i]);
            lo3[i] = fminf(cf[i] - s0 * sn, c1 - r1 * sn);
            hi3[i] = fmaxf(cf[i] + s0 * sn, c1 + r1 * sn);
          }
        } else {
          const bool ecyl = typ == HT_ECYLINDER;
          for (int i = 0; i < 3; ++i) {
            const float f0 = (float)F[i * 4 + 0] * s0;
            const float f1 = (float)F[i * 4 + 1] * (ecyl ? s2 : s1);
            const float f2 = ecyl ? 0.0f : (float)F[i * 4 + 2] * s2;
            const float e = fast_sqrt(fmaf(f0, f0, fmaf(f1, f1, f2 * f2)));
            const float c1 = ecyl ? fmaf(s1, uf[i], cf[i]) : cf[i];
            lo3[i] = fminf(cf[i], c1) - e;
            hi3[i] = fmaxf(cf[i], c1) + e;
          }
        }
      }
      int4 box;
      if (!(lo3[2] > 1.0f)) {
        box = make_int4(0, fs.W - 1, 0, fs.H - 1);
      } else if (fs.bg > 0.0f && lo3[2] >= fs.bg) {
        box = make_int4(1, 0, 1, 0);   // entirely behind the background plane
      } else {
        const float izl = fast_rcp(lo3[2]), izh = fast_rcp(hi3[2]);
        const float xmin = fminf(lo3[0] * izl, lo3[0] * izh);
        const float xmax = fmaxf(hi3[0] * izl, hi3[0] * izh);
        const float ymin = fminf(lo3[1] * izl, lo3[1] * izh);
        const float ymax = fmaxf(hi3[1] * izl, hi3[1] * izh);
        const float lim = 1.0e6f;
        const float u0 = fminf(fmaxf(floorf(fmaf(fs.fx, xmin, fs.cx) - 0.25f), -1.0f), lim);
        const float u1 = fminf(fmaxf(ceilf(fmaf(fs.fx, xmax, fs.cx) + 0.25f), -1.0f), lim);
        const float v0 = fminf(fmaxf(floorf(fmaf(fs.fy, ymin, fs.cy) - 0.25f), -1.0f), lim);
        const float v1 = fminf(fmaxf(ceilf(fmaf(fs.fy, ymax, fs.cy) + 0.25f), -1.0f), lim);
        box.x = max((int)u0, 0);
        box.y = min((int)u1, fs.W - 1);
        box.z = max((int)v0, 0);
        box.w = min((int)v1, fs.H - 1);
      }
      float4 cap = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      float2 capr = make_float2(0.0f, INFINITY);
      if (a.cull && box.x <= box.y && box.z <= box.w) {
        // tighter: the exact image extent of a bounding capsule (segment q0-q1, radius cr),
        // intersected with the box above (the capsule reaches past a cylinder's ends).  An
        // ellipsoid with semi-axes a >= b >= c lies in the capsule along its a-axis from
        // -(a - b) to (a - b) with radius b.
        double q0[3], q1[3], cr;
        if (typ == HT_SPHERE) {
          for (int i = 0; i < 3; ++i) q0[i] = q1[i] = c[i];
          cr = sz[0];
        } else if (typ == HT_CYLINDER || typ == HT_CONE || typ == HT_ECYLINDER) {
          for (int i = 0; i < 3; ++i) {
            q0[i] = c[i];
            q1[i] = c[i] + sz[1] * u[i];
          }
          cr = typ == HT_CYLINDER ? sz[0] : fmax(sz[0], sz[2]);
        } else {
          // longest semi-axis ia (the first of equal ones) by selects, so that no array is
          // indexed at run time
          const double s0 = sz[0], s1 = sz[1], s2 = sz[2];
          const int i01 = s1 > s0 ? 1 : 0;
          const double m01 = i01 ? s1 : s0;
          const int ia = s2 > m01 ? 2 : i01;
          const double sa = ia == 2 ? s2 : m01;
          const double b2 = ia == 0 ? fmax(s1, s2) : (ia == 1 ? fmax(s0, s2) : fmax(s0, s1));
          const double hl = sa - b2;
          for (int i = 0; i < 3; ++i) {
            const double ax = ia == 0 ? F[i * 4] : (ia == 1 ? F[i * 4 + 1] : F[i * 4 + 2]);
            q0[i] = c[i] - hl * ax;
            q1[i] = c[i] + hl * ax;
          }
          cr = b2;
        }
        cr += 0.01 + 1e-6 * (fabs(c[0]) + fabs(c[1]) + fabs(c[2]));
        float e[4];
        if (capsule_extent(q0, q1, cr, fs, e)) {
          const float lim = 1.0e6f;
          const int u0 = (int)fminf(fmaxf(floorf(e[0]), -1.0f), lim);
          const int u1 = (int)fminf(fmaxf(ceilf(e[1]), -1.0f), lim);
          const int v0 = (int)fminf(fmaxf(floorf(e[2]), -1.0f), lim);
          const int v1 = (int)fminf(fmaxf(ceilf(e[3]), -1.0f), lim);
          box.x = max(box.x, u0);
          box.y = min(box.y, u1);
          box.z = max(box.z, v0);
          box.w = min(box.w, v1);
          // the capsule's image is the convex hull of its end spheres' images, so it lies
          // within the larger of their bounding discs' radii of the segment joining the
          // discs' centres; a tile is reached when its centre is within that radius plus the
          // tile's half-diagonal (padded for the FP32 rounding)
          float D0[2], D1[2], r0, r1;
          sphere_image_disc(q0, cr, fs, D0, r0);
          sphere_image_disc(q1, cr, fs, D1, r1);
          const float reach = fmaxf(r0, r1) * 1.0001f + kTileHalfDiag + 0.5f;
          const float dx = D1[0] - D0[0], dy = D1[1] - D0[1];
          const float vv = fmaf(dx, dx, dy * dy);
          // (the first disc's centre stored less the tile-centre offset 3.5 px, so the ray
          // cast measures from a tile's corner pixel index)
          cap = make_float4(D0[0] - 3.5f, D0[1] - 3.5f, dx, dy);
          capr = make_float2(vv > 0.0f ? fast_rcp(vv) : 0.0f, reach * reach);
        }
      }
      ws.caps[(size_t)p * n_prim + k] = cap;
      ws.capr[(size_t)p * n_prim + k] = capr;
      if (box.x > box.y || box.z > box.w) box = make_int4(1, 0, 1, 0);
      ws.boxes[(size_t)p * n_prim + k] = box;
      if (box.x <= box.y) {
        int* rq = s_rect[pb][pin.root];
        atomicMin(rq + 0, box.x);
        atomicMax(rq + 1, box.y);
        atomicMin(rq + 2, box.z);
        atomicMax(rq + 3, box.w);
      }
    }
  }
  __syncthreads();
  if (active && h == 0) {
    // every lane computes the record from wave-uniform values (scalar instructions); lane 0
    // stores it
    PInfo pi{};
    pi.slot = slot_ok ? slot : -1;
    pi.valid = valid ? 1 : 0;
    pi.skip = skip ? 1 : 0;
    double kc = 0.0;
    int kc_mask = 0;
    if (valid) {
      // the terms are differences of FP32 values: their FP64 sum is exact in any order
#pragma unroll
      for (int i = 0; i < HT_MAX_KC; ++i) {
        const double v = s_kc[pb][i];
        kc += v;
        kc_mask |= v > 0.0 ? 1 << i : 0;
      }
    }
    pi.kc = (float)kc;
    pi.kc_mask = kc_mask;
    pi.bg_td = bg_td;
    pi.bg_or = bg_or;
    // one tile rectangle per tree, as (x0, y0, x1, y1) inclusive; overlapping ones are merged
    // (into the lower index) so that no tile is visited twice.  Every index below is a
    // compile-time constant, so the rectangles stay in registers.
    int4 R[kMaxRects];
    bool live[kMaxRects];
#pragma unroll
    for (int r = 0; r < kMaxRects; ++r) {
      const int x0 = __builtin_amdgcn_readfirstlane(s_rect[pb][r][0]);
      const int x1 = __builtin_amdgcn_readfirstlane(s_rect[pb][r][1]);
      const int y0 = __builtin_amdgcn_readfirstlane(s_rect[pb][r][2]);
      const int y1 = __builtin_amdgcn_readfirstlane(s_rect[pb][r][3]);
      live[r] = valid && x0 <= x1;
      R[r] = make_int4(x0 / kTile, y0 / kTile, x1 / kTile, y1 / kTile);
    }
    // a sweep without a merge is the fixed point; each earlier sweep merges at least once.
    // Only the model's trees can hold rectangles (a one-hand model needs no merge, two hands
    // one pair test per sweep); the bounds are wave-uniform, so the skipped tests cost nothing.
    const int nr = M.n_roots;
#pragma unroll
    for (int sweep = 0; sweep < kMaxRects - 1; ++sweep) {
      if (sweep + 1 >= nr) break;
#pragma unroll
      for (int i = 0; i < kMaxRects; ++i) {
#pragma unroll
        for (int j = i + 1; j < kMaxRects; ++j) {
          if (j >= nr) break;
          if (live[i] && live[j] && R[i].x <= R[j].z && R[j].x <= R[i].z &&
              R[i].y <= R[j].w && R[j].y <= R[i].w) {
            R[i] = make_int4(min(R[i].x, R[j].x), min(R[i].y, R[j].y), max(R[i].z, R[j].z),
                             max(R[i].w, R[j].w));
            live[j] = false;
          }
        }
      }
    }
    int n = 0, nt = 0;
#pragma unroll
    for (int r = 0; r < kMaxRects; ++r) {
      if (live[r]) {
        const int tw = R[r].z - R[r].x + 1, th = R[r].w - R[r].y + 1;
        const int4 q = make_int4(R[r].x, R[r].y, tw, th);
#pragma unroll
        for (int d = 0; d <= r; ++d)
          if (d == n) pi.rect[d] = q;
        ++n;
        nt += tw * th;
      }
    }
    pi.n_rects = n;
    pi.n_tiles = nt;
    if (lane == 0) {
      ws.pinfo[p] = pi;
      ws.tiles[p] = skip ? -1 : nt;
    }
  }
}

// The work list is built by its own one-workgroup launch: folding it into the kinematics
// kernel as "the last workgroup to finish builds it" needs a device-scope fence in every
// workgroup, which on a multi-XCD part (one L2 per XCD) costs far more than a launch.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void sched_kernel(EvalArgs a, Workspace ws) {
  schedule_items<BLOCK>(a, a.n_frames * a.n_particles, ws);
}

// ------------------------------------------------------------------------------------
// per-pixel background for the debug images

__global__ __launch_bounds__(kBlock) void debug_fill_kernel(ht_debug dbg, size_t n, float bg) {
  const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  if (dbg.depth) dbg.depth[i] = bg > 0.0f ? bg : 0.0f;
  if (dbg.hit) dbg.hit[i] = 0;
  if (dbg.rm) dbg.rm[i] = 0;
  if (dbg.winner) dbg.winner[i] = -1;
  if (dbg.margin) dbg.margin[i] = -INFINITY;
}

// ------------------------------------------------------------------------------------
// ray-primitive intersections (FP32; centres carried as hi + lo pairs)
//
// The ray is x = t d with d = ((u - cx) sx, (v - cy) sy, sz), formed in FP32 (to within a
// rounding of its components) and then taken as exact; depth = t sz.  Every test first forms
// the offset of the ray's closest-approach point from the primitive centre, which is accurate
// because the tests use that same FP32 d and the centre is a double-float pair; the
// hit decision and the half-chord then come from small, well-conditioned quantities.

// A test may report a miss as ok with a NaN entry (the half-chord of a ray that misses is the
// square root of a negative number): the caller compares entries as unsigned integers, and a
// NaN's bit pattern exceeds +inf's, so such an entry is never taken.
struct Hit {
  float t;        // ray parameter of the entry point
  bool ok;
  float nx, ny, nz;   // outward normal direction at the entry (unnormalised)
  float rx, ry, rz;   // entry point minus the primitive reference point
  float m;            // ray-surface margin (debug images only, MRG)
};

// Margin of a capped side and its two caps (the survey's rule, as the oracle computes it): a
// side root's slack is the least of the radial slack and the axial slacks s/L, (L - s)/L at the
// root (the radial slack alone when the ray misses the side); a cap's slack is its disc's
// radial slack at the cap point; the margin is the largest of the four.  radial: the side's
// radial slack; s_a, s_b: axial coordinates of the two side roots; cap0, cap1: the caps'.
__device__ __forceinline__ float capped_margin(float radial, bool side_hit, float s_a, float s_b,
                                               float L, float cap0, float cap1) {
  const float iL = 1.0f / L;
  const float sa = fminf(radial, fminf(s_a * iL, (L - s_a) * iL));
  const float sb = fminf(radial, fminf(s_b * iL, (L - s_b) * iL));
  const float side = side_hit ? fmaxf(sa, sb) : radial;
  return fmaxf(fmaxf(side, cap0), cap1);
}

template <bool GRAD, bool MRG = false>
__device__ __forceinline__ void sphere_test(const float* r, float dx, float dy, float dz,
                                            float inv_dd, Hit& h) {
  const float b = fmaf(dx, r[0], fmaf(dy, r[1], r[7]));   // r[7] = dz r[2]
  const float t0 = b * inv_dd;
  const float vx = fmaf(t0, dx, -r[0]) - r[4];
  const float vy = fmaf(t0, dy, -r[1]) - r[5];
  const float vz = fmaf(t0, dz, -r[2]) - r[6];
  const float rho2 = fmaf(vx, vx, fmaf(vy, vy, vz * vz));
  const float h2 = r[3] - rho2;
  h.ok = true;   // a miss (h2 < 0) has a NaN entry
  const float hs = fast_sqrt(h2 * inv_dd);
  h.t = t0 - hs;
  if (MRG) h.m = h2 / r[3];
  if (GRAD) {
    h.rx = fmaf(-hs, dx, vx);
    h.ry = fmaf(-hs, dy, vy);
    h.rz = fmaf(-hs, dz, vz);
    h.nx = h.rx;
    h.ny = h.ry;
    h.nz = h.rz;
  }
}

template <bool GRAD, bool MRG = false>
__device__ __forceinline__ void ellipsoid_test(const float* r, float dx, float dy, float dz,
                                               Hit& h) {
  const float q00 = r[3], q01 = r[7], q02 = r[8], q11 = r[9], q12 = r[10], q22 = r[11];
  // r[16..18] = (q02, q12, q22) dz
  const float qdx = fmaf(q00, dx, fmaf(q01, dy, r[16]));
  const float qdy = fmaf(q01, dx, fmaf(q11, dy, r[17]));
  const float qdz = fmaf(q02, dx, fmaf(q12, dy, r[18]));
  const float dqd = fmaf(dx, qdx, fmaf(dy, qdy, dz * qdz));
  const float cqd = fmaf(r[0], qdx, fmaf(r[1], qdy, r[2] * qdz));
  const float inv = fast_rcp(dqd);
  const float t0 = cqd * inv;
  const float vx = fmaf(t0, dx, -r[0]) - r[4];
  const float vy = fmaf(t0, dy, -r[1]) - r[5];
  const float vz = fmaf(t0, dz, -r[2]) - r[6];
  const float qvx = fmaf(q00, vx, fmaf(q01, vy, q02 * vz));
  const float qvy = fmaf(q01, vx, fmaf(q11, vy, q12 * vz));
  const float qvz = fmaf(q02, vx, fmaf(q12, vy, q22 * vz));
  // t0 carries the rounding of c.Qd; the linear term B re-centres the chord exactly
  const float B = fmaf(vx, qdx, fmaf(vy, qdy, vz * qdz));
  const float cc = -B * inv;
  const float m = fmaf(B, B * inv, 1.0f - fmaf(vx, qvx, fmaf(vy, qvy, vz * qvz)));
  h.ok = true;   // a miss (m < 0) has a NaN entry
  const float tin = cc - fast_sqrt(m * inv);
  h.t = t0 + tin;
  if (MRG) h.m = m;
  if (GRAD) {
    h.rx = fmaf(tin, dx, vx);
    h.ry = fmaf(tin, dy, vy);
    h.rz = fmaf(tin, dz, vz);
    h.nx = fmaf(tin, qdx, qvx);
    h.ny = fmaf(tin, qdy, qvy);
    h.nz = fmaf(tin, qdz, qvz);
  }
}

// Closed cylinder as the intersection of the infinite cylinder and the slab 0 <= s <= L:
// both intervals are expressed as offsets from the reference parameter t_r (the closest
// approach to the axis), so the hit test compares small accurate numbers.
//
// Margin of the cylinder at one pixel (debug images): offsets tau from t_r, radius^2 at tau
// is rho2 + 2 tau B + tau^2 A, axial coordinate a3 + tau da.
__device__ __forceinline__ float cylinder_margin(const float* r, bool par, float A, float B,
                                                 float rho2, float h2, float invA, float cc,
                                                 float a3, float da, float inv_da) {
  const float L = r[7];
  const float ir2 = 1.0f / r[3];
  const float hsf = fast_sqrt(fmaxf(h2, 0.0f) * invA);
  const float sa = fmaf(cc - hsf, da, a3), sb = fmaf(cc + hsf, da, a3);
  const float c0 = -a3 * inv_da, c1 = (L - a3) * inv_da;
  const float q0 = fmaf(c0, fmaf(c0, A, 2.0f * B), rho2);
  const float q1 = fmaf(c1, fmaf(c1, A, 2.0f * B), rho2);
  const bool axial = da != 0.0f;
  return capped_margin(par ? -INFINITY : h2 * ir2, !par && h2 >= 0.0f, sa, sb, L,
                       axial ? (r[3] - q0) * ir2 : -INFINITY,
                       axial ? (r[3] - q1) * ir2 : -INFINITY);
}

template <bool GRAD, bool MRG = false>
__device__ __forceinline__ void cylinder_test(const float* r, float dx, float dy, float dz,
                                              float dd, Hit& h) {
  const float ux = r[8], uy = r[9], uz = r[10], L = r[7];
  const float da = fmaf(dx, ux, fmaf(dy, uy, r[16]));   // r[16] = dz uz
  const float px = fmaf(-da, ux, dx), py = fmaf(-da, uy, dy), pz = fmaf(-da, uz, dz);
  const float A = fmaf(px, px, fmaf(py, py, pz * pz));
  const bool par = A < 1.0e-6f * dd;          // ray within ~1e-3 rad of the axis
  const float inv_da = fast_rcp(da);
  const float invA = fast_rcp(A);
  // (p . c = d . q: q, the cap centre's part perpendicular to the axis, is in r[17..19])
  const float t_side = fmaf(dx, r[18], fmaf(dy, r[19], r[17])) * invA;
  {
    // every lane first as if its ray were not near-parallel to the axis: the side-centred
    // reference, and a miss of the side surface (h2 < 0) gives a NaN half-chord, which fails
    // both interval comparisons.  The values equal the general path's for such lanes.
    const float tr = t_side;
    const float vx = fmaf(tr, dx, -r[0]) - r[4];
    const float vy = fmaf(tr, dy, -r[1]) - r[5];
    const float vz = fmaf(tr, dz, -r[2]) - r[6];
    const float a3 = fmaf(vx, ux, fmaf(vy, uy, vz * uz));
    const float wx = fmaf(-a3, ux, vx), wy = fmaf(-a3, uy, vy), wz = fmaf(-a3, uz, vz);
    const float rho2 = fmaf(wx, wx, fmaf(wy, wy, wz * wz));
    const float B = fmaf(wx, px, fmaf(wy, py, wz * pz));
    const float cc = -B * invA;
    const float h2 = fmaf(B, B * invA, r[3] - rho2);
    const float hs = fast_sqrt(h2 * invA);
    const float d0 = -a3 * inv_da, d1 = (L - a3) * inv_da;
    const float din = fminf(d0, d1), dout = fmaxf(d0, d1);
    const float s_in = cc - hs, s_out = cc + hs;
    h.ok = (s_in <= dout) & (din <= s_out);
    const float tin = fmaxf(s_in, din);
    {
      // a plain sum, as on the general path (where t_r is a select): not fused with t_r's
      // product
#pragma clang fp contract(off)
      h.t = tr + tin;
    }
    if (MRG) h.m = cylinder_margin(r, false, A, B, rho2, h2, invA, cc, a3, da, inv_da);
    if (GRAD) {
      const bool cap = din > s_in;
      h.rx = fmaf(tin, dx, vx);
      h.ry = fmaf(tin, dy, vy);
      h.rz = fmaf(tin, dz, vz);
      const float sgn = da > 0.0f ? -1.0f : 1.0f;
      h.nx = cap ? sgn * ux : fmaf(tin, px, wx);
      h.ny = cap ? sgn * uy : fmaf(tin, py, wy);
      h.nz = cap ? sgn * uz : fmaf(tin, pz, wz);
    }
  }
  // a near-parallel ray (its pixel lies within about half a pixel of the image of the axis's
  // vanishing point, so few wavefronts ever have one) sends the wavefront down the general
  // path, which recomputes every lane
  if (__builtin_expect(__ballot(par) == 0ull, 1)) return;
  // general path: near-parallel rays take the reference at the slab's middle
  const float t_mid = fmaf(0.5f, L, r[11]) * inv_da;    // r[11] = c . u
  const float tr = par ? t_mid : t_side;
  const float vx = fmaf(tr, dx, -r[0]) - r[4];
  const float vy = fmaf(tr, dy, -r[1]) - r[5];
  const float vz = fmaf(tr, dz, -r[2]) - r[6];
  const float a3 = fmaf(vx, ux, fmaf(vy, uy, vz * uz));
  const float wx = fmaf(-a3, ux, vx), wy = fmaf(-a3, uy, vy), wz = fmaf(-a3, uz, vz);
  const float rho2 = fmaf(wx, wx, fmaf(wy, wy, wz * wz));
  // t_side carries the rounding of the perpendicular part of d (large when the ray is close
  // to the axis); the linear term B of the side quadratic re-centres the chord exactly
  const float B = fmaf(wx, px, fmaf(wy, py, wz * pz));
  // near-parallel rays drop the linear term: a zero in place of 1/A (selects, no branch;
  // B is finite, so B * 0 = 0 and the values equal the parallel case's exactly)
  const float invA_s = par ? 0.0f : invA;
  const float cc = -B * invA_s;
  const float h2 = fmaf(B, B * invA_s, r[3] - rho2);
  const float hs = par ? INFINITY : fast_sqrt(fmaxf(h2, 0.0f) * invA);
  // slab 0 <= s <= L as offsets from t_r.  A ray perpendicular to the axis (da == 0) needs no
  // case of its own: 1/da is infinite, so the offsets are -inf and +inf inside the slab and
  // both +inf or both -inf outside it (only a ray exactly in a cap plane, a zero-margin
  // pixel, gives 0 * inf; min and max then drop it and the ray misses).
  const float d0 = -a3 * inv_da, d1 = (L - a3) * inv_da;
  const float din = fminf(d0, d1), dout = fmaxf(d0, d1);
  const float tin = fmaxf(cc - hs, din), tout = fminf(cc + hs, dout);
  h.ok = (h2 >= 0.0f) & (tin <= tout);
  h.t = tr + tin;
  if (MRG) h.m = cylinder_margin(r, par, A, B, rho2, h2, invA, cc, a3, da, inv_da);
  if (GRAD) {
    // entry point relative to p0 and the outward normal of the entry surface
    const bool cap = din > cc - hs;
    h.rx = fmaf(tin, dx, vx);
    h.ry = fmaf(tin, dy, vy);
    h.rz = fmaf(tin, dz, vz);
    const float sgn = da > 0.0f ? -1.0f : 1.0f;
    h.nx = cap ? sgn * ux : fmaf(tin, px, wx);
    h.ny = cap ? sgn * uy : fmaf(tin, py, wy);
    h.nz = cap ? sgn * uz : fmaf(tin, pz, wz);
  }
}

// Closed truncated cone: radius R(s) = r0 + k s on 0 <= s <= L.  As for the cylinder, the
// reference parameter t_r is the closest approach to the axis and every quantity is an offset
// from it.  With w, p the perpendicular parts of the offset and of d, a3 the axial coordinate
// at t_r and R0 = r0 + k a3, the side condition |w + tau p|^2 <= (R0 + k d_a tau)^2 is
// alpha tau^2 + 2 beta tau + gamma <= 0 with alpha = A - (k d_a)^2, beta = B - k d_a R0,
// gamma = rho^2 - R0^2.  For alpha >= 0 its solutions are the interval between the roots;
// for alpha < 0 (a ray steeper than the cone's flank) they are the two rays outside the roots,
// of which the slab meets at most one (the solid is convex).  The roots come from
// q = -(beta + sign(beta) sqrt(disc)), tau = q / alpha and gamma / q, finite as alpha -> 0.
template <bool GRAD, bool MRG = false>
__device__ __forceinline__ void cone_test(const float* r, float dx, float dy, float dz,
                                          float dd, Hit& h) {
  const float ux = r[8], uy = r[9], uz = r[10], L = r[7], r0 = r[3], k = r[11];
  const float da = fmaf(dx, ux, fmaf(dy, uy, dz * uz));
  const float px = fmaf(-da, ux, dx), py = fmaf(-da, uy, dy), pz = fmaf(-da, uz, dz);
  const float A = fmaf(px, px, fmaf(py, py, pz * pz));
  const bool par = A < 1.0e-6f * dd;
  const float inv_da = fast_rcp(da);
  const float t_side = fmaf(px, r[0], fmaf(py, r[1], pz * r[2])) * fast_rcp(A);
  const float cu = fmaf(r[0], ux, fmaf(r[1], uy, r[2] * uz));
  const float t_mid = (cu + 0.5f * L) * inv_da;
  const float tr = par ? t_mid : t_side;
  const float vx = fmaf(tr, dx, -r[0]) - r[4];
  const float vy = fmaf(tr, dy, -r[1]) - r[5];
  const float vz = fmaf(tr, dz, -r[2]) - r[6];
  const float a3 = fmaf(vx, ux, fmaf(vy, uy, vz * uz));
  const float wx = fmaf(-a3, ux, vx), wy = fmaf(-a3, uy, vy), wz = fmaf(-a3, uz, vz);
  const float rho2 = fmaf(wx, wx, fmaf(wy, wy, wz * wz));
  const float B = fmaf(wx, px, fmaf(wy, py, wz * pz));
  const float R0 = fmaf(k, a3, r0);
  const float kd = k * da;
  const float alpha = fmaf(-kd, kd, A);
  const float beta = fmaf(-kd, R0, B);
  const float gamma = fmaf(-R0, R0, rho2);
  const float disc = fmaf(beta, beta, -alpha * gamma);
  const float sq = fast_sqrt(fmaxf(disc, 0.0f));
  const float q = -(beta + copysignf(sq, beta));
  const float ra = q / alpha, rb = gamma / q;
  const float lo = fminf(ra, rb), hi = fmaxf(ra, rb);
  // slab 0 <= s <= L as offsets from t_r
  const float d0 = -a3 * inv_da, d1 = (L - a3) * inv_da;   // infinite for da == 0, as above
  const float din = fminf(d0, d1), dout = fmaxf(d0, d1);
  const bool has = disc >= 0.0f;
  float tin;
  bool side;
  if (alpha >= 0.0f) {
    tin = fmaxf(lo, din);
    side = lo >= din;
    h.ok = has & (tin <= fminf(hi, dout));
  } else {
    // outside the roots: the piece below lo, else the piece above hi
    const bool first = !has | (din <= fminf(dout, lo));
    const float t2 = fmaxf(din, hi);
    tin = first ? din : t2;
    side = !first & (hi >= din);
    h.ok = first ? (din <= dout) : (t2 <= dout);
  }
  h.t = tr + tin;
  if (MRG) {
    // the oracle's cone margin: disc / (|alpha| r_max^2) for the side (slack at each root the
    // least of it and the axial slacks), the caps' disc slacks with their own radii
    const float r1 = fmaf(k, L, r0), rmax2 = fmaxf(r0 * r0, r1 * r1);
    const float dsl = alpha != 0.0f ? disc / (fabsf(alpha) * rmax2) : INFINITY;
    const float s_a = fmaf(ra, da, a3), s_b = fmaf(rb, da, a3);
    const float c0 = -a3 * inv_da, c1 = (L - a3) * inv_da;
    const float q0 = fmaf(c0, fmaf(c0, A, 2.0f * B), rho2);
    const float q1 = fmaf(c1, fmaf(c1, A, 2.0f * B), rho2);
    const bool axial = da != 0.0f;
    const float iL = 1.0f / L;
    const bool fa = isfinite(ra), fb = isfinite(rb);
    const float sla = fa ? fminf(dsl, fminf(s_a * iL, (L - s_a) * iL)) : -INFINITY;
    const float slb = fb ? fminf(dsl, fminf(s_b * iL, (L - s_b) * iL)) : -INFINITY;
    const float side = has ? fmaxf(sla, slb) : ((fa || fb) ? dsl : -INFINITY);
    h.m = fmaxf(fmaxf(side, axial ? (r0 * r0 - q0) / (r0 * r0) : -INFINITY),
                axial ? (r1 * r1 - q1) / (r1 * r1) : -INFINITY);
  }
  if (GRAD) {
    h.rx = fmaf(tin, dx, vx);
    h.ry = fmaf(tin, dy, vy);
    h.rz = fmaf(tin, dz, vz);
    // side normal: perpendicular offset minus k R(s) along the axis; caps: -/+ u
    const float Rt = fmaf(kd, tin, R0);
    const float sgn = da > 0.0f ? -1.0f : 1.0f;
    h.nx = side ? fmaf(-k * Rt, ux, fmaf(tin, px, wx)) : sgn * ux;
    h.ny = side ? fmaf(-k * Rt, uy, fmaf(tin, py, wy)) : sgn * uy;
    h.nz = side ? fmaf(-k * Rt, uz, fmaf(tin, pz, wz)) : sgn * uz;
  }
}

// Closed elliptic cylinder: the side is x^T Q x <= 1 for the offset x from the first cap
// centre (Q = ex ex^T / a^2 + ey ey^T / b^2, Q u = 0), intersected with the slab 0 <= s <= L.
// The reference parameter is the closest approach to the axis in the Q metric.
template <bool GRAD, bool MRG = false>
__device__ __forceinline__ void ecylinder_test(const float* r, float dx, float dy, float dz,
                                               float dd, Hit& h) {
  const float q00 = r[3], q01 = r[7], q02 = r[8], q11 = r[9], q12 = r[10], q22 = r[11];
  const float ux = r[16], uy = r[17], uz = r[18], L = r[19];
  const float qdx = fmaf(q00, dx, fmaf(q01, dy, q02 * dz));
  const float qdy = fmaf(q01, dx, fmaf(q11, dy, q12 * dz));
  const float qdz = fmaf(q02, dx, fmaf(q12, dy, q22 * dz));
  const float dqd = fmaf(dx, qdx, fmaf(dy, qdy, dz * qdz));
  const float da = fmaf(dx, ux, fmaf(dy, uy, dz * uz));
  const bool par = dqd < 1.0e-6f * dd * (q00 + q11 + q22);
  const float inv = fast_rcp(dqd);
  const float inv_da = fast_rcp(da);
  const float cqd = fmaf(r[0], qdx, fmaf(r[1], qdy, r[2] * qdz));
  const float cu = fmaf(r[0], ux, fmaf(r[1], uy, r[2] * uz));
  const float tr = par ? (cu + 0.5f * L) * inv_da : cqd * inv;
  const float vx = fmaf(tr, dx, -r[0]) - r[4];
  const float vy = fmaf(tr, dy, -r[1]) - r[5];
  const float vz = fmaf(tr, dz, -r[2]) - r[6];
  const float qvx = fmaf(q00, vx, fmaf(q01, vy, q02 * vz));
  const float qvy = fmaf(q01, vx, fmaf(q11, vy, q12 * vz));
  const float qvz = fmaf(q02, vx, fmaf(q12, vy, q22 * vz));
  const float vqv = fmaf(vx, qvx, fmaf(vy, qvy, vz * qvz));
  const float B = fmaf(vx, qdx, fmaf(vy, qdy, vz * qdz));
  const float inv_s = par ? 0.0f : inv;     // as for the cylinder: selects, no branch
  const float cc = -B * inv_s;
  const float m = fmaf(B, B * inv_s, 1.0f - vqv);
  const float hs = par ? INFINITY : fast_sqrt(fmaxf(m, 0.0f) * inv);
  const float a3 = fmaf(vx, ux, fmaf(vy, uy, vz * uz));
  const float d0 = -a3 * inv_da, d1 = (L - a3) * inv_da;   // infinite for da == 0, as above
  const float din = fminf(d0, d1), dout = fmaxf(d0, d1);
  const float tin = fmaxf(cc - hs, din), tout = fminf(cc + hs, dout);
  h.ok = (m >= 0.0f) & (tin <= tout);
  h.t = tr + tin;
  if (MRG) {
    // in the unit-radius frame of the Q metric: radius^2 at offset tau is
    // vQv + 2 tau B + tau^2 dQd
    const float hsf = fast_sqrt(fmaxf(m, 0.0f) * inv);
    const float sa = fmaf(cc - hsf, da, a3), sb = fmaf(cc + hsf, da, a3);
    const float c0 = -a3 * inv_da, c1 = (L - a3) * inv_da;
    const float q0 = fmaf(c0, fmaf(c0, dqd, 2.0f * B), vqv);
    const float q1 = fmaf(c1, fmaf(c1, dqd, 2.0f * B), vqv);
    const bool axial = da != 0.0f;
    h.m = capped_margin(par ? -INFINITY : m, !par && m >= 0.0f, sa, sb, L,
                        axial ? 1.0f - q0 : -INFINITY, axial ? 1.0f - q1 : -INFINITY);
  }
  if (GRAD) {
    const bool cap = din > cc - hs;
    h.rx = fmaf(tin, dx, vx);
    h.ry = fmaf(tin, dy, vy);
    h.rz = fmaf(tin, dz, vz);
    const float sgn = da > 0.0f ? -1.0f : 1.0f;
    h.nx = cap ? sgn * ux : fmaf(tin, qdx, qvx);
    h.ny = cap ? sgn * uy : fmaf(tin, qdy, qvy);
    h.nz = cap ? sgn * uz : fmaf(tin, qdz, qvz);
  }
}

// ------------------------------------------------------------------------------------
// wave-uniform values: read once from lane 0 into scalar registers, so that the per-tile
// bookkeeping runs on the scalar unit and holds no vector registers

__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ float uni(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
template <class T>
__device__ __forceinline__ T* uni(T* x) {
  const uint64_t v = reinterpret_cast<uint64_t>(x);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ FrameSlot uni(const FrameSlot& f) {
  FrameSlot u;
  u.W = uni(f.W);
  u.H = uni(f.H);
  u.TW = uni(f.TW);
  u.TH = uni(f.TH);
  u.sx = uni(f.sx);
  u.sy = uni(f.sy);
  u.sz = uni(f.sz);
  u.cx = uni(f.cx);
  u.cy = uni(f.cy);
  u.fx = uni(f.fx);
  u.fy = uni(f.fy);
  u.bg = uni(f.bg);
  u.set = uni(f.set);
  u.words = uni(f.words);
  u.tile_td = uni(f.tile_td);
  u.tile_skin = uni(f.tile_skin);
  u.totals = uni(f.totals);
  u.grad_mask = uni(f.grad_mask);
  return u;
}

// Walks a particle's tiles (the union of its rectangles, each row-major) in steps of the
// number of wavefronts per workgroup, without a division per tile.
struct TileWalk {
  const PInfo* pi;
  int n, ri, rx, ry, rw, rh, ox, oy;

  __device__ void load(int r) {
    const int4 rc = pi->rect[r];
    rx = uni(rc.x);
    ry = uni(rc.y);
    rw = uni(rc.z);
    rh = uni(rc.w);
  }
  // position at tile t of the union
  __device__ void seek(int t) {
    while (t >= rw * rh && ri + 1 < n) {
      t -= rw * rh;
      load(++ri);
    }
    oy = t / rw;
    ox = t - oy * rw;
  }
  __device__ void start(const PInfo* p, int t) {
    pi = p;
    n = uni(p->n_rects);
    ri = 0;
    load(0);
    seek(t);
  }
  __device__ void step(int s) {
    ox += s;
    while (ox >= rw) {
      ox -= rw;
      ++oy;
    }
    if (oy >= rh && ri + 1 < n) {
      const int t = (oy - rh) * rw + ox;
      load(++ri);
      seek(t);
    }
  }
  __device__ int tx() const { return rx + ox; }
  __device__ int ty() const { return ry + oy; }
};

// ------------------------------------------------------------------------------------
// persistent ray cast + cost terms + reduction

// Workgroups are dispatched to the chip's 8 XCDs round-robin (workgroup b on XCD b mod 8), each
// XCD with its own L2.  The first item of workgroup b is taken XCD-major: XCD x's workgroups
// take the x-th eighth of the items in order, so the consecutive items of one particle (and
// its staged tables) stay on one XCD instead of spreading over all eight.  A bijection of
// 0 .. G-1 for any grid size G.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_major_item(int b, int G) {
  const int q = G / kXcds, rem = G % kXcds;
  const int x = b % kXcds, j = b / kXcds;
  return x * q + min(x, rem) + j;
}

// Launches of at most kSelfSched particles build their work list in every ray-cast workgroup
// (no work-list launch before them): one thread per particle reads its tile count, two block
// scans give the item size (the work-list kernel's rule) and the item offsets in LDS, and the
// workgroups take items in a static stride of the grid size (the items are sized to about
// one per workgroup, so there is nothing to balance dynamically).  Workgroup 0 stores the
// offsets for the finalize and refinement kernels and adds the launch's evaluations to the
// counts.
constexpr int kSelfSched = kBlock;
static_assert(kSelfSched == kSelfSchedMax, "one thread per particle of a self-scheduled launch");

__device__ void self_schedule(const EvalArgs& a, const Workspace& ws, int* s_off, int& total,
                              int& tpi, bool& interleave) {
  __shared__ int2 s_sum2[kWavesPerBlock];
  __shared__ int s_sum[kWavesPerBlock];
  const int n_total = a.n_frames * a.n_particles;
  const int t = threadIdx.x;
  const int v = t < n_total ? ws.tiles[src_of(a, min(t, n_total - 1))] : -1;
  int total_tiles, total_evaluated;
  block_scan2<kWavesPerBlock>(s_sum2, max(v, 0), v >= 0 ? 1 : 0, &total_tiles,
                              &total_evaluated);
  const long long target = (long long)a.grid * kItemsPerGroup;
  long long tq = ((long long)total_tiles + target - 1) / target;
  tq = (tq + kWavesPerBlock - 1) / kWavesPerBlock * kWavesPerBlock;
  const long long lo = a.grad ? (long long)kFloorTilesGrad : (long long)kFloorTilesFwd;
  tpi = (int)max(min(lo, (long long)a.tiles_per_item), min(tq, (long long)a.tiles_per_item));
  const int items = (max(v, 0) + tpi - 1) / tpi;
  int total_items;
  const int incl = block_scan<kWavesPerBlock>(s_sum, items, &total_items);
  if (t < n_total) s_off[t + 1] = incl;
  if (t == 0) s_off[0] = 0;
  __syncthreads();
  total = total_items;
  // items in a static stride, about one per workgroup: interleaved tiles, so that every item
  // samples the whole hand (runs of consecutive tiles left the launch waiting on the items
  // from the hand's middle: 128 forward candidates 26.7 -> 24.1 us)
  interleave = total_items <= 2 * a.grid;
  if (blockIdx.x == 0) {
    // n_total + 1 offsets: one per thread, the end offset by thread 0
    if (t < n_total) ws.item_off[t] = s_off[t];
    if (t == 0) {
      ws.item_off[n_total] = total_items;
      if (a.eval_count)
        atomicAdd(&a.eval_count[a.grad ? 1 : 0], (unsigned long long)total_evaluated);
      ws.counters[1] = total_items;
      ws.counters[2] = tpi;
      ws.counters[3] = interleave ? 1 : 0;
    }
  }
}

// The evaluated particle r of item i in a self-scheduled launch: s_off[r] <= i < s_off[r + 1]
// (a binary search over the LDS offsets; wave-uniform).
__device__ __forceinline__ int self_item_particle(const int* s_off, int n_total, int i) {
  int lo = 0, hi = n_total;   // s_off[lo] <= i < s_off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (uni(s_off[mid]) <= i) lo = mid;
    else hi = mid;
  }
  return lo;
}

// NT: primitive types the model uses (3: spheres, cylinders, ellipsoids; kNumTypes: also
// cones and elliptic cylinders), so a model without the latter keeps the smaller register
// footprint.  (Forcing more wavefronts per SIMD than the vector register count allows
// spills vector registers and measured slower.)  SELF: the launch builds its own work list (at most
// kSelfSched particles, no debug images); a variant of its own, so the larger launches keep
// the dequeue loop without the self-scheduling code (which cost them about 5%).
//
// The work-list launches of the plain forward cast ask for eight wavefronts per SIMD: left to
// itself the compiler needs more scalar registers than eight allow (seven fit), and the few
// it then keeps in vector-register lanes are reloaded per item, outside the tile loop
// (1.2 % off the two-hand frame; the self-scheduled launches, at most six workgroups per
// CU, measured slower with the same request).
template <bool GRAD, bool DEBUG, int NT, bool SELF>
__global__ __attribute__((amdgpu_flat_work_group_size(1, kBlock),
                          amdgpu_waves_per_eu((GRAD || DEBUG || SELF) ? 1 : 8)))
void raycast_kernel(EvalArgs a, Workspace ws, TypeMasks tm) {
  __shared__ float4 s_rec[HT_MAX_PRIM * (kRec / 4)];
  __shared__ int4 s_box[HT_MAX_PRIM];
  __shared__ float4 s_cap[HT_MAX_PRIM];
  __shared__ float2 s_capr[HT_MAX_PRIM];
  __shared__ int s_item;
  __shared__ PInfo s_pi;
  __shared__ double s_td[kWavesPerBlock];
  __shared__ int s_a[kWavesPerBlock], s_o[kWavesPerBlock];
  // gradient: per wavefront, segment and 16-lane row, the six wrench components of the item
  __shared__ float s_wr[GRAD ? kWavesPerBlock : 1][GRAD ? HT_MAX_SEG : 1][GRAD ? 4 : 1][6];

  // the wavefront index as a scalar, so that the tile walk, the tile's coordinates and the
  // observation addresses are wave-uniform (scalar instructions)
  const int tid = threadIdx.x, lane = tid & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int n_prim = a.n_prim, n_seg = a.n_seg;
  static_assert(!(SELF && DEBUG), "debug launches take the work-list kernel");
  constexpr bool self = SELF;
  __shared__ int s_off[SELF ? kSelfSched + 1 : 1];
  int total, tpi;
  bool interleave;
  if constexpr (SELF) {
    self_schedule(a, ws, s_off, total, tpi, interleave);
  } else {
    total = uni(ws.counters[1]);
    tpi = uni(ws.counters[2]);
    interleave = uni(ws.counters[3]) != 0;
  }
  const int n_eval = a.n_frames * a.n_particles;
  int cur_p = -1;
  FrameSlot fs{};
  // the lane's pixel offset within a tile as a ray component: ((lane & 7) - cx) sx and
  // ((lane >> 3) - cy) sy, so that a tile's rays cost one multiply-add per component
  float lane_dx = 0.0f, lane_dy = 0.0f;
  const PInfo& pi = s_pi;

  // the first item of every workgroup is its own index; later ones come from the dequeue
  // counter (offset by the grid size), so the launch does not start with one atomic per
  // workgroup on a single address (which stalls the memory channel that holds it)
  bool first = true;
  int item = 0;
  for (;;) {
    if (first) {
      item = xcd_major_item(blockIdx.x, gridDim.x);
      first = false;
    } else if constexpr (SELF) {
      // the next item in the static stride; the barrier keeps its per-wavefront LDS sums
      // clear of the previous item's (whose readers may still be at work when both items
      // belong to one particle and so no staging barrier follows)
      item += gridDim.x;
      __syncthreads();
    } else {
      if (tid == 0) s_item = (int)gridDim.x + atomicAdd(&ws.counters[0], 1);
      __syncthreads();
      item = uni(s_item);
      __syncthreads();
    }
    if (item >= total) break;
    // evaluated particle
    const int r = self ? self_item_particle(s_off, n_eval, item) : uni(ws.item_map[item]);
    const int p = a.src ? uni(src_of(a, r)) : r;   // the workspace particle of its kinematics
    if (p != cur_p) {
      const float4* src = reinterpret_cast<const float4*>(ws.recs + (size_t)p * n_prim * kRec);
      for (int i = tid; i < n_prim * (kRec / 4); i += kBlock) s_rec[i] = src[i];
      for (int i = tid; i < n_prim; i += kBlock) {
        s_box[i] = ws.boxes[(size_t)p * n_prim + i];
        s_cap[i] = ws.caps[(size_t)p * n_prim + i];
        s_capr[i] = ws.capr[(size_t)p * n_prim + i];
      }
      if (tid == 0) s_pi = ws.pinfo[p];
      cur_p = p;
      __syncthreads();
      fs = uni(a.slots[uni(s_pi.slot)]);
      lane_dx = ((float)(lane & 7) - fs.cx) * fs.sx;
      lane_dy = ((float)(lane >> 3) - fs.cy) * fs.sy;
    }
    if (GRAD) {
      float* wr = &s_wr[wave][0][0][0];
      for (int i = lane; i < n_seg * 24; i += kWave) wr[i] = 0.0f;
    }
    // item c of a particle with n_it items takes tiles c tpi .. (c + 1) tpi - 1, or, when
    // interleaved, tiles c, c + n_it, c + 2 n_it, ...: then every item samples the whole hand
    // and carries about equal work (runs of consecutive tiles differed threefold, and a launch
    // with about one item per workgroup lasts as long as its longest item); wavefront w takes
    // every fourth of an item's tiles
    const int off = self ? uni(s_off[r]) : uni(ws.item_off[r]);
    const int c = item - off;
    const int n_it = (self ? uni(s_off[r + 1]) : uni(ws.item_off[r + 1])) - off;
    const int n_tiles = uni(pi.n_tiles);
    const int first = interleave ? c : c * tpi;
    const int gap = interleave ? n_it : 1;
    const int t_end = interleave ? n_tiles : min((c + 1) * tpi, n_tiles);
    const int stride = gap * kWavesPerBlock;
    double acc_td = 0.0;   // exact: the FP32 terms are multiples of 2^-15 mm
    double acc_bg = 0.0;   // the tiles' background depth sums (the same on every lane)
    int acc_a = 0, acc_o = 0;   // wavefront totals: popcounts of lane masks (scalar unit)
    const float* recs = reinterpret_cast<const float*>(s_rec);

    TileWalk walk;
    walk.start(&pi, first + wave * gap);
    for (int t = first + wave * gap; t < t_end; t += stride, walk.step(stride)) {
      const int tx = walk.tx(), ty = walk.ty();
      const int x0 = tx * kTile, y0 = ty * kTile;
      const float x0f = (float)x0, y0f = (float)y0;
      // culling, one lane per primitive: screen box overlap, then the distance of the tile's
      // centre from the primitive's image segment
      // (the three loads are issued together, the index clamped, so no branch waits on LDS;
      // the segment test runs only where some lane's box overlaps; the second half is skipped
      // outright for models of at most 64 primitives)
      uint64_t mk[2] = {0ull, 0ull};
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        if (half * kWave >= n_prim) break;
        const int k = lane + half * kWave;
        const int kk = min(k, n_prim - 1);
        const int4 b = s_box[kk];
        const float4 cp = s_cap[kk];
        const float2 cq = s_capr[kk];
        // one ballot per comparison, combined on the scalar unit with the half's primitive
        // lanes (a ballot of the combined condition routes its lane mask through a vector
        // register and back)
        const int left = n_prim - half * kWave;
        uint64_t m = (left >= kWave ? ~0ull : (1ull << left) - 1ull) &
                     __builtin_amdgcn_ballot_w64(b.x <= x0 + kTile - 1) &
                     __builtin_amdgcn_ballot_w64(b.y >= x0) &
                     __builtin_amdgcn_ballot_w64(b.z <= y0 + kTile - 1) &
                     __builtin_amdgcn_ballot_w64(b.w >= y0);
        if (m) {
          // on every lane (a uniform branch), the result a lane mask combined on the scalar
          // unit: no per-lane branch whose outcome would go through a vector register
          // tile centre (x0 + 3.5, y0 + 3.5) minus the first disc's centre (cp: less 3.5)
          const float wx = x0f - cp.x, wy = y0f - cp.y;
          const float sp = fminf(fmaxf(fmaf(wx, cp.z, wy * cp.w) * cq.x, 0.0f), 1.0f);
          const float ex = fmaf(-sp, cp.z, wx), ey = fmaf(-sp, cp.w, wy);
          m &= __builtin_amdgcn_ballot_w64(fmaf(ex, ex, ey * ey) <= cq.y);
        }
        mk[half] = m;
      }
      if ((mk[0] | mk[1]) == 0ull) continue;

      const int tile_idx = ty * fs.TW + tx;
      const int u = x0 + (lane & 7), v = y0 + (lane >> 3);
      const uint32_t word = global_ptr(fs.words)[(size_t)tile_idx * kTilePx + lane];
      // the tile's background sums, loaded with the words (one address for every lane) so
      // that their latency overlaps the tests; lane 0 subtracts them after the tests
      const float bg_td = global_ptr(fs.tile_td)[tile_idx];
      const int bg_sk = global_ptr(fs.tile_skin)[tile_idx];
      const bool valid = (word & kValidBit) != 0;
      const float od = (float)(word & 0xFFFFu);
      const bool os = (word & kSkinBit) != 0;
      const float dx = fmaf(x0f, fs.sx, lane_dx);
      const float dy = fmaf(y0f, fs.sy, lane_dy);
      const float dz = fs.sz;
      const float dd = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
      const float inv_dd = fast_rcp(dd);
      float tmin = INFINITY;
      int win = -1;   // tracked for the gradient and the debug images only
      float wnx = 0, wny = 0, wnz = 0, wrx = 0, wry = 0, wrz = 0;
      float wm = -INFINITY, mmax = -INFINITY;   // margins (debug images only)

#pragma unroll
      for (int half = 0; half < 2; ++half) {
#pragma unroll
        for (int typ = 0; typ < NT; ++typ) {
          uint64_t m = mk[half] & tm.m[typ][half];
          while (m) {
            const int k = __builtin_ctzll(m) + half * kWave;
            m &= m - 1;
            const float* r = recs + k * kRec;
            Hit h;
            if (typ == HT_SPHERE) sphere_test<GRAD, DEBUG>(r, dx, dy, dz, inv_dd, h);
            else if (typ == HT_CYLINDER) cylinder_test<GRAD, DEBUG>(r, dx, dy, dz, dd, h);
            else if (typ == HT_ELLIPSOID) ellipsoid_test<GRAD, DEBUG>(r, dx, dy, dz, h);
            else if (typ == HT_CONE) cone_test<GRAD, DEBUG>(r, dx, dy, dz, dd, h);
            else ecylinder_test<GRAD, DEBUG>(r, dx, dy, dz, dd, h);
            // nearest entry in front of the camera: as unsigned integers the bit patterns of
            // non-negative floats keep their order and negative ones (entries behind the
            // camera) exceed +inf; exact ties keep the first tested (branch-free selects)
            const bool take = h.ok & (__float_as_uint(h.t) < __float_as_uint(tmin));
            tmin = take ? h.t : tmin;
            if (GRAD || DEBUG) win = take ? k : win;
            if (DEBUG) {
              // the nearest primitive's margin, and the largest of the tested ones (misses)
              wm = take ? h.m : wm;
              mmax = fmaxf(mmax, h.m);
            }
            if (GRAD) {
              wnx = take ? h.nx : wnx;
              wny = take ? h.ny : wny;
              wnz = take ? h.nz : wnz;
              wrx = take ? h.rx : wrx;
              wry = take ? h.ry : wry;
              wrz = take ? h.rz : wrz;
            }
          }
        }
      }
      // depth of the nearest entry; behind the background plane it is hidden
      const float zmin = tmin * dz;
      const bool any = (GRAD || DEBUG) ? win >= 0 : __float_as_uint(tmin) < 0x7F800000u;
      const bool hit = any & !(fs.bg > 0.0f && zmin >= fs.bg);
      win = hit ? win : -1;
      const float rd = hit ? zmin : (fs.bg > 0.0f ? fs.bg : 0.0f);
      const float diff = fabsf(od - rd);
      const float td = fminf(diff, kDClamp);
      const bool rm = hit && (diff < kDMatch || od == 0.0f);
      acc_td += (double)(valid ? td : 0.0f);
      {
        // one ballot per condition, combined on the scalar unit
        const uint64_t m_valid = __builtin_amdgcn_ballot_w64(valid);
        const uint64_t m_os = __builtin_amdgcn_ballot_w64(os);
        const uint64_t m_rm = __builtin_amdgcn_ballot_w64(rm);
        acc_a += __builtin_popcountll(m_valid & m_os & m_rm);
        acc_o += __builtin_popcountll(m_valid & (m_os | m_rm));
      }
      {
        // read back here (a convergent read, so the wait for the loads stays after the tests)
        const float bgt = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(bg_td)));
        const int bgs = __builtin_amdgcn_readfirstlane(bg_sk);
        acc_bg += (double)bgt;
        acc_o -= bgs;
      }
      // the debug images have the host's W x H of the debug slot; a frame slot of another
      // size would write past them, so stores outside that extent are dropped
      if (DEBUG && valid && u < a.dbg_W && v < a.dbg_H) {
        const size_t pix = ((size_t)r * a.dbg_H + v) * a.dbg_W + u;
        if (a.dbg.depth) a.dbg.depth[pix] = rd;
        if (a.dbg.hit) a.dbg.hit[pix] = hit ? 1 : 0;
        if (a.dbg.rm) a.dbg.rm[pix] = rm ? 1 : 0;
        if (a.dbg.winner) a.dbg.winner[pix] = win;
        if (a.dbg.margin) a.dbg.margin[pix] = any ? wm : mmax;
      }
      if (GRAD) {
        // adjoint: coefficient of the depth term, then the per-segment wrench
        bool act = valid && hit && diff < kDClamp && od != rd;
        // the call's mask (one frame), else the frame's slot mask
        const uint8_t* gmask = a.pixel_mask ? a.pixel_mask : fs.grad_mask;
        if (act && gmask) act = global_ptr(gmask)[(size_t)v * fs.W + u] != 0;
        int seg = -1;
        float kap = 0.0f;
        float mx = 0, my = 0, mz = 0;
        if (act) {
          const float* r = recs + win * kRec;
          seg = __float_as_int(r[15]);
          const float nd = fmaf(wnx, dx, fmaf(wny, dy, wnz * dz));
          // (the hardware reciprocal: a quotient would expand into a range-safe sequence of
          // ten instructions; nd is a dot product of normal and ray, far from the range ends)
          kap = ((rd > od ? dz : -dz)) * fast_rcp(nd);
          // lever arm from the segment origin: (entry - ref) + (ref - origin)
          const float lx = wrx + r[12], ly = wry + r[13], lz = wrz + r[14];
          mx = kap * (ly * wnz - lz * wny);
          my = kap * (lz * wnx - lx * wnz);
          mz = kap * (lx * wny - ly * wnx);
        }
        const float fx = kap * wnx, fy = kap * wny, fz = kap * wnz;
        // segments present in this tile, one at a time (uniform loop): row sums on the
        // vector unit, added by the first lane of each row into that row's accumulators (an
        // LDS atomic add without return; the four lanes hit distinct addresses and the adds of
        // a wavefront are applied in program order, so the result is deterministic)
        uint32_t segmask = wave_or(act ? (1u << seg) : 0u);
        while (segmask) {
          const int s = __builtin_ctz(segmask);
          segmask &= segmask - 1;
          const bool mine = seg == s;
          const float vals[6] = {mine ? mx : 0.f, mine ? my : 0.f, mine ? mz : 0.f,
                                 mine ? fx : 0.f, mine ? fy : 0.f, mine ? fz : 0.f};
          float sum[6];
#pragma unroll
          for (int q = 0; q < 6; ++q) sum[q] = row_total(vals[q]);
          if ((lane & 15) == 0) {
            float* dst = &s_wr[wave][s][lane >> 4][0];
#pragma unroll
            for (int q = 0; q < 6; ++q) atomicAdd(dst + q, sum[q]);
          }
        }
      }
    }

    acc_td = wave_sum(acc_td) - acc_bg;
    if (lane == 0) {
      s_td[wave] = acc_td;
      s_a[wave] = acc_a;
      s_o[wave] = acc_o;
    }
    __syncthreads();
    if (tid == 0) {
      Partial pr;
      pr.td = ((s_td[0] + s_td[1]) + s_td[2]) + s_td[3];
      pr.a = s_a[0] + s_a[1] + s_a[2] + s_a[3];
      pr.o = s_o[0] + s_o[1] + s_o[2] + s_o[3];
      pr.pad = 0;
      ws.partial[item] = pr;
    }
    if (GRAD) {
      for (int i = tid; i < n_seg * 6; i += kBlock) {
        const int s = i / 6, q = i % 6;
        float v = 0.0f;
#pragma unroll
        for (int w = 0; w < kWavesPerBlock; ++w)
          v += (s_wr[w][s][0][q] + s_wr[w][s][1][q]) + (s_wr[w][s][2][q] + s_wr[w][s][3][q]);
        ws.wrench[(size_t)item * n_seg * 6 + i] = v;
      }
    }
  }
}

// ------------------------------------------------------------------------------------
// finalize: combine partials in item order, Eq. 4-5, and the kinematic adjoint

// This lane's partial among a particle's first 64 items (items b .. e-1), loaded without a
// branch: the index is clamped into the buffer and the value is used only when in range.
__device__ __forceinline__ Partial first_partial(const Workspace& ws, int b, int e, int lane) {
  return ws.partial[max(min(b + lane, e - 1), 0)];
}

// S_d, S_and, S_or of a particle: the ROI's background totals plus its items' partials,
// summed by the lanes of one wavefront (pr0: this lane's first_partial, loaded early by the
// caller).  Every depth term is a multiple of 2^-15 mm, so the FP64 sums are exact and equal
// to any other summation order.
__device__ inline void wave_partial_sums(const PInfo& pi, const Workspace& ws, int b, int e,
                                         int lane, const Partial& pr0, double& S_d,
                                         long long& S_and, long long& S_or) {
  const bool in0 = b + lane < e;
  double d = in0 ? pr0.td : 0.0;
  int sa = in0 ? pr0.a : 0, so = in0 ? pr0.o : 0;
  for (int i = b + kWave + lane; i < e; i += kWave) {
    const Partial pr = ws.partial[i];
    d += pr.td;
    sa += pr.a;
    so += pr.o;
  }
  d = wave_sum(d);
  sa = wave_sum(sa);
  so = wave_sum(so);
  S_d = pi.bg_td + d;
  S_and = sa;
  S_or = (long long)pi.bg_or + so;
}

// Eq. 4-5 from the sums (FP64).
__device__ inline float cost_from_sums(double S_d, long long S_and, long long S_or, float kc) {
  double D;
  if (S_or == 0) {
    D = kLambda;
  } else {
    D = S_d / (double)S_or + kLambda * (1.0 - 2.0 * (double)S_and / (double)(S_and + S_or));
  }
  return (float)(D + kLambdaK * (double)kc);
}

// Forward: one wavefront per particle.
__global__ __launch_bounds__(kBlock) void finalize_kernel(EvalArgs a, Workspace ws) {
  const int lane = threadIdx.x & (kWave - 1);
  // evaluated particle, wave-uniform (its record and item range are scalar loads)
  const int p = blockIdx.x * kWavesPerBlock + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n_total = a.n_frames * a.n_particles;
  if (p >= n_total) return;
  // the item range and the record are independent loads; the partials are summed before the
  // record is tested (a skipped or invalid particle has no items), so no branch waits on it
  const int b = ws.item_off[p], e = ws.item_off[p + 1];
  const PInfo pi = ws.pinfo[src_of(a, p)];
  const Partial pr0 = first_partial(ws, b, e, lane);
  double S_d;
  long long S_and, S_or;
  wave_partial_sums(pi, ws, b, e, lane, pr0, S_d, S_and, S_or);
  if (pi.skip) return;
  if (!pi.valid) {
    if (lane == 0) a.cost[p] = pi.slot < 0 ? NAN : INFINITY;
    return;
  }
  if (lane == 0) a.cost[p] = cost_from_sums(S_d, S_and, S_or, pi.kc);
}

// Gradient: one workgroup per particle.  Threads (segment, component) sum the per-item
// wrenches in item order; then one thread per pose parameter applies the kinematic adjoint
//   dE/dh_j = (1/S_or) sum_{s moved by j} a_j . (M_s + (q_s - q_j) x F_s)   (rotation)
//   dE/dh_j = (1/S_or) sum_{s moved by j} e_j . F_s                       (translation)
// with M_s, F_s the moment about the segment origin q_s and the force of segment s.
__global__ __launch_bounds__(kBlock) void finalize_grad_kernel(EvalArgs a, Workspace ws) {
  __shared__ double s_W[HT_MAX_SEG * 6];
  __shared__ double s_part[kWavesPerBlock][HT_MAX_SEG * 6];
  __shared__ double s_inv_or;
  __shared__ float s_org[HT_MAX_SEG * 4];
  __shared__ int s_kca[HT_MAX_KC], s_kcb[HT_MAX_KC];
  const int p = blockIdx.x, t = threadIdx.x;   // evaluated particle
  const int ps = src_of(a, p);                  // the workspace particle of its kinematics
  const int n_dof = a.n_dof, n_seg = a.n_seg;
  // every load that depends on the particle index alone is issued here: the item range, the
  // record, and this thread's pose parameter (descendant mask, camera-frame axis and point;
  // threads past n_dof have none).  The record is tested only after the sums below (a skipped
  // or invalid particle has no items), so no branch holds these loads back.
  const int b = ws.item_off[p], e = ws.item_off[p + 1];
  const PInfo pi = ws.pinfo[ps];
  const int j = t, jc = min(t, n_dof - 1);   // loads clamped in bounds, unconditional
  const uint32_t desc = j < n_dof ? a.model->dof_desc[jc] : 0u;
  const float4* f4 = reinterpret_cast<const float4*>(ws.dof_frame + ((size_t)ps * n_dof + jc) * 8);
  const float4 f0 = f4[0], f1 = f4[1];
  const float fr[8] = {f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w};
  // segment origins and collision pairs for the adjoint below, loaded into registers now and
  // staged in LDS after the wrench loads have been issued (one value per thread)
  static_assert(HT_MAX_SEG * 4 <= kBlock, "one segment-origin value per thread");
  const float org_v = t < n_seg * 4 ? ws.seg_org[(size_t)ps * n_seg * 4 + t] : 0.0f;
  const int kc_i = t < HT_MAX_KC ? t : 0;
  const int kca_v = a.model->kc_a[kc_i], kcb_v = a.model->kc_b[kc_i];
  // wave q sums items b+q, b+q+4, ... (kFinItems at a time, loads first); lane l sums values
  // l, l+64, l+128; then the four partial sums are added in a fixed order
  const int nv = n_seg * 6, lane = t & (kWave - 1);
  const int q = __builtin_amdgcn_readfirstlane(t >> 6);   // wave-uniform
  // the first partials, for the second wavefront's cost sums below; loaded by every wavefront
  // (unconditionally, so that no branch waits on them), issued with the wrench loads
  const Partial pr0 = first_partial(ws, b, e, lane);
  constexpr int kFinItems = 4;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int i = b + q; i < e; i += kFinItems * kWavesPerBlock) {
    // the loads are unconditional (items and offsets clamped into the particle's), so they are
    // in flight together; items past the end and lanes past nv add zero
    float v[kFinItems][3];
#pragma unroll
    for (int u = 0; u < kFinItems; ++u) {
      const float* src = ws.wrench + (size_t)min(i + u * kWavesPerBlock, e - 1) * nv;
#pragma unroll
      for (int k = 0; k < 3; ++k) v[u][k] = src[min(lane + k * kWave, nv - 1)];
    }
#pragma unroll
    for (int u = 0; u < kFinItems; ++u)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if (i + u * kWavesPerBlock < e)
          acc[k] += lane + k * kWave < nv ? (double)v[u][k] : 0.0;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if (lane + k * kWave < nv) s_part[q][lane + k * kWave] = acc[k];
  if (t < n_seg * 4) s_org[t] = org_v;
  if (t < HT_MAX_KC) {
    const bool on = t < a.model->n_kc;
    s_kca[t] = on ? kca_v : -1;
    s_kcb[t] = on ? kcb_v : -1;
  }
  // the cost sums go to the second wavefront, which has no pose parameter (at most 64 of them,
  // all in the first), so they overlap the first one's wrench sums
  static_assert(HT_MAX_DOF <= kWave, "pose parameters fit the first wavefront");
  double S_d = 0.0;
  long long S_and = 0, S_or = 0;
  if (q == 1) wave_partial_sums(pi, ws, b, e, lane, pr0, S_d, S_and, S_or);
  if (pi.skip) return;
  if (!pi.valid) {
    if (t == 0) a.cost[p] = pi.slot < 0 ? NAN : INFINITY;
    for (int i = t; i < n_dof; i += kBlock) a.grad[(size_t)p * n_dof + i] = 0.0f;
    return;
  }
  if (q == 1 && lane == 0) {
    a.cost[p] = cost_from_sums(S_d, S_and, S_or, pi.kc);
    s_inv_or = S_or > 0 ? 1.0 / (double)S_or : 0.0;
  }
  __syncthreads();
  if (t < nv) s_W[t] = ((s_part[0][t] + s_part[1][t]) + s_part[2][t]) + s_part[3][t];
  __syncthreads();
  if (j < n_dof) {
    const float* f = fr;
    const float* org = s_org;
    const bool trans = f[0] != 0.0f;
    const double ax = f[1], ay = f[2], az = f[3];
    double g = 0.0;
    // the segments this parameter moves, in increasing order, four per round (their LDS reads
    // issued together)
    for (uint32_t m = desc; m;) {
      int sg[4];
      bool has[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        has[q] = m != 0u;
        sg[q] = has[q] ? __builtin_ctz(m) : 0;
        m &= m - 1u;
      }
      double t[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double* W = s_W + sg[q] * 6;
        const double lx = (double)org[sg[q] * 4 + 0] - f[4];
        const double ly = (double)org[sg[q] * 4 + 1] - f[5];
        const double lz = (double)org[sg[q] * 4 + 2] - f[6];
        const double mx = W[0] + (ly * W[5] - lz * W[4]);
        const double my = W[1] + (lz * W[3] - lx * W[5]);
        const double mz = W[2] + (lx * W[4] - ly * W[3]);
        t[q] = trans ? ax * W[3] + ay * W[4] + az * W[5] : ax * mx + ay * my + az * mz;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (has[q]) g += t[q];
    }
    g *= s_inv_or;
    // collision term of Eq. 5: the pairs whose term is positive (recorded by the kinematics)
    for (int m = pi.kc_mask; m; m &= m - 1) {
      const int i = __builtin_ctz(m);
      if (s_kca[i] == j) g -= kLambdaK;
      if (s_kcb[i] == j) g += kLambdaK;
    }
    a.grad[(size_t)p * n_dof + j] = (float)g;
  }
}

// ------------------------------------------------------------------------------------
// gradient refinement update, fused with the assembly of the preceding evaluation
//
// One workgroup per refined particle r.  First the evaluation that precedes this update is
// assembled, one wavefront per evaluated particle, as the finalize kernels would (the cost of
// Eq. 4-5 from the item partials; with gradients the per-segment wrench sums in item order
// and the kinematic adjoint, one lane per pose parameter): the particle itself after the
// gradient evaluation of the selected particles (wavefront 0), or its four candidates after a
// candidate evaluation (wavefront j: candidate j).  Then wavefront 0, one lane per dimension:
//   accept  - take the longest of the four steps that lowers E (the first in halving order);
//             when the candidates were evaluated with gradients the accepted one's becomes
//             the particle's gradient; no step lowers E: the particle stops refining;
//   propose - four candidates x - eta * (g_s / max|g_s|) / 2^j, j = 0..3, g_s = eta * dE/dh,
//             clamped to the bounds; a particle that has stopped (or whose g_s is zero or not
//             finite, which stops it) writes its own position four times, and its candidates
//             are skipped by the evaluation (its active flag is 0);
//   gather  - write the refined positions and costs back into the swarm.

// Cost of evaluated particle p and, with grad, lane j's component of its gradient (lanes past
// n_dof: 0), assembled by one wavefront.  W, org: this wavefront's LDS rows ([n_seg * 6]
// wrench sums, [n_seg * 4] segment origins).  Returns false for a particle that was skipped
// (not evaluated).  Holds no barrier.
__device__ bool assemble_wave(const EvalArgs& a, const Workspace& ws, int p, bool grad,
                              double* W, float* org, float& cost, float& g) {
  const int lane = threadIdx.x & (kWave - 1);
  const int n_seg = a.n_seg, n_dof = a.n_dof, nv = n_seg * 6;
  const int ps = uni(src_of(a, p));
  const int b = uni(ws.item_off[p]), e = uni(ws.item_off[p + 1]);
  // loads that depend on the particle alone, issued before any branch: the record, the first
  // partials, this lane's pose-parameter frame and segment-origin values (clamped indices)
  const PInfo pi = ws.pinfo[ps];
  const Partial pr0 = first_partial(ws, b, e, lane);
  const int jc = min(lane, n_dof - 1);
  const float4* f4 = reinterpret_cast<const float4*>(ws.dof_frame + ((size_t)ps * n_dof + jc) * 8);
  const float4 f0 = f4[0], f1 = f4[1];
  const uint32_t desc = lane < n_dof ? a.model->dof_desc[jc] : 0u;
  const float* org_src = ws.seg_org + (size_t)ps * n_seg * 4;
  const float o0 = org_src[min(lane, n_seg * 4 - 1)];
  const float o1 = org_src[min(lane + kWave, n_seg * 4 - 1)];
  double S_d;
  long long S_and, S_or;
  wave_partial_sums(pi, ws, b, e, lane, pr0, S_d, S_and, S_or);
  g = 0.0f;
  if (pi.skip) return false;
  if (!pi.valid) {
    cost = pi.slot < 0 ? NAN : INFINITY;
    return true;
  }
  cost = cost_from_sums(S_d, S_and, S_or, pi.kc);
  if (!grad) return true;
  // wrench rows summed in item order (lane l: values l, l + 64, l + 128), kAsmItems items'
  // loads in flight at a time (indices clamped into the particle's items; past the end adds
  // zero): each round is one memory latency, and small gradient launches give a particle
  // some 30 items
  constexpr int kAsmItems = 16;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int i0 = b; i0 < e; i0 += kAsmItems) {
    float v[kAsmItems][3];
#pragma unroll
    for (int u = 0; u < kAsmItems; ++u) {
      const float* src = ws.wrench + (size_t)min(i0 + u, e - 1) * nv;
#pragma unroll
      for (int k = 0; k < 3; ++k) v[u][k] = src[min(lane + k * kWave, nv - 1)];
    }
#pragma unroll
    for (int u = 0; u < kAsmItems; ++u)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        acc[k] += (i0 + u < e && lane + k * kWave < nv) ? (double)v[u][k] : 0.0;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if (lane + k * kWave < nv) W[lane + k * kWave] = acc[k];
  if (lane < n_seg * 4) org[lane] = o0;
  if (lane + kWave < n_seg * 4) org[lane + kWave] = o1;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // the kinematic adjoint of the finalize kernel, lane j = pose parameter j
  const int j = lane;
  if (j < n_dof) {
    const double inv_or = S_or > 0 ? 1.0 / (double)S_or : 0.0;
    const bool trans = f0.x != 0.0f;
    const double ax = f0.y, ay = f0.z, az = f0.w;
    double acc_g = 0.0;
    // the segments this parameter moves, in increasing order, kAdjRound per round: their LDS
    // reads are issued together (one segment per round waited on the reads of each in turn;
    // eight per round measured no faster than four)
    constexpr int kAdjRound = 4;
    for (uint32_t m = desc; m;) {
      int sg[kAdjRound];
      bool has[kAdjRound];
#pragma unroll
      for (int q = 0; q < kAdjRound; ++q) {
        has[q] = m != 0u;
        sg[q] = has[q] ? __builtin_ctz(m) : 0;
        m &= m - 1u;
      }
      double t[kAdjRound];
#pragma unroll
      for (int q = 0; q < kAdjRound; ++q) {
        const double* Ws = W + sg[q] * 6;
        const double lx = (double)org[sg[q] * 4 + 0] - f1.x;
        const double ly = (double)org[sg[q] * 4 + 1] - f1.y;
        const double lz = (double)org[sg[q] * 4 + 2] - f1.z;
        const double mx = Ws[0] + (ly * Ws[5] - lz * Ws[4]);
        const double my = Ws[1] + (lz * Ws[3] - lx * Ws[5]);
        const double mz = Ws[2] + (lx * Ws[4] - ly * Ws[3]);
        t[q] = trans ? ax * Ws[3] + ay * Ws[4] + az * Ws[5] : ax * mx + ay * my + az * mz;
      }
#pragma unroll
      for (int q = 0; q < kAdjRound; ++q)
        if (has[q]) acc_g += t[q];
    }
    acc_g *= inv_or;
    for (int m = pi.kc_mask; m; m &= m - 1) {
      const int i = __builtin_ctz(m);
      if (a.model->kc_a[i] == j) acc_g -= kLambdaK;
      if (a.model->kc_b[i] == j) acc_g += kLambdaK;
    }
    g = (float)acc_g;
  }
  return true;
}

__global__ __launch_bounds__(kBlock) void refine_update_kernel(EvalArgs a, Workspace ws,
                                                               RefineArgs ra) {
  __shared__ double s_W[kWavesPerBlock][HT_MAX_SEG * 6];
  __shared__ float s_org[kWavesPerBlock][HT_MAX_SEG * 4];
  __shared__ float s_cost[kWavesPerBlock];
  __shared__ float s_g[kWavesPerBlock][HT_MAX_DOF];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = blockIdx.x;                       // refined particle (frame * K + rank)
  const int n_dof = ra.n_dof;
  const bool on = lane < n_dof;
  const int d = on ? lane : 0;
  const size_t xi = (size_t)r * n_dof + d;
  // the inputs of wavefront 0's decisions below, loaded before the assembly so that their
  // latency overlaps it (no kernel writes them meanwhile; this one writes them only after
  // reading them); buffers a mode does not use are allocated, their values unused
  const int act_in = ra.active[r];
  const float x_in = ra.rx[xi], c_in = ra.rcost[r], g_in = ra.grad[xi];
  float cx_in[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) cx_in[j] = ra.cand[((size_t)r * 4 + j) * n_dof + d];
  const int trans_in = a.model->dof_trans[d];
  const float lo_in = a.model->lo[d], hi_in = a.model->hi[d];
  // 1. the preceding evaluation: the particle itself (propose only), else its candidates
  const bool mine = ra.op.accept ? true : w == 0;
  if (mine) {
    const int p = ra.op.accept ? r * 4 + w : r;
    float c = INFINITY, g = 0.0f;
    if (!assemble_wave(a, ws, p, ra.eval_grad, s_W[w], s_org[w], c, g)) c = INFINITY;
    if (lane == 0) s_cost[w] = c;
    if (lane < HT_MAX_DOF) s_g[w][lane] = g;
  }
  __syncthreads();
  if (w != 0) return;
  bool act = act_in != 0;
  float x = x_in;
  float c, gd;
  if (!ra.op.accept) {
    // the gradient evaluation of the selected particle: its cost and gradient
    c = s_cost[0];
    gd = s_g[0][d];
    if (on) ra.grad[xi] = gd;
    if (lane == 0) ra.rcost[r] = c;
  } else {
    c = c_in;
    gd = g_in;
  }
  if (ra.op.accept && act) {
    // the four candidates' costs (a skipped one counts as +inf) and positions
    float cc[4], cx[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      cc[j] = s_cost[j];
      cx[j] = cx_in[j];
    }
    int pick = -1;
#pragma unroll
    for (int j = 3; j >= 0; --j)
      if (cc[j] < c) pick = j;
    if (pick < 0) {
      act = false;
      if (lane == 0) ra.active[r] = 0;
    } else {
      float nx = cx[0], ng = s_g[0][d];
      c = cc[0];
#pragma unroll
      for (int j = 1; j < 4; ++j) {
        nx = pick == j ? cx[j] : nx;
        ng = pick == j ? s_g[j][d] : ng;
        c = pick == j ? cc[j] : c;
      }
      x = nx;
      if (on) {
        ra.rx[xi] = x;
        if (ra.eval_grad) {
          gd = ng;
          ra.grad[xi] = gd;
        }
      }
      if (lane == 0) ra.rcost[r] = c;
    }
  }
  if (ra.op.propose) {
    const float eta = trans_in ? ra.eta_trans : ra.eta_rot;
    const float gs = on ? eta * gd : 0.0f;
    float gmax = fabsf(gs);
    bool fin = isfinite(gs);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) gmax = fmaxf(gmax, __shfl_xor(gmax, o));
    fin = __ballot(!fin) == 0ull;
    const bool ok = act && fin && gmax > 0.0f;
    // a particle without a usable step stops refining: its candidates are not evaluated
    if (act && !ok && lane == 0) ra.active[r] = 0;
    if (on) {
      for (int j = 0; j < 4; ++j) {
        float xn = x;
        if (ok) {
          const float step = eta * (gs / gmax) * ldexpf(1.0f, -j);
          xn = fminf(fmaxf(x - step, lo_in), hi_in);
        }
        ra.cand[((size_t)r * 4 + j) * n_dof + d] = xn;
      }
    }
  }
  if (ra.op.gather) {
    const int f = r / ra.K;
    if (ra.sw.stop_gen && ra.sw.stop_gen[f] != 0) return;
    const size_t gp = (size_t)f * ra.sw.n_particles + ra.sel[r];
    if (on) ra.sw.x[gp * n_dof + d] = x;
    if (lane == 0) ra.sw.cost[gp] = c;
  }
}

hipError_t launch_refine_update(const EvalArgs& a, const Workspace& ws, const RefineArgs& ra,
                                hipStream_t s) {
  if (ra.n_ref == 0) return hipSuccess;
  hipLaunchKernelGGL(refine_update_kernel, dim3(ra.n_ref), dim3(kBlock), 0, s, a, ws, ra);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------

// The ray-cast variant of a launch.
template <bool GRAD, int NT>
static const void* raycast_fn_nt(bool dbg, bool self) {
  if (dbg) return reinterpret_cast<const void*>(&raycast_kernel<GRAD, true, NT, false>);
  return self ? reinterpret_cast<const void*>(&raycast_kernel<GRAD, false, NT, true>)
              : reinterpret_cast<const void*>(&raycast_kernel<GRAD, false, NT, false>);
}

static const void* raycast_fn(bool grad, bool dbg, bool all_types, bool self) {
  if (all_types)
    return grad ? raycast_fn_nt<true, kNumTypes>(dbg, self)
                : raycast_fn_nt<false, kNumTypes>(dbg, self);
  return grad ? raycast_fn_nt<true, 3>(dbg, self) : raycast_fn_nt<false, 3>(dbg, self);
}

// Workgroups of a ray-cast variant that are resident on one CU at once (its registers and
// LDS decide).  The persistent grid is capped at this many per CU: a workgroup beyond it
// starts only when another has finished, and its statically assigned first item then
// finishes late (a 128-particle launch spent half its time in that tail).
int raycast_groups_per_cu(bool grad, bool dbg, bool all_types, bool self) {
  self = self && !dbg;
  static int cache[2][2][2][2] = {};
  int& n = cache[grad][dbg][all_types][self];
  if (n > 0) return n;
  const void* f = raycast_fn(grad, dbg, all_types, self);
  int r = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&r, f, kBlock, 0) != hipSuccess || r < 1) {
    (void)hipGetLastError();
    r = 1;
  }
  n = r;
  return n;
}

// The evaluation is four launches on one stream; `stage` selects one so the host can
// bracket each with HIP events when profiling.
hipError_t launch_eval_stage(int stage, const EvalArgs& a, const Workspace& ws, hipStream_t s) {
  const int n_total = a.n_frames * a.n_particles;
  if (n_total == 0) return hipSuccess;
  const bool dbg = a.dbg.depth || a.dbg.hit || a.dbg.rm || a.dbg.winner || a.dbg.margin;
  switch (stage) {
    case kStageFk:
      if (a.src) break;   // the kinematics of the previous evaluation are reused
      if (a.n_prim > kWave)
        hipLaunchKernelGGL(fk_kernel<2>, dim3((n_total + kWavesPerBlock / 2 - 1) / (kWavesPerBlock / 2)),
                           dim3(kBlock), 0, s, a, ws);
      else
        hipLaunchKernelGGL(fk_kernel<1>, dim3((n_total + kWavesPerBlock - 1) / kWavesPerBlock),
                           dim3(kBlock), 0, s, a, ws);
      break;
    case kStageSched:
      if (a.self_sched) return hipErrorInvalidValue;   // the ray cast builds its work list
      if (n_total <= kSchedSmall)
        hipLaunchKernelGGL(sched_kernel<kSchedSmall>, dim3(1), dim3(kSchedSmall), 0, s, a, ws);
      else
        hipLaunchKernelGGL(sched_kernel<kSchedBlock>, dim3(1), dim3(kSchedBlock), 0, s, a, ws);
      if (dbg) {
        const size_t n = (size_t)a.n_particles * a.dbg_H * a.dbg_W;
        hipLaunchKernelGGL(debug_fill_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)),
                           dim3(kBlock), 0, s, a.dbg, n, a.dbg_bg);
      }
      break;
    case kStageRaycast: {
      const TypeMasks tm = a.type_masks;
      const bool all = (tm.m[HT_CONE][0] | tm.m[HT_CONE][1] | tm.m[HT_ECYLINDER][0] |
                        tm.m[HT_ECYLINDER][1]) != 0ull;
      if (a.self_sched && (dbg || n_total > kSelfSched)) return hipErrorInvalidValue;
      const void* f = raycast_fn(a.grad != nullptr, dbg, all, a.self_sched != 0);
      EvalArgs ka = a;
      Workspace kw = ws;
      TypeMasks kt = tm;
      void* args[] = {&ka, &kw, &kt};
      return hipLaunchKernel(f, dim3(a.grid), dim3(kBlock), args, 0, s);
    }
    case kStageFinalize:
      if (a.grad)
        hipLaunchKernelGGL(finalize_grad_kernel, dim3(n_total), dim3(kBlock), 0, s, a, ws);
      else
        hipLaunchKernelGGL(finalize_kernel, dim3((n_total + kWavesPerBlock - 1) / kWavesPerBlock),
                           dim3(kBlock), 0, s, a, ws);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ht
