// Particle swarm kernels: initialisation, the generation update of Eq. 6-7 with the mutation
// of section III.B, and the selection of the particles that gradient refinement starts from
// (its update kernel, fused with assembling the evaluations, is in ht_kernels.hip).
//
// Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by the 64-bit seed, counter
// (dimension, frame * P + particle, generation, stream); uniform = (word >> 8) * 2^-24.
// Stream 0 gives r1 (word 0) and r2 (word 1) of Eq. 6, stream 1 the initial positions,
// stream 2 the mutation re-draws.
//
// A generation's update is two launches: `pso_best_kernel` (one workgroup per frame: personal
// and global bests, the mutation ranking, the generation counter) and `pso_move_kernel` (one
// thread per particle dimension: personal-best copy, then mutation or Eq. 6-7 with clamping).
#include <math.h>

#include "ht_device.h"

namespace ht {

namespace {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u, kPhiloxW1 = 0xBB67AE85u;

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += kPhiloxW0;
      k1 += kPhiloxW1;
    }
    const uint32_t hi0 = __umulhi(kPhiloxM0, c.x), lo0 = kPhiloxM0 * c.x;
    const uint32_t hi1 = __umulhi(kPhiloxM1, c.z), lo1 = kPhiloxM1 * c.z;
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}

__device__ __forceinline__ float unit(uint32_t w) { return (float)(w >> 8) * 0x1.0p-24f; }

__device__ __forceinline__ uint4 draw(uint64_t seed, int dim, int gpart, int gen, int stream) {
  return philox4x32_10(make_uint4((uint32_t)dim, (uint32_t)gpart, (uint32_t)gen, (uint32_t)stream),
                       (uint32_t)seed, (uint32_t)(seed >> 32));
}

// The swarm's Philox key: read from device memory when the swarm has a device seed (so that a
// captured run replays with new random numbers once the caller writes it), else the seed.
__device__ __forceinline__ uint64_t swarm_key(const ht_swarm& sw) {
  return sw.seed_dev ? *sw.seed_dev : sw.seed;
}

__device__ __forceinline__ float cost_key(float c) { return isnan(c) ? INFINITY : c; }

// A (cost, index) pair as one 64-bit key: the cost's bits mapped to an unsigned integer of the
// same order (negative floats inverted, others with the sign bit set; NaN counted as +inf and
// -0 as +0) above the index, so one unsigned compare orders by cost and then by index.
__device__ __forceinline__ uint64_t select_key(float c, int i) {
  const uint32_t b = __float_as_uint(cost_key(c) + 0.0f);
  const uint32_t u = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
  return ((uint64_t)u << 32) | (uint32_t)i;
}

__device__ __forceinline__ float select_cost(uint64_t key) {
  const uint32_t u = (uint32_t)(key >> 32);
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u);
}

// per-particle flags from part 1 to part 2 of a generation: personal best improved, mutated,
// the frame stopped in this generation (bests kept, no move), the frame had stopped before
constexpr int kFlagImproved = 1, kFlagMutated = 2, kFlagStop = 4, kFlagFrozen = 8;
constexpr int kPsoBlock = 1024;

int threads_for(int n) { return n >= kPsoBlock ? kPsoBlock : ((n + kWave - 1) / kWave) * kWave; }

int pow2_at_least(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

// Sort the P costs of a frame ascending by (cost, particle index) with a bitonic network in
// LDS: key[i], idx[i] for i < n_pad (a power of two); entries past P sort last.  Afterwards
// position r holds the particle of rank r, so the K best are positions 0..K-1 (ties: lower
// index first) and the worst are the last positions (ties: the higher index is worse).
__device__ void sort_costs(const float* __restrict__ cost, int P, int n_pad, float* key,
                           int* idx) {
  for (int i = threadIdx.x; i < n_pad; i += blockDim.x) {
    key[i] = i < P ? cost_key(cost[i]) : INFINITY;
    idx[i] = i;                     // padding indices exceed every particle index
  }
  __syncthreads();
  for (int k = 2; k <= n_pad; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n_pad; i += blockDim.x) {
        const int l = i ^ j;
        if (l <= i) continue;
        const float ki = key[i], kl = key[l];
        const int ii = idx[i], il = idx[l];
        const bool i_after_l = ki > kl || (ki == kl && ii > il);
        if (i_after_l == ((i & k) == 0)) {
          key[i] = kl;
          key[l] = ki;
          idx[i] = il;
          idx[l] = ii;
        }
      }
      __syncthreads();
    }
  }
}

}  // namespace

// ------------------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void pso_init_kernel(const DevModel* __restrict__ M,
                                                          ht_swarm sw, int n_dof) {
  const int F = sw.n_frames, P = sw.n_particles;
  const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  const size_t n = (size_t)F * P * n_dof;
  if (i < n) {
    const int d = (int)(i % n_dof);
    const int gp = (int)(i / n_dof);
    const int f = gp / P;
    const float lo = fmaxf(sw.init_lo[(size_t)f * n_dof + d], M->lo[d]);
    const float hi = fminf(sw.init_hi[(size_t)f * n_dof + d], M->hi[d]);
    const float u = unit(draw(swarm_key(sw), d, gp, 0, 1).x);
    const float x = fminf(fmaxf(fmaf(u, hi - lo, lo), lo), hi);
    sw.x[i] = x;
    sw.v[i] = 0.0f;
    sw.pbest_x[i] = x;
    if (gp % P == 0) sw.gbest_x[(size_t)f * n_dof + d] = x;
    if (d == 0) {
      sw.pbest_cost[gp] = INFINITY;
      sw.cost[gp] = INFINITY;
      if (gp % P == 0) {
        sw.gbest_cost[f] = INFINITY;
        sw.gen[f] = 0;
        if (sw.stop_gen) sw.stop_gen[f] = 0;
      }
    }
  }
}

hipError_t launch_pso_init(const DevModel* model, const ht_swarm& sw, int n_dof, hipStream_t s) {
  const size_t n = (size_t)sw.n_frames * sw.n_particles * n_dof;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(pso_init_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                     0, s, model, sw, n_dof);
  return hipGetLastError();
}

// tracking box: clamp(center) -/+ halfwidth within the model bounds, one thread per entry
__global__ __launch_bounds__(kBlock) void box_around_kernel(const DevModel* __restrict__ M,
                                                            int n, int n_dof,
                                                            const float* __restrict__ center,
                                                            const float* __restrict__ hw,
                                                            float* __restrict__ lo,
                                                            float* __restrict__ hi) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int d = i % n_dof;
  const float c = fminf(fmaxf(center[i], M->lo[d]), M->hi[d]);
  lo[i] = fmaxf(c - hw[d], M->lo[d]);
  hi[i] = fminf(c + hw[d], M->hi[d]);
}

hipError_t launch_box_around(const DevModel* model, int n_frames, int n_dof, const float* center,
                             const float* halfwidth, float* lo, float* hi, hipStream_t s) {
  const int n = n_frames * n_dof;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(box_around_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                     model, n, n_dof, center, halfwidth, lo, hi);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// Ascending bitonic sort of one 64-bit key per thread across the workgroup (blockDim.x a
// power of two, at most kPsoBlock): exchanges between lanes of a wavefront are lane shuffles,
// wider ones go through LDS with a barrier (10 of the 55 steps at 1024 threads).  Returns the
// key of rank threadIdx.x.
__device__ uint64_t block_sort_keys(uint64_t k, uint64_t* s_x) {
  const int t = threadIdx.x, n = blockDim.x;
  for (int size = 2; size <= n; size <<= 1) {
    for (int j = size >> 1; j > 0; j >>= 1) {
      uint64_t pk;
      if (j >= kWave) {
        s_x[t] = k;
        __syncthreads();
        pk = s_x[t ^ j];
        __syncthreads();
      } else {
        pk = __shfl_xor(k, j);
      }
      const bool up = (t & size) == 0, lower = (t & j) == 0;
      const bool take = lower == up ? pk < k : k < pk;
      k = take ? pk : k;
    }
  }
  return k;
}

// generation update, part 1: one workgroup per frame

__global__ __launch_bounds__(kPsoBlock) void pso_best_kernel(ht_swarm sw, ht_pso_params prm,
                                                             int n_dof, int n_pad,
                                                             int* __restrict__ flags) {
  extern __shared__ float s_mem[];
  const int P = sw.n_particles;
  float* s_pb = s_mem;                                  // [P] personal bests after this step
  float* s_key = s_mem + P;                             // [n_pad] sort keys
  int* s_idx = reinterpret_cast<int*>(s_key + n_pad);   // [n_pad] sort payload
  __shared__ float s_rv[kPsoBlock / kWave];
  __shared__ int s_ri[kPsoBlock / kWave];
  __shared__ int s_g;
  const int f = blockIdx.x, tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wv = tid / kWave;
  const int gen = sw.gen[f];
  const size_t base = (size_t)f * P;
  if (sw.stop_gen && sw.stop_gen[f] != 0) {   // stopped earlier: nothing changes
    for (int i = tid; i < P; i += blockDim.x) flags[base + i] = kFlagFrozen;
    return;
  }

  for (int i = tid; i < P; i += blockDim.x) {
    const float c = cost_key(sw.cost[base + i]);
    float pb = sw.pbest_cost[base + i];
    int fl = 0;
    if (c < pb) {
      pb = c;
      sw.pbest_cost[base + i] = c;
      fl = kFlagImproved;
    }
    s_pb[i] = pb;
    flags[base + i] = fl;
  }
  __syncthreads();

  // global best: lowest personal-best cost, ties to the lowest index
  float bv = INFINITY;
  int bi = INT_MAX;
  for (int i = tid; i < P; i += blockDim.x) {
    const float v = s_pb[i];
    if (v < bv || (v == bv && i < bi)) {
      bv = v;
      bi = i;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const float ov = __shfl_xor(bv, o);
    const int oi = __shfl_xor(bi, o);
    if (ov < bv || (ov == bv && oi < bi)) {
      bv = ov;
      bi = oi;
    }
  }
  if (lane == 0) {
    s_rv[wv] = bv;
    s_ri[wv] = bi;
  }
  __syncthreads();
  if (tid == 0) {
    float v = s_rv[0];
    int idx = s_ri[0];
    for (int q = 1; q < (int)blockDim.x / kWave; ++q) {
      if (s_rv[q] < v || (s_rv[q] == v && s_ri[q] < idx)) {
        v = s_rv[q];
        idx = s_ri[q];
      }
    }
    // all personal bests +inf (no finite cost yet): keep particle 0
    s_g = idx == INT_MAX ? 0 : idx;
    sw.gbest_cost[f] = s_pb[s_g];
  }
  __syncthreads();
  const int g = s_g;
  // the global best position is the best particle's personal best, which is its current
  // position if it improved in this generation (read before any position moves)
  const bool g_improved = (flags[base + g] & kFlagImproved) != 0;
  for (int d = tid; d < n_dof; d += blockDim.x)
    sw.gbest_x[(size_t)f * n_dof + d] =
        g_improved ? sw.x[(base + g) * n_dof + d] : sw.pbest_x[(base + g) * n_dof + d];

  // stop rule: the best cost is below the threshold after this generation's evaluation
  const bool stop = sw.stop_gen && prm.stop_cost > 0.0f && s_pb[g] < prm.stop_cost;
  const bool mutate_gen = prm.mutate_every > 0 && (gen + 1) % prm.mutate_every == 0;
  const int n_mut = (int)floorf((float)P * prm.mutate_frac);
  if (stop) {
    for (int i = tid; i < P; i += blockDim.x) flags[base + i] |= kFlagStop;
  } else if (mutate_gen && n_mut > 0) {
    // the worst n_mut by current cost are the last positions of the ascending sort (ties: the
    // higher index is worse)
    if (n_pad == (int)blockDim.x) {   // one key per thread
      __shared__ uint64_t s_x[kPsoBlock];
      const uint64_t k = block_sort_keys(
          select_key(tid < P ? sw.cost[base + min(tid, P - 1)] : INFINITY, tid), s_x);
      if (tid >= P - n_mut && tid < P) flags[base + (uint32_t)k] |= kFlagMutated;
    } else {
      sort_costs(sw.cost + base, P, n_pad, s_key, s_idx);
      for (int r = P - n_mut + tid; r < P; r += blockDim.x)
        flags[base + s_idx[r]] |= kFlagMutated;
    }
  }
  __syncthreads();
  if (tid == 0) {
    sw.gen[f] = gen + 1;
    if (stop) sw.stop_gen[f] = gen + 1;
  }
}

// generation update, part 2: one thread per (frame, particle, dimension)
__global__ __launch_bounds__(kBlock) void pso_move_kernel(const DevModel* __restrict__ M,
                                                          ht_swarm sw, ht_pso_params prm,
                                                          int n_dof,
                                                          const int* __restrict__ flags) {
  const int P = sw.n_particles;
  const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= (size_t)sw.n_frames * P * n_dof) return;
  const int d = (int)(i % n_dof);
  const int gp = (int)(i / n_dof);
  const int f = gp / P;
  const int gen = sw.gen[f] - 1;            // part 1 already advanced the counter
  const int fl = flags[gp];
  if (fl & kFlagFrozen) return;
  const float xd = sw.x[i];
  float pb = sw.pbest_x[i];
  if (fl & kFlagImproved) {
    pb = xd;
    sw.pbest_x[i] = xd;
  }
  if (fl & kFlagStop) return;
  const float lo = M->lo[d], hi = M->hi[d];
  if (fl & kFlagMutated) {
    if (M->mutate[d]) {
      const float u = unit(draw(swarm_key(sw), d, gp, gen, 2).x);
      sw.x[i] = fmaf(u, hi - lo, lo);
      sw.v[i] = 0.0f;
    }
    return;
  }
  const uint4 r = draw(swarm_key(sw), d, gp, gen, 0);
  const float r1 = unit(r.x), r2 = unit(r.y);
  const float gb = sw.gbest_x[(size_t)f * n_dof + d];
  const float t = fmaf(prm.c2 * r2, gb - xd, fmaf(prm.c1 * r1, pb - xd, sw.v[i]));
  float vn = prm.w * t;
  float xn = xd + vn;
  if (xn < lo) {
    xn = lo;
    vn = 0.0f;
  } else if (xn > hi) {
    xn = hi;
    vn = 0.0f;
  }
  sw.x[i] = xn;
  sw.v[i] = vn;
}

hipError_t launch_pso_update(const DevModel* model, const ht_swarm& sw, const ht_pso_params& p,
                             int n_dof, int* flags, hipStream_t s) {
  if (sw.n_frames == 0 || sw.n_particles == 0) return hipSuccess;
  const int n_pad = pow2_at_least(sw.n_particles);
  const size_t shm = (size_t)sw.n_particles * sizeof(float) + (size_t)n_pad * 8;
  hipLaunchKernelGGL(pso_best_kernel, dim3(sw.n_frames), dim3(threads_for(sw.n_particles)), shm,
                     s, sw, p, n_dof, n_pad, flags);
  const size_t n = (size_t)sw.n_frames * sw.n_particles * n_dof;
  hipLaunchKernelGGL(pso_move_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                     0, s, model, sw, p, n_dof, flags);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// gradient refinement
//
// select: the K lowest current costs of each frame (ties: lower index first), copied into
// the refinement buffers.  The steps that follow (propose four step lengths 1, 1/2, 1/4, 1/8
// of the normalised steepest-descent step in the eta-scaled space; accept the first length
// whose cost is lower than the current one, else stop refining; gather back into the swarm)
// are the update kernel in ht_kernels.hip.

__global__ __launch_bounds__(kPsoBlock) void refine_select_kernel(ht_swarm sw, int K, int n_dof,
                                                                  int n_pad,
                                                                  int* __restrict__ sel,
                                                                  float* __restrict__ rx,
                                                                  float* __restrict__ rcost,
                                                                  int* __restrict__ active) {
  extern __shared__ float s_key[];
  int* s_idx = reinterpret_cast<int*>(s_key + n_pad);
  const int P = sw.n_particles, f = blockIdx.x;
  const size_t base = (size_t)f * P;
  sort_costs(sw.cost + base, P, n_pad, s_key, s_idx);
  for (int r = threadIdx.x; r < K; r += blockDim.x) {
    const size_t q = (size_t)f * K + r;
    sel[q] = s_idx[r];
    rcost[q] = s_key[r];
    active[q] = 1;
  }
  for (int e = threadIdx.x; e < K * n_dof; e += blockDim.x) {
    const int r = e / n_dof, d = e % n_dof;
    rx[((size_t)f * K + r) * n_dof + d] = sw.x[(base + s_idx[r]) * n_dof + d];
  }
}

// Select for up to 1024 particles and K <= 64 without a full sort: every wavefront sorts its
// 64 (cost, index) pairs with a bitonic network across its lanes, then sorted lists are merged
// pairwise in rounds keeping the first K (an element's rank in the union of two sorted lists
// is its own position plus the number of the other list's elements before it; the keys are
// unique, so the ranks are distinct).  The K lowest, ties by lower index, as the full sort.


// Elements of the sorted list x[0 .. n) (n <= 64) below key: a binary search with a fixed trip
// count (loads clamped into the list, selects instead of branches).
__device__ __forceinline__ int count_below(const uint64_t* x, int n, uint64_t key) {
  int pos = 0;
#pragma unroll
  for (int step = kWave; step > 0; step >>= 1) {
    const int q = min(pos + step, n) - 1;
    const bool ok = pos + step <= n && x[q] < key;
    pos = ok ? pos + step : pos;
  }
  return pos;
}

__global__ __launch_bounds__(kPsoBlock) void refine_select_small_kernel(
    ht_swarm sw, int K, int n_dof, int* __restrict__ sel, float* __restrict__ rx,
    float* __restrict__ rcost, int* __restrict__ active) {
  __shared__ uint64_t s_k[2][kPsoBlock / kWave][kWave];
  const int P = sw.n_particles, f = blockIdx.x;
  const size_t base = (size_t)f * P;
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x >> 6;
  int nl = blockDim.x / kWave;                  // sorted lists
  // 1. bitonic sort of each wavefront's 64 entries (padding: +inf, indices past P); the cost
  // load is clamped into the frame and replaced for padding lanes
  const int e = w * kWave + lane;
  const float c = sw.cost[base + min(e, P - 1)];
  uint64_t k = select_key(e < P ? c : INFINITY, e);
  for (int size = 2; size <= kWave; size <<= 1) {
    for (int j = size >> 1; j > 0; j >>= 1) {
      const uint64_t pk = __shfl_xor(k, j);
      const bool up = (lane & size) == 0, lower = (lane & j) == 0;
      const bool take = lower == up ? pk < k : k < pk;
      k = take ? pk : k;
    }
  }
  s_k[0][w][lane] = k;
  __syncthreads();
  // 2. pairwise merges keeping the first K of each union
  int cur = 0;
  while (nl > 1) {
    const int pairs = nl >> 1;
    if (w < pairs && lane < K) {
      const uint64_t* a = s_k[cur][2 * w];
      const uint64_t* b = s_k[cur][2 * w + 1];
      const uint64_t ka = a[lane], kb = b[lane];
      const int ra = lane + count_below(b, K, ka);
      const int rb = lane + count_below(a, K, kb);
      if (ra < K) s_k[cur ^ 1][w][ra] = ka;
      if (rb < K) s_k[cur ^ 1][w][rb] = kb;
    }
    if ((nl & 1) && w == pairs && lane < K)      // odd list passes through
      s_k[cur ^ 1][w][lane] = s_k[cur][nl - 1][lane];
    __syncthreads();
    nl = pairs + (nl & 1);
    cur ^= 1;
  }
  // 3. the K best, and their positions gathered (up to four per thread, loads issued first,
  // offsets clamped into the K x n_dof block)
  const uint64_t* best = s_k[cur][0];
  for (int r = threadIdx.x; r < K; r += blockDim.x) {
    const size_t q = (size_t)f * K + r;
    sel[q] = (int)(uint32_t)best[r];
    rcost[q] = select_cost(best[r]);
    active[q] = 1;
  }
  const int n = K * n_dof;
  for (int x0 = 0; x0 < n; x0 += 4 * (int)blockDim.x) {
    float v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int x = min(x0 + u * (int)blockDim.x + (int)threadIdx.x, n - 1);
      const int r = x / n_dof, d = x - r * n_dof;
      v[u] = sw.x[(base + (uint32_t)best[r]) * n_dof + d];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int x = x0 + u * (int)blockDim.x + (int)threadIdx.x;
      if (x < n) rx[(size_t)f * n + x] = v[u];
    }
  }
}

hipError_t launch_refine_select(const ht_swarm& sw, int K, int n_dof, int* sel, float* rx,
                                float* rcost, int* active, hipStream_t s) {
  if (sw.n_particles <= kPsoBlock && K <= kWave) {
    hipLaunchKernelGGL(refine_select_small_kernel, dim3(sw.n_frames),
                       dim3(threads_for(sw.n_particles)), 0, s, sw, K, n_dof, sel, rx, rcost,
                       active);
    return hipGetLastError();
  }
  const int n_pad = pow2_at_least(sw.n_particles);
  hipLaunchKernelGGL(refine_select_kernel, dim3(sw.n_frames), dim3(threads_for(sw.n_particles)),
                     (size_t)n_pad * 8, s, sw, K, n_dof, n_pad, sel, rx, rcost, active);
  return hipGetLastError();
}

}  // namespace ht
