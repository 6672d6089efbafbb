/*
 * handtrack.h -- C ABI of libhandtrack.so, the MI355X (gfx950) hot path of model-based
 * 26-DOF hand tracking: score particle-swarm particles (hand poses) against an RGB-D
 * observation and move the swarm.
 *
 * What is computed (paper: "Recognition of 26 Degrees of Freedom of Hands Using Model-based
 * approach and Depth-Color Images", arXiv:2005.07068):
 *   - a pose h is the 26-vector of Eq. 1-3 (five fingers x (MP flexion, MP abduction, PIP,
 *     DIP), then wrist x, y, z, theta_x, theta_y, theta_z); a two-hand particle is 52-D;
 *   - the model depth image r_d(h, C) of section III.A is the exact nearest entry depth of a
 *     hand built from spheres, ellipsoids, closed truncated cones, closed elliptic and
 *     circular cylinders (section II.A) along each pixel ray;
 *   - the cost is E(h, O) = D(O, h, C) + lambda_k kc(h) of Eq. 4-5 with d_m = 10 mm,
 *     d_M = 40 mm, lambda = 20, lambda_k = 10, sums over every ROI pixel;
 *   - the swarm moves by Eq. 6-7 with bounds (Tables 1-2) and the mutation of section III.B.
 *
 * Conventions shared by every call:
 *   - Status: every entry point returns HT_OK or a negative ht_status and never throws;
 *     ht_last_error() gives a thread-local message for the last failure.  Arguments are
 *     validated on the host before anything is enqueued; on an error nothing is enqueued.
 *   - Asynchrony: eval / grad / pso calls only enqueue work on the given HIP stream (NULL =
 *     the legacy default stream) and never synchronise, so they can be captured in a HIP
 *     graph once the context's workspace is reserved (ht_reserve); without a reservation a
 *     call may grow the workspace with hipMalloc, which is refused during capture.
 *   - Memory: "device" pointers are HIP device memory owned by the caller and must stay alive
 *     until the enqueued work completes; the library deep-copies the model and observations
 *     into memory owned by the context.
 *   - Layout: poses are float32 [n_frames][n_particles][n_dof] row-major; costs are
 *     float32 [n_frames][n_particles]; images are row-major [H][W].
 *   - Non-finite pose components give cost = +inf and a zero gradient (not an error).
 *   - A context is bound to one HIP device and is not thread-safe.
 */
#ifndef HANDTRACK_H
#define HANDTRACK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ht_ctx ht_ctx;

typedef enum {
  HT_OK = 0,
  HT_ERR_ARG = -1,          /* NULL pointer, size out of range, inconsistent shapes        */
  HT_ERR_STATE = -2,        /* call before set_model / set_observation, unset frame slot   */
  HT_ERR_OOM = -3,          /* device allocation failed                                    */
  HT_ERR_HIP = -4,          /* a HIP runtime call failed (message names it)                */
  HT_ERR_UNSUPPORTED = -5   /* valid request outside what this library supports            */
} ht_status;

enum { HT_SPHERE = 0, HT_CYLINDER = 1, HT_ELLIPSOID = 2, HT_CONE = 3, HT_ECYLINDER = 4 };
enum { HT_PTR_HOST = 0, HT_PTR_DEVICE = 1 };

/* Limits of this library. */
#define HT_MAX_DOF 64
#define HT_MAX_SEG 32
#define HT_MAX_PRIM 128
#define HT_MAX_KC 16
#define HT_MAX_SLOTS 1024
#define HT_MAX_ROI 4096

/* Message of the last failed call on this thread ("" if none).  Valid until the next call. */
const char* ht_last_error(void);

/* Library version string. */
const char* ht_version(void);

/* Create a context on HIP device `hip_device`.  *out is set on success. */
ht_status ht_create(ht_ctx** out, int hip_device);

/* Destroy a context and free everything it owns.  NULL is a no-op.  The caller must make
 * sure no enqueued work of this context is still running. */
void ht_destroy(ht_ctx* ctx);

/* Hand model (section II.A), read from host memory and deep-copied to the device.
 * Kinematics: segment s is placed by parent * offset_s * Rot(axis_s0, h[dof_s0]) *
 * Rot(axis_s1, h[dof_s1]); a root segment (parent -1) is placed by the six wrist parameters
 * h[root_dof .. root_dof + 5] = (x, y, z, theta_x, theta_y, theta_z) as
 * Trans(x, y, z) Rz(theta_z) Ry(theta_y) Rx(theta_x) * offset_s (Eq. 2; the rotation order is
 * this library's reading).  Parents must precede their children.
 * Primitives: type, segment, local frame (3x4 in the segment frame) and sizes:
 *   HT_SPHERE     centre = frame origin, radius = size[0]
 *   HT_CYLINDER   closed, flat caps; first cap centre = frame origin, axis = frame z,
 *                 radius = size[0], length = size[1]
 *   HT_ELLIPSOID  centre = frame origin, semi-axes size[0..2] along frame x, y, z
 *   HT_CONE       truncated cone (the phalanges of section II.A), closed, flat caps; first
 *                 cap centre = frame origin, axis = frame z, radius size[0] at the first cap,
 *                 length size[1], radius size[2] at the second cap
 *   HT_ECYLINDER  elliptic cylinder (the palm of section II.A), closed, flat caps; first cap
 *                 centre = frame origin, axis = frame z, semi-axes size[0] along frame x and
 *                 size[2] along frame y, length size[1]
 * kc (Eq. 5): sum over pairs of max(-(h[a] - h[b]), 0).
 * Errors: HT_ERR_ARG for counts beyond the limits, a bad parent order, a non-unit axis, a
 * dof index out of range, non-positive sizes or lo > hi. */
typedef struct {
  int32_t n_dof, n_seg, n_prim, n_kc;
  const int32_t* seg_parent;     /* [n_seg], -1 = root                                      */
  const int32_t* seg_root_dof;   /* [n_seg], first wrist dof of a root, else ignored         */
  const double* seg_offset;      /* [n_seg][3][4] rotation | translation, mm                 */
  const double* seg_joint_axis;  /* [n_seg][2][3] unit axes in the segment frame             */
  const int32_t* seg_joint_dof;  /* [n_seg][2], -1 = no joint                                */
  const int32_t* prim_type;      /* [n_prim] HT_SPHERE .. HT_ECYLINDER                        */
  const int32_t* prim_seg;       /* [n_prim]                                                 */
  const double* prim_frame;      /* [n_prim][3][4]                                           */
  const double* prim_size;       /* [n_prim][3], mm                                          */
  const double* bounds_lo;       /* [n_dof] joint limits (Tables 1-2), rad / mm              */
  const double* bounds_hi;       /* [n_dof]                                                  */
  const uint8_t* mutate_mask;    /* [n_dof] 1 = re-drawn by the mutation step                */
  const int32_t* kc_pairs;       /* [n_kc][2] (a, b): a is the finger nearer the thumb       */
} ht_model;

ht_status ht_set_model(ht_ctx* ctx, const ht_model* model);

/* The checks of ht_set_model without a context or a device: HT_OK or HT_ERR_ARG. */
ht_status ht_check_model(const ht_model* model);

/* Pinhole camera C of section III.A (pixels); depth is camera z in mm.  The ray of pixel
 * (u, v) has direction ((u - cx)/fx, (v - cy)/fy, 1). */
typedef struct {
  float fx, fy, cx, cy;
} ht_camera;

/* Observation O = (O_s, O_d) of section II.B for frame slot `frame_slot` (0..HT_MAX_SLOTS-1):
 * depth_mm [H][W] (0 = undefined), skin [H][W] (nonzero = skin), camera and the background
 * plane depth B (model misses render B; B <= 0 means no plane and misses render 0).
 * `ptr_kind` says whether depth_mm / skin are host or device pointers.  The data are copied
 * (stream-ordered on hip_stream); the caller may free them once the stream has passed this
 * call.  May allocate (set-up call: not for graph capture).
 * Errors: HT_ERR_ARG for W or H outside 1..HT_MAX_ROI, a bad slot, NULL data, fx or fy <= 0. */
ht_status ht_set_observation(ht_ctx* ctx, int frame_slot, int W, int H, const uint16_t* depth_mm,
                             const uint8_t* skin, ht_camera cam, float bg_depth_mm,
                             int ptr_kind, void* hip_stream);

/* Gradient pixel mask of frame slot `frame_slot`: mask [H][W] with the slot's ROI size (the W,
 * H of its ht_set_observation), nonzero = the pixel contributes to dE/dh (the cost is never
 * masked).  Every gradient evaluation of a frame held in this slot (ht_eval_particles_grad with
 * any n_frames, the swarm's refinement) then leaves out the pixels it excludes; a call's own
 * pixel_mask, where given, is used instead.  This is the per-frame mask of the finite-difference
 * protocol of the gradient (the gradient is not in the paper; its cost is Eq. 4-5).  NULL clears
 * the mask; ht_set_observation on the slot clears it too.  `ptr_kind` as for
 * ht_set_observation; the data are copied (stream-ordered on hip_stream).  May allocate (set-up
 * call: not for graph capture).
 * Errors: HT_ERR_ARG for a bad slot or ptr_kind; HT_ERR_STATE for a slot without observation. */
ht_status ht_set_pixel_mask(ht_ctx* ctx, int frame_slot, const uint8_t* mask, int ptr_kind,
                            void* hip_stream);

/* Observation preprocessing (section II.B: the hand is extracted from the RGB-D frame by
 * skin-colour detection and depth segmentation; the paper names no method, this is the
 * library's, in exact integer arithmetic):
 *   skin: Cb = 128 + ((-43 R - 85 G + 128 B + 128) >> 8), Cr = 128 + ((128 R - 107 G - 21 B
 *         + 128) >> 8) (BT.601 chroma, >> = floor division by 256), skin iff cb_lo <= Cb <=
 *         cb_hi and cr_lo <= Cr <= cr_hi;
 *   band: z0 = the smallest defined depth (> 0) among skin pixels; in band iff
 *         z0 <= depth <= z0 + band_mm;
 *   out:  skin_out = skin and in band; depth_out = depth in band, 0 where depth is 0, else
 *         bg_depth_mm (segmented away = background).  No skin pixel with a defined depth:
 *         skin_out = 0 and every defined depth becomes bg_depth_mm.
 * Defaults: cb 77..127, cr 133..173, band 150 mm.  rgb: device uint8 [H][W][3]; depth,
 * depth_out: device uint16 [H][W]; skin_out: device uint8 [H][W]; the outputs may feed
 * ht_set_observation (HT_PTR_DEVICE).  Enqueue only (graph-capturable once the context has
 * run it once at this or a larger size: the first call may allocate a small scratch array).
 * Errors: HT_ERR_ARG for NULL pointers, W or H outside 1..HT_MAX_ROI, a bad box or band. */
typedef struct {
  int32_t cb_lo, cb_hi, cr_lo, cr_hi;
  int32_t band_mm;
  float bg_depth_mm;
} ht_seg_params;

ht_status ht_preprocess_rgbd(ht_ctx* ctx, int W, int H, const uint8_t* rgb,
                             const uint16_t* depth, const ht_seg_params* params,
                             uint16_t* depth_out, uint8_t* skin_out, void* hip_stream);

/* Pre-allocate the workspace for up to `max_particles` particles in total (all frames of one
 * call) over observations of up to `max_pixels` pixels each, so that later calls allocate
 * nothing (required for graph capture).  HT_ERR_OOM on failure. */
ht_status ht_reserve(ht_ctx* ctx, int max_particles, int max_pixels);

/* Optional per-pixel outputs of ht_eval_particles for a single frame (n_frames == 1); each
 * pointer may be NULL.  Device memory, [n_particles][H][W].  Pixels of tiles that no primitive
 * reaches keep the background (r_d = B or 0, no hit, winner -1, margin -inf).  `slot` must repeat, on the host,
 * the observation slot held in frame_slots[0] (it gives W, H and B for the images). */
typedef struct {
  int32_t slot;
  float* depth;      /* r_d                                         */
  uint8_t* hit;      /* model hit (nearest entry in front of B)      */
  uint8_t* rm;       /* r_m of Eq. 4                                 */
  int32_t* winner;   /* index of the nearest primitive, -1 on a miss */
  float* margin;     /* ray-surface margin (dimensionless, > 0 inside the silhouette): of the
                        primitive with the nearest entry; where no primitive is entered, the
                        largest over the primitives tested at the pixel (-inf if none was).
                        Sphere (r^2 - rho^2) / r^2, ellipsoid 1 - rho'^2, closed cylinders and
                        cones the largest of their side's and caps' slacks (radial and axial),
                        in FP32; a pixel within 1e-5 of 0 is decided by rounding. */
} ht_debug;

/* E(h, O) (Eq. 5) for n_frames x n_particles poses.  frame_slots: device int32 [n_frames],
 * the observation slot of each frame.  poses: device float32 [n_frames][n_particles][n_dof];
 * cost: device float32 [n_frames][n_particles].  dbg may be NULL.
 * Errors: HT_ERR_STATE before set_model, HT_ERR_ARG for NULL pointers or counts < 0,
 * HT_ERR_UNSUPPORTED for dbg with n_frames != 1.  n_frames * n_particles == 0 is a no-op.
 * The frame slots are read on the device: every slot used must have been set; a particle of an
 * unset slot scores NaN and raises HT_DEVERR_UNSET_SLOT (ht_device_errors). */
ht_status ht_eval_particles(ht_ctx* ctx, int n_frames, const int32_t* frame_slots,
                            int n_particles, const float* poses, float* cost,
                            const ht_debug* dbg, void* hip_stream);

/* E and dE/dh.  The gradient is that of the clamped depth sum of Eq. 4 over the hit pixels
 * (with sum(o_s or r_m) held fixed; it and the Dice term are piecewise constant) plus
 * lambda_k dkc/dh.  grad: device float32 [n_frames][n_particles][n_dof].  pixel_mask: NULL for
 * the frames' slot masks (ht_set_pixel_mask; every pixel where a slot has none), else device
 * uint8 [H][W] of the frame's slot (n_frames must be 1): pixels with 0 are left out of the
 * gradient (not of the cost).  Errors as ht_eval_particles. */
ht_status ht_eval_particles_grad(ht_ctx* ctx, int n_frames, const int32_t* frame_slots,
                                 int n_particles, const float* poses, float* cost, float* grad,
                                 const uint8_t* pixel_mask, void* hip_stream);

/* ht_eval_particles (forward, no debug images) for callers that cannot allocate device
 * memory: code under HIP graph capture without a prior ht_reserve, tight serving loops,
 * harnesses that forbid allocation.  The call allocates nothing: its workspace (kinematics
 * records, work list, partial sums) is a 64 MiB device array inside the library, one per GPU,
 * held until the process ends.  Every call on a GPU shares that GPU's array, so calls that
 * overlap on one GPU (on different streams, or from different contexts) race: enqueue them on
 * one stream.  Nothing in it must start at zero (the work-list kernel of each call resets its
 * dequeue counter), and it keeps the last call's contents.  Same arguments, layouts and
 * results as ht_eval_particles.  Errors as ht_eval_particles, and HT_ERR_ARG when the call
 * needs more than the 64 MiB (about 1800 two-hand particles over 640x480 observations, 8000
 * one-hand particles over 128x128 ones: the size grows with the particles and the largest
 * set observation). */
ht_status ht_eval_particles_noalloc(ht_ctx* ctx, int n_frames, const int32_t* frame_slots,
                                    int n_particles, const float* poses, float* cost,
                                    void* hip_stream);

/* Swarm state, all device memory owned by the caller, float32 unless noted:
 *   x, v, pbest_x [F][P][n_dof]; pbest_cost, cost [F][P]; gbest_x [F][n_dof];
 *   gbest_cost [F]; gen: int32 [F] generation counters; frame_slots: int32 [F];
 *   init_lo, init_hi [F][n_dof]: box of the initial positions (ht_pso_init); seed: the 64-bit
 *   Philox key (or, with seed_dev, read from device memory);
 *   stop_gen: int32 [F] or NULL, needed for the stop rule (ht_pso_params.stop_cost): 0 while
 *   a frame runs, else the generation count at which its best cost fell below stop_cost;
 *   from then on nothing of that frame's swarm changes (its particles are not evaluated). */
typedef struct {
  int32_t n_frames, n_particles;
  const int32_t* frame_slots;
  float *x, *v, *pbest_x, *pbest_cost, *gbest_x, *gbest_cost, *cost;
  int32_t* gen;
  const float *init_lo, *init_hi;
  uint64_t seed;
  int32_t* stop_gen;
  /* NULL, or a device uint64: the Philox key is read from it by every swarm kernel instead of
   * `seed`, so a captured run (ht_pso_run_graph, cached per swarm struct) replays with new
   * random numbers once the caller writes a new value there (e.g. one per tracked frame). */
  const uint64_t* seed_dev;
} ht_swarm;

/* Swarm constants.  Plain PSO of the paper: c1 = 2.8, c2 = 1.3, w = 2/|2 - psi -
 * sqrt(psi^2 - 4 psi)| (psi = c1 + c2), mutate_every = 3, mutate_frac = 0.5.  refine_topk > 0
 * adds gradient refinement (not in the paper) of the refine_topk lowest-cost particles:
 * refine_steps normalised steepest-descent steps in the eta-scaled space (eta_rot rad for
 * angles, eta_trans mm for translations), halving the step up to 3 times until E drops.
 * stop_cost > 0: the stop rule of section III.B (the paper stops at E < 1.0): after a
 * generation's evaluation, a frame whose best cost is below stop_cost keeps its personal and
 * global bests of that generation and stops (swarm.stop_gen must then be set); 0: never. */
typedef struct {
  float w, c1, c2;
  int32_t mutate_every;
  float mutate_frac;
  int32_t refine_topk, refine_steps;
  float eta_rot, eta_trans;
  float stop_cost;
} ht_pso_params;

/* Initialise: x ~ U[init_lo, init_hi] clamped to the joint limits (Philox4x32-10, stream 1),
 * v = 0, best costs = +inf, gen = 0.  Enqueue-only.  HT_ERR_STATE before set_model. */
ht_status ht_pso_init(ht_ctx* ctx, const ht_swarm* swarm, void* hip_stream);

/* One generation (section III.B): evaluate E at x (into cost), refine the top-K if asked,
 * update personal / global bests, then mutation (every mutate_every-th generation, the worst
 * floor(P * mutate_frac) by current cost re-draw their mutate-mask dimensions) or Eq. 6-7 with
 * clamping to the joint limits.  Random numbers: Philox4x32-10 keyed by the seed with counter
 * (dim, frame * P + particle, generation, stream).  Enqueue-only; generation counters live on
 * the device, so a captured sequence of calls can be replayed.
 * Errors: HT_ERR_STATE before set_model, HT_ERR_ARG for bad pointers / counts / params. */
ht_status ht_pso_step(ht_ctx* ctx, const ht_swarm* swarm, const ht_pso_params* params,
                      void* hip_stream);

/* A whole run: ht_pso_init followed by n_generations x ht_pso_step, captured once into a HIP
 * graph (cached in the context per swarm / params / n_generations, at most 32 graphs: a full
 * cache is emptied before the next capture) and launched on hip_stream.  A new launch shape
 * (ht_set_launch_config, ht_autotune), model or larger workspace drops the cached graphs (the
 * device is synchronised first).  Requires ht_reserve to cover the swarm.  HT_ERR_HIP if
 * capture fails. */
ht_status ht_pso_run_graph(ht_ctx* ctx, const ht_swarm* swarm, const ht_pso_params* params,
                           int n_generations, void* hip_stream);

/* Initial-position box for tracking (section II: a frame's search starts around the previous
 * frame's solution): per frame f and pose parameter d, with c = center clamped to the model
 * bounds, lo = max(c - halfwidth[d], bound_lo[d]) and hi = min(c + halfwidth[d],
 * bound_hi[d]).  center: device float32 [n_frames][n_dof] (e.g. a swarm's gbest_x);
 * halfwidth: device float32 [n_dof] (>= 0); lo, hi: device float32 [n_frames][n_dof] (e.g.
 * the swarm's init_lo / init_hi, then ht_pso_init or ht_pso_run_graph).  Enqueue only;
 * graph-capturable.  Errors: HT_ERR_ARG for NULL pointers or n_frames out of 0..2^22. */
ht_status ht_pso_box_around(ht_ctx* ctx, int n_frames, const float* center,
                            const float* halfwidth, float* lo, float* hi, void* hip_stream);

/* Launch shape of the batched persistent ray-cast kernel.  tiles_per_item is shortened
 * automatically for launches too small to give every compute unit a work item. */
typedef struct {
  int32_t tiles_per_item;   /* 8x8-pixel tiles per work item (one work item per workgroup) */
  int32_t groups_per_cu;    /* persistent workgroups per compute unit                       */
  int32_t cull;             /* 0: primitive screen boxes from their 3D bounding boxes;
                               1: clipped to the image extent of a bounding capsule        */
} ht_launch_config;

ht_status ht_get_launch_config(ht_ctx* ctx, ht_launch_config* out);
ht_status ht_set_launch_config(ht_ctx* ctx, const ht_launch_config* cfg);

/* Autotune the launch shape on the given workload (timed with HIP events on hip_stream,
 * synchronising it), keep the fastest in the context and return it in *out.
 * The candidates are tiles_per_item in {4..64} x groups_per_cu in {1..8} (powers of two) x
 * cull in {0, 1}, tried from cull 1, 64 tiles and 8 workgroups down; a candidate must be more
 * than 1 % faster than the best before it to replace it. */
ht_status ht_autotune(ht_ctx* ctx, int n_frames, const int32_t* frame_slots, int n_particles,
                      const float* poses, float* cost, int repeats, ht_launch_config* out,
                      void* hip_stream);

/* Per-kernel tracing of eager calls: between ht_profile_begin and ht_profile_end every kernel
 * the library enqueues outside graph capture is bracketed by HIP events on its own stream.
 * ht_profile_end synchronises those events, fills stats[HT_K_COUNT] (launch count, particles
 * processed, summed device milliseconds per kernel kind) and stops tracing. */
enum {
  HT_K_FK = 0,            /* kinematics prologue             */
  HT_K_SCHED = 1,         /* work-list scan                  */
  HT_K_RAYCAST = 2,       /* ray cast + cost terms (forward) */
  HT_K_RAYCAST_GRAD = 3,  /* ray cast + cost + adjoint       */
  HT_K_FINALIZE = 4,      /* cost assembly (+ kinematic adjoint) */
  HT_K_PSO = 5,           /* swarm init / update             */
  HT_K_REFINE = 6,        /* refinement select/propose/accept/gather */
  HT_K_COUNT = 7
};
typedef struct {
  int32_t launches;
  int64_t particles;
  double total_ms;
} ht_kernel_stat;

ht_status ht_profile_begin(ht_ctx* ctx);
ht_status ht_profile_end(ht_ctx* ctx, ht_kernel_stat* stats);

/* Particle evaluations the context has performed since it was created or last reset: forward
 * (cost only) and with gradients, counted on the device by every evaluation call, in graph
 * replays too.  Particles that are not evaluated -- of a frame stopped by the stop rule, or the
 * candidates of a refined particle that has stopped refining -- are not counted.  Synchronises
 * the device; reset != 0 sets both counts to zero afterwards.  Errors: HT_ERR_ARG for NULL. */
ht_status ht_eval_counts(ht_ctx* ctx, int64_t* forward, int64_t* gradient, int reset);

/* Errors that the device met in enqueued work since the context was created or last reset, as
 * bit flags (the evaluation calls return before their kernels run; frame slots are device
 * data).  HT_DEVERR_UNSET_SLOT: a particle's frame slot held no observation (or was out of
 * 0..HT_MAX_SLOTS-1); its cost is NaN and its gradient zero.  Synchronises the device; reset != 0
 * clears the flags afterwards.  Errors: HT_ERR_ARG for NULL. */
#define HT_DEVERR_UNSET_SLOT 1u
ht_status ht_device_errors(ht_ctx* ctx, uint32_t* flags, int reset);

#ifdef __cplusplus
}
#endif

#endif /* HANDTRACK_H */
