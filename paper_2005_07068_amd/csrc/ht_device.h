// Internal data layout shared by the host API (ht_api.cpp) and the kernels (ht_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "handtrack.h"

namespace ht {

constexpr int kTile = 8;            // 8x8 pixel tile = one wavefront of 64 lanes
constexpr int kTilePx = kTile * kTile;
constexpr int kWave = 64;
constexpr int kBlock = 256;         // 4 wavefronts per workgroup
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kRec = 20;            // floats per primitive record
constexpr int kNumTypes = 5;        // HT_SPHERE .. HT_ECYLINDER
// Work items of the ray-cast kernel (tiles): never shorter than kMinTilesPerItem (the lower
// bound of the configured tiles_per_item, which sizes the workspace); the work-list kernel
// aims at kFloorTilesFwd / kFloorTilesGrad at least, capped by the configured value.
constexpr int kMinTilesPerItem = 4;
constexpr int kFloorTilesFwd = 8;
constexpr int kFloorTilesGrad = 8;  // 16 left a 32-particle gradient launch at 22.5 us (19.2)
constexpr float kDMatch = 10.0f;    // d_m, mm
constexpr float kDClamp = 40.0f;    // d_M, mm
constexpr double kLambda = 20.0;
constexpr double kLambdaK = 10.0;

// Observation word: bits 0..15 depth (mm, 0 = undefined), bit 16 skin, bit 17 pixel inside
// the ROI (tiles over-hang the ROI on its right and bottom edges).
constexpr uint32_t kSkinBit = 1u << 16;
constexpr uint32_t kValidBit = 1u << 17;

// Hand model as laid out in device memory.
struct DevModel {
  int n_dof, n_seg, n_prim, n_kc;
  int max_depth;
  int n_roots;                           // independent kinematic trees (hands), <= kMaxRects
  int seg_parent[HT_MAX_SEG];
  int seg_root_dof[HT_MAX_SEG];
  int seg_depth[HT_MAX_SEG];
  int seg_dof[HT_MAX_SEG][2];
  double seg_off[HT_MAX_SEG][12];        // row-major 3x4
  double seg_axis[HT_MAX_SEG][2][3];
  int prim_type[HT_MAX_PRIM];
  int prim_seg[HT_MAX_PRIM];
  double prim_frame[HT_MAX_PRIM][12];
  double prim_size[HT_MAX_PRIM][3];
  float lo[HT_MAX_DOF], hi[HT_MAX_DOF];
  int mutate[HT_MAX_DOF];
  int kc_a[HT_MAX_KC], kc_b[HT_MAX_KC];
  uint32_t dof_desc[HT_MAX_DOF];         // segments moved by each pose parameter
  int dof_trans[HT_MAX_DOF];             // 1 for the wrist translations (mm), else angle
  int prim_root[HT_MAX_PRIM];            // tree of each primitive
  int prim_order[HT_MAX_PRIM];           // primitive indices sorted by type
  double prim_inv2[HT_MAX_PRIM][3];      // 1 / size^2 (ellipsoid semi-axes)
};

constexpr int kMaxRects = 4;             // tile rectangles per particle (one per tree)

// Primitive index masks per type (bits for primitives 0..63 and 64..127).
struct TypeMasks {
  uint64_t m[kNumTypes][2];
};

// One observation slot.
struct FrameSlot {
  int W, H, TW, TH;          // ROI size and tile grid
  float sx, sy, sz;          // ray d = ((u-cx)*sx, (v-cy)*sy, sz); depth = t * sz
  float cx, cy, fx, fy;
  float bg;                  // background plane depth B (<= 0: none)
  int set;
  const uint32_t* words;     // [TH*TW][64] tile-major observation words
  const float* tile_td;      // [TH*TW] sum of min(|o_d - r_bg|, d_M) over the tile
  const int* tile_skin;      // [TH*TW] skin pixels of the tile
  const double* totals;      // [2]: the same two sums over the whole ROI
  const uint8_t* grad_mask;  // [H][W] gradient pixel mask of the slot, NULL: every pixel
};

// Per-particle summary written by the kinematics kernel.  The tiles to visit are the union of
// up to kMaxRects disjoint rectangles (one per kinematic tree, overlapping ones merged), each
// covering its primitives' screen boxes; tile t of the particle is found by walking them.
struct PInfo {
  int4 rect[kMaxRects];       // tx0, ty0, tw, th (tiles)
  int n_rects;
  int n_tiles;                // sum of the rectangles' tiles
  int slot;                   // observation slot (-1: unset slot)
  float kc;                   // collision term of Eq. 5
  int valid;                  // 0: non-finite pose or unset slot
  int skip;                   // 1: not evaluated (its frame has stopped, or it is a candidate
                              // of a refined particle that has stopped): nothing is written
  int kc_mask;                // collision pairs with a positive term (bit i: pair i)
  double bg_td, bg_or;        // the observation's ROI-wide background sums (copied from its
                              // slot, so the finalize kernels need no slot lookup)
};

struct Partial {
  double td;  // clamped depth sum minus the background sum of the processed tiles
  int a;      // sum(o_s and r_m)
  int o;      // sum(o_s or r_m) minus the background skin count of the processed tiles
  int pad;
};

// Workspace of one evaluation call (device pointers, owned by the context).
struct Workspace {
  float* recs;           // [n_total][n_prim][kRec]
  int4* boxes;           // [n_total][n_prim] pixel box (u0, u1, v0, v1), empty = (1, 0, 1, 0)
  float4* caps;          // [n_total][n_prim] image segment (x0, y0, dx, dy) of the bounding
                         // capsule: the centres of its end spheres' image discs (pixels)
  float2* capr;          // [n_total][n_prim] (1 / |(dx, dy)|^2 or 0, reach^2): a tile whose
                         // centre lies farther than reach from the segment sees none of it
  PInfo* pinfo;          // [n_total]
  float* dof_frame;      // [n_total][n_dof][8]: kind, axis xyz, point xyz (camera frame)
  float* seg_org;        // [n_total][n_seg][4]
  int* tiles;            // [n_total] tiles of each particle (a compact copy for the
                         // scheduler), -1 for a particle that is not evaluated (skipped)
  int* item_off;         // [n_total + 1]
  int* item_map;         // [max_items]
  Partial* partial;      // [max_items]
  float* wrench;         // [max_items][n_seg][6] (gradient only)
  int* counters;         // [0] dequeue counter, [1] total items, [2] tiles per item,
                         // [3] 1: a particle's items take interleaved tiles
  int max_items;
};

struct EvalArgs {
  const DevModel* model;
  const FrameSlot* slots;
  const int* frame_slots;
  int n_frames, n_particles;
  const float* poses;
  float* cost;
  float* grad;                 // NULL for forward only
  const uint8_t* pixel_mask;   // gradient mask of frame 0, may be NULL
  const int* frame_stop;       // [n_frames] stop flags of a swarm, may be NULL
  // NULL, or per group of active_div consecutive particles a flag: 0 = the group is not
  // evaluated (the candidates of a refined particle that has stopped refining)
  const int* active;
  int active_div;
  // evaluations performed (not skipped), [0] forward and [1] gradient, added up by the
  // work-list kernel of every call; may be NULL
  unsigned long long* eval_count;
  unsigned int* dev_errors;    // HT_DEVERR_* flags raised on the device, may be NULL
  // NULL, or per evaluated particle r its source s = src[r]: the particle reuses the kinematics
  // of workspace particle (r / n_particles) * src_stride + s from the previous evaluation
  // (same poses; the kinematics stage is skipped)
  const int* src;
  int src_stride;
  ht_debug dbg;                // pointers may be NULL
  int dbg_W, dbg_H;
  float dbg_bg;
  TypeMasks type_masks;
  int tiles_per_item;
  int cull;                    // 1: screen boxes clipped to the bounding capsule's image extent
  int grid;                    // persistent workgroups
  int self_sched;              // 1: the ray cast builds the work list (at most kSelfSchedMax
                               // particles, no debug images)
  int n_prim, n_seg, n_dof;
};

// Launch helpers implemented in ht_kernels.hip.
hipError_t launch_pack_observation(const uint16_t* depth, const uint8_t* skin, int W, int H,
                                   int TW, int TH, uint32_t* words, float* tile_td,
                                   int* tile_skin, double* totals, float bg, hipStream_t s);
enum { kStageFk = 0, kStageSched = 1, kStageRaycast = 2, kStageFinalize = 3, kNumStages = 4 };
constexpr int kSelfSchedMax = 256;   // launches of at most this many particles self-schedule
// persistent workgroups per CU of a self-scheduled launch, at most: on the two-hand 640x480
// workload the 128-particle forward launch took 31.5, 27.9, 26.9, 30.5 and 30.7 us at 4..8
constexpr int kSelfGroupsPerCu = 6;
hipError_t launch_eval_stage(int stage, const EvalArgs& a, const Workspace& ws, hipStream_t s);
int raycast_groups_per_cu(bool grad, bool dbg, bool all_types, bool self_sched);
hipError_t launch_pso_init(const DevModel* model, const ht_swarm& sw, int n_dof, hipStream_t s);
int preprocess_partials(int W, int H);
hipError_t launch_preprocess(int W, int H, const uint8_t* rgb, const uint16_t* depth,
                             const ht_seg_params& p, int* partial, uint16_t* depth_out,
                             uint8_t* skin_out, hipStream_t s);
hipError_t launch_box_around(const DevModel* model, int n_frames, int n_dof, const float* center,
                             const float* halfwidth, float* lo, float* hi, hipStream_t s);
hipError_t launch_pso_update(const DevModel* model, const ht_swarm& sw, const ht_pso_params& p,
                             int n_dof, int* flags, hipStream_t s);
hipError_t launch_refine_select(const ht_swarm& sw, int K, int n_dof, int* sel, float* rx,
                                float* rcost, int* active, hipStream_t s);
// One refinement update (ht_kernels.hip), fused with the assembly of the evaluation before
// it (whose arguments and workspace it reads): the gradient evaluation of the selected
// particles (propose only) or the evaluation of their candidates, four per particle.
struct RefineOp {
  int accept, propose, gather;
};
struct RefineArgs {
  int n_ref, K, n_dof;
  float eta_rot, eta_trans;
  RefineOp op;
  int eval_grad;             // the preceding evaluation computed gradients
  ht_swarm sw;
  const int* sel;            // [n_ref] swarm index of each refined particle
  float* rx;                 // [n_ref][n_dof] positions
  float* rcost;              // [n_ref] costs
  int* active;               // [n_ref] 1 while refining
  float* cand;               // [4 n_ref][n_dof] candidates
  float* grad;               // [n_ref][n_dof] gradients at rx
};
hipError_t launch_refine_update(const EvalArgs& a, const Workspace& ws, const RefineArgs& ra,
                                hipStream_t s);

}  // namespace ht
