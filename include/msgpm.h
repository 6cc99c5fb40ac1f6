/*
 * msgpm.h - C ABI of the MI355X (gfx950) library for the data-parallel hot
 * path of multi-scale generalized plane match (MSGPM): Choi & Banerjee,
 * "Multi-Scale Generalized Plane Match for Optical Flow", arXiv 1804.03787.
 *
 * Problem statement (Sec. 3, Alg. 1): two frames in, optional initial nearest-
 * neighbour field (NNF), patch size, list of plane-fit window sizes (one per
 * level) and iteration counts; dense flow, per-window homographies and an
 * occlusion mask out, for both directions (frame 1 -> 2 and frame 2 -> 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers named d_* are device pointers (HIP global memory of the current
 *    device); everything else is host memory.  The caller owns every buffer,
 *    including the workspace; the library allocates no device memory.
 *  - Work is enqueued on `stream` (a hipStream_t, NULL = default stream) and the
 *    call returns once it is enqueued.  Calls on one workspace must be ordered
 *    on one stream.
 *  - Pixel (x, y) has index y*width + x; y points down; pixel centres are on
 *    integer coordinates.  A flow or NNF offset is target - source.
 *  - NNF offsets are packed int32: (dx & 0xffff) | (dy << 16), both int16.
 *  - Direction 0 matches frame 1 against frame 2, direction 1 frame 2 against
 *    frame 1; every phase entry point processes both directions.
 *  - Homographies are row-major 3x3 doubles mapping a source-frame pixel to the
 *    target frame (Eq. 1), normalised so that H[8] = 1.
 *  - Errors are returned as msgpm_status; nothing is thrown across the ABI.
 *    msgpm_last_error() returns a message for the calling thread's last error.
 *    On an error nothing is enqueued.
 */
#ifndef MSGPM_H
#define MSGPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MSGPM_MAX_LEVELS 8

typedef enum msgpm_status {
  MSGPM_OK = 0,
  MSGPM_E_INVALID = 1,     /* bad argument: sizes, parameters, null pointer, unknown ticket */
  MSGPM_E_OOM = 2,         /* memory: a request that can never fit a server's budget, or an
                              allocation the library makes (pinned staging, events) failed */
  MSGPM_E_DEVICE = 3,      /* the HIP runtime reported an error (also: no device) */
  MSGPM_E_UNSUPPORTED = 4, /* valid but not built (e.g. patch radius > 4) */
  MSGPM_E_BUSY = 5,        /* transient refusal: a server's queue is full; retry later */
  MSGPM_E_CANCELLED = 6,   /* the pair was cancelled (msgpm_server_wait) */
  MSGPM_E_TIMEOUT = 7      /* the pair was not done within the timeout (msgpm_server_wait) */
} msgpm_status;

/* Storage flag: features stored as binary16 (FP16) with FP32 accumulation. */
#define MSGPM_FLAG_FP16 1u
/* Optional occlusion cues of Sec. 3.4 beyond the forward-backward plane
   symmetry (off by default):
   cue 3, MSGPM_FLAG_CUE_OVERLAP: a plane is kept only if more than eta of its
     colour-consistent pixels are also inliers of its own RANSAC test
     (msgpm_plane.rin / rk);
   cue 2, MSGPM_FLAG_CUE_UNIQUE: at the end of each level, after the
     forward-backward check, of the assigned pixels whose plane sends them
     (rounded to the grid) to the same in-frame target only the one with the
     smallest loss keeps its plane (ties: smallest pixel index). */
#define MSGPM_FLAG_CUE_OVERLAP 2u
#define MSGPM_FLAG_CUE_UNIQUE 4u
/* Input flag: histogram-equalise each frame's HSV value channel before the
   features (the illumination experiment of Sec. 4.2).  V = max(R, G, B) is
   binned to the nearest of 256 levels, floor(255 V + 1/2) clamped to 0..255;
   level q maps to V' = (cdf(q) - cdf_min) / (n - cdf_min), where cdf_min is the
   count of the lowest occupied level (computed in FP64, rounded to FP32).
   R, G, B are scaled by V'/V (V <= 0: grey V'); a frame whose pixels all share
   one level is used as it is.  The frames themselves are not modified. */
#define MSGPM_FLAG_HISTEQ 8u
/* Merge flag: the level priority of Sec. 3.3 (when the levels' flows are
   merged, earlier levels, whose windows are larger and so less disturbed by
   noisy matches, come first) taken strictly.  A pixel assigned at some level
   keeps that plane: the assignment of every later level (both stages) is
   offered only the pixels that are unassigned when it runs, as stage 2 always
   is (Sec. 3.2).  RANSAC, the plane-symmetry counts and the forward-backward
   checks are unchanged (the end-of-level check can still unassign a pixel,
   which a later level may then assign).  Without the flag every stage-1
   assignment is offered every pixel, and a finer level's plane replaces the
   incumbent when its loss is strictly smaller, the level breaking exact ties
   in favour of the coarser one (key (L, level, stage, window)). */
#define MSGPM_FLAG_MERGE_STRICT 16u
/* Execution option, not part of the method: the two launches of each
   restricted half-sweep (pixels with a region plane, pixels without) are
   issued one after the other on the caller's stream instead of side by side
   on the caller's stream and a second stream of the library's.  Results are
   the same either way (the two launches update disjoint pixels and read only
   the other colour); with the flag the library creates no second stream, and
   the per-kind kernel times of msgpm_timing_read are each kernel's own,
   without the other's interference.  msgpm_solve_static always runs this
   way.  Ignored by the batched and served forms, which take every pair's
   restricted half-sweep in shared launches of their own. */
#define MSGPM_FLAG_ONE_STREAM 32u

/* Method parameters.  Defaults in brackets are those of the 1024x436 workload. */
typedef struct msgpm_params {
  int32_t width, height;     /* frame size, 2..32767 each */
  int32_t channels;          /* 3 = RGB, 5 = RGB + luma gradients gx, gy [5] */
  int32_t patch_radius;      /* r: square patch of (2r+1)^2 taps, 1..4 [4] (Sec. 4 uses 7x7) */
  int32_t n_levels;          /* number of plane-fit levels, 0..8 [3] (Sec. 3.3) */
  int32_t block[MSGPM_MAX_LEVELS]; /* window side per level, largest first, 4..128 [64, 32, 16];
                                      windows overlap by half (Sec. 3.1.2) */
  int32_t pm_iters;          /* PatchMatch iterations per pass [8] */
  int32_t ransac_hyps;       /* RANSAC hypotheses per window, 1..1024 [256] (Sec. 3.1.2) */
  int32_t search_radius0;    /* first random-search radius; 0 = max(width, height) */
  int32_t min_support_abs;   /* detection needs max(this, ceil(frac * window area)) inliers [8] */
  int32_t eta_num, eta_den;  /* plane-symmetry ratio eta = num/den [1/2] (Alg. 1, Sec. 3.4) */
  uint32_t flags;            /* MSGPM_FLAG_* */
  int32_t fill_sweeps;       /* filling by homography-model propagation (Sec. 3.4.1) after the
                                last level: red-black half-sweeps over the unassigned pixels,
                                0..65536, 0 = no filling [0]; see msgpm_fill */
  int32_t reserved;          /* set to 0 */
  double grad_weight;        /* weight of gx, gy in the patch cost [1] */
  double inlier_px;          /* RANSAC reprojection threshold tau in pixels [1] */
  double eps_color;          /* colour-consistency threshold epsilon, RMS over RGB [0.1] (Eq. 4) */
  double fb_px;              /* forward-backward point threshold in pixels [1] */
  double min_support_frac;   /* see min_support_abs [0.25] */
  uint64_t seed;             /* key of the counter-based random stream */
} msgpm_params;

/* Per-window plane record, 144 bytes.  One record per (direction, level,
   stage, window); the record index is
     dir * n_planes/2 + 2 * (windows of the levels before) + (stage-1) * windows(level) + window
   with windows numbered row-major over their origins. */
typedef struct msgpm_plane {
  double H[9];               /* fitted homography (source -> target), H[8] = 1 when fitted */
  int32_t dir, level, stage, block;
  int32_t x0, y0, bw, bh;    /* window rectangle */
  int32_t support;           /* points handed to RANSAC (stage 2: the window's unassigned pixels) */
  int32_t count;             /* inliers of H */
  int32_t hyp, hyp_count;    /* winning hypothesis and its inliers (-1, 0 if none) */
  int32_t refit;             /* 1 if the least-squares refit replaced the hypothesis */
  int32_t detected;          /* count >= minimum support */
  int32_t rk, pass;          /* colour-consistent pixels and those passing forward-backward */
  int32_t valid;             /* detected and kept by the plane-symmetry test (and cue 3 if enabled) */
  int32_t rin;               /* colour-consistent pixels that are also RANSAC inliers of H */
} msgpm_plane;

/* Byte offsets of every array inside the caller-allocated workspace (one per
   frame pair), each 256-byte aligned.  Per-pixel arrays hold width*height
   elements; [d] indexes the direction. */
typedef struct msgpm_layout {
  uint64_t total_bytes;
  uint64_t feat[2];        /* features of frame 1 and frame 2, see below */
  uint64_t feat_bytes;     /* bytes of one frame's features */
  uint64_t nnf[2];         /* int32 packed offsets */
  uint64_t cost[2];        /* float: warped-patch SSD of the current offset */
  uint64_t win[2];         /* int32: assigned plane index, -1 = unassigned,
                              -2 - k = filled with plane k (after msgpm_fill) */
  uint64_t loss[2];        /* double: colour-consistency loss of the assignment */
  uint64_t hlabel[2];      /* int32: region plane used for the patch distortion, -1 = identity */
  uint64_t twin[2];        /* int32: tentative assignment (scratch) */
  uint64_t tloss[2];       /* double: its loss (scratch) */
  uint64_t planes;         /* msgpm_plane[n_planes] */
  uint64_t counters;       /* uint64[16][64]: evaluation counters, see below */
  uint64_t histeq;         /* equalisation: uint32 histograms [2][256], FP32 maps [2][256],
                              int32 single-level flags [2] */
  uint64_t active;         /* scratch of restricted passes: per direction and colour an int32
                              buffer of ceil(width/2)*height entries (256-byte aligned) listing
                              the pixels to update, those with a region plane from the front,
                              the others from the back; then 8 uint32 list lengths, then
                              2 x 4 uint32 counters of the filling half-sweeps */
  int32_t n_planes;
  int32_t n_levels;
  int32_t level_blocks[MSGPM_MAX_LEVELS]; /* windows per level and stage */
  int32_t level_nbx[MSGPM_MAX_LEVELS];    /* windows per row */
} msgpm_layout;
/* Feature storage of one frame: width*height + 1 pixel records, interleaved,
   the last one zero.  FP32: `channels` floats (R, G, B[, gx, gy]).  FP16:
   4 halves (R, G, B, 0) for 3 channels, 6 halves (R, G, B, gx, gy, 0) for 5. */

/* Fills *out for the given parameters; validates them.  No device work. */
msgpm_status msgpm_layout_query(const msgpm_params* p, msgpm_layout* out);

/* Text of the calling thread's last error ("" if none).  Owned by the library. */
const char* msgpm_last_error(void);

/* ---------------------------------------------------------------------------
 * Whole pipeline (Alg. 1 for every level, Sec. 3.4 forward-backward check at
 * the end of each level, Sec. 4 set-up): features, initial NNF (random unless
 * given), PatchMatch init pass, then per level two plane stages (Sec. 3.1,
 * 3.2), FB, NNF update (Sec. 3.3.1) and a PatchMatch pass restricted to the
 * unassigned pixels (Sec. 3.3.2); then, if fill_sweeps > 0, filling by
 * model propagation (Sec. 3.4.1).
 *   d_rgb1, d_rgb2: frames, height x width x 3 float32 (HWC).
 *   d_init_nnf0/1:  optional initial NNF per direction (packed, may be NULL).
 *   d_ws:           workspace of layout.total_bytes, 256-byte aligned.
 *   d_flow0/1:      height x width x 2 float32: plane flow where a plane is
 *                   assigned or filled, else the NNF offset.
 *   d_occ0/1:       height x width uint8: 0 = plane assigned, 1 = no plane
 *                   (occluded, Sec. 3.4), 2 = filled by model propagation
 *                   (no plane of its own: occluded by the same rule, with a
 *                   neighbour's plane flow).
 * The plane table stays in the workspace (layout.planes).  Work is enqueued
 * on `stream` and the call returns; the identity-patch half of each restricted
 * half-sweep runs on a second stream of the calling thread (created on first
 * use, default priority), forked from and joined back into `stream` by events.
 * ------------------------------------------------------------------------- */
msgpm_status msgpm_solve(const msgpm_params* p, const float* d_rgb1, const float* d_rgb2,
                         const int32_t* d_init_nnf0, const int32_t* d_init_nnf1, void* d_ws,
                         float* d_flow0, float* d_flow1, uint8_t* d_occ0, uint8_t* d_occ1, void* stream);

/* ---------------------------------------------------------------------------
 * Phase entry points.  Each runs one step of the pipeline on the state held in
 * the workspace, for both directions, exactly as msgpm_solve does; together
 * they let a caller run, inspect or replace the state between steps.
 * ------------------------------------------------------------------------- */

/* Features of both frames (pixel colours plus optional luma gradients gx, gy
   with replicate borders; the paper's cost is colour only, Sec. 3.1.3), of
   the equalised frames with MSGPM_FLAG_HISTEQ. */
msgpm_status msgpm_features(const msgpm_params* p, const float* d_rgb1, const float* d_rgb2, void* d_ws,
                            void* stream);

/* Initial state: NNF from d_init_nnf0/1 (targets clamped into the frame) or, if
   NULL, a uniformly random target per pixel from the counter-based stream;
   every pixel unassigned with the identity region plane; plane table reset;
   evaluation counters zeroed. */
msgpm_status msgpm_init_state(const msgpm_params* p, const int32_t* d_init_nnf0, const int32_t* d_init_nnf1,
                              void* d_ws, void* stream);

/* Recomputes the warped-patch cost of the current offset.  mode 0: every pixel
   under the identity; mode 1: unassigned pixels under their region plane (the
   identity where they have none), over the restricted pass's pixel lists, which
   this call builds; mode 2: assigned pixels under their assigned plane. */
msgpm_status msgpm_eval_cost(const msgpm_params* p, void* d_ws, int mode, void* stream);

/* One red-black half-sweep of PatchMatch (propagation from the four
   neighbours, then random search; Barnes et al. as used in Sec. 3.1) over the
   pixels with (x + y) % 2 == colour.  restricted = 0: every pixel, identity
   patch; restricted = 1: unassigned pixels only, patches distorted by the region
   plane, plus the candidate that plane predicts (Sec. 3.3.2); this call builds
   the pixel lists, and its two launches (pixels with and without a region
   plane) run side by side on the caller's stream and a second stream of the
   calling thread, joined back into the caller's stream before it returns.
   iter and slot (0 = initial pass, level + 1 = pass after that level) key the
   random stream.  restricted may carry MSGPM_PM_FRESH: each swept pixel's
   current cost is then computed first, exactly as msgpm_eval_cost (mode 0
   for restricted = 0, mode 1 for restricted = 1) would compute it, instead of
   being read from the workspace; the result equals that refresh followed by
   the plain half-sweep, over this colour's pixels.  msgpm_solve uses it for
   the first half-sweep of each colour in every pass.  Any other value of
   restricted is MSGPM_E_INVALID. */
#define MSGPM_PM_FRESH 2
msgpm_status msgpm_pm_halfsweep(const msgpm_params* p, void* d_ws, int colour, int iter, int slot, int restricted,
                                void* stream);

/* RANSAC plane fit in every window of `level` (Sec. 3.1.2; stage 2 = residual
   region, Sec. 3.2): writes the (level, stage) plane records. */
msgpm_status msgpm_ransac(const msgpm_params* p, void* d_ws, int level, int stage, void* stream);

/* Colour-consistency assignment (Eq. 3-4, overlap rule of Sec. 3.1.3 and the
   level priority of Sec. 3.3).  tentative = 1 uses the detected planes and
   writes twin/tloss; tentative = 0 uses the valid planes and updates win/loss. */
msgpm_status msgpm_assign(const msgpm_params* p, void* d_ws, int level, int stage, int tentative, void* stream);

/* Plane-symmetry test (Alg. 1, Sec. 3.4 first cue) of every detected plane of
   (level, stage) against the other direction's tentative assignment.  Also
   counts rin (colour-consistent pixels whose NNF match is a RANSAC inlier of the
   plane); with MSGPM_FLAG_CUE_OVERLAP a valid plane further needs
   rin / rk > eta (third cue). */
msgpm_status msgpm_symmetry(const msgpm_params* p, void* d_ws, int level, int stage, void* stream);

/* End-of-level forward-backward check (Sec. 4): assigned pixels failing it
   become unassigned, both directions judged on the same snapshot. */
msgpm_status msgpm_fb_unassign(const msgpm_params* p, void* d_ws, void* stream);

/* Occlusion cue 2, many-to-one matches (Sec. 3.4, second cue): of the assigned
   pixels whose plane maps them to the same in-frame pixel (the mapped position
   rounded half up), only the one with the smallest colour loss keeps its plane,
   ties to the smallest pixel index; the others become unassigned.  Both
   directions.  Overwrites the tentative assignment (twin/tloss) as scratch.
   Runs whatever the flags say; msgpm_solve calls it after msgpm_fb_unassign
   when MSGPM_FLAG_CUE_UNIQUE is set. */
msgpm_status msgpm_unique(const msgpm_params* p, void* d_ws, void* stream);

/* Filling by homography-model propagation (Sec. 3.4.1), both directions:
   fill_sweeps red-black half-sweeps (half-sweep t updates the pixels with
   (x + y) % 2 == t % 2).  An unassigned pixel takes, of the planes of its four
   neighbours (assigned or already filled), the one with the smallest colour
   error (ties: the smallest plane index) if that error is below eps_color^2;
   it is then filled: win = -2 - plane, loss = that error.  Half-sweeps after
   two in a row that filled nothing exit at once (nothing can change).
   msgpm_solve calls it after the last level when fill_sweeps > 0; filled
   pixels get their plane's flow and mask value 2. */
msgpm_status msgpm_fill(const msgpm_params* p, void* d_ws, void* stream);

/* NNF update from the assigned planes (Sec. 3.3.1) and region plane choice for
   the next restricted pass. */
msgpm_status msgpm_nnf_update(const msgpm_params* p, void* d_ws, int level, void* stream);

/* Outputs: refreshes the cost of assigned pixels, writes flow and occlusion
   mask of both directions (see msgpm_solve). */
msgpm_status msgpm_finalize(const msgpm_params* p, void* d_ws, float* d_flow0, float* d_flow1, uint8_t* d_occ0,
                            uint8_t* d_occ1, void* stream);

/* msgpm_solve through a HIP graph: the first call with a given parameter set
 * and set of buffer addresses captures the whole launch sequence (on a stream
 * of the library's) into a graph; every call launches that graph on `stream`,
 * so the pipeline's ~200 launches cost one.  Results are identical to
 * msgpm_solve.  Up to 16 graphs are kept (oldest dropped); kernel timing does
 * not see graph launches.  msgpm_graph_cache_clear drops them all (call it
 * before freeing buffers a cached graph refers to, if the addresses may be
 * reused with other contents and the same parameters). */
msgpm_status msgpm_solve_graph(const msgpm_params* p, const float* d_rgb1, const float* d_rgb2,
                               const int32_t* d_init_nnf0, const int32_t* d_init_nnf1, void* d_ws,
                               float* d_flow0, float* d_flow1, uint8_t* d_occ0, uint8_t* d_occ1, void* stream);
msgpm_status msgpm_graph_cache_clear(void);

/* msgpm_solve without any allocation, for callers that cannot allocate device
 * memory or create HIP objects (code under stream capture, tight serving
 * loops, harnesses that forbid it).  The workspace is not an argument: it is
 * a static array of MSGPM_STATIC_WS_BYTES inside the library's device code,
 * one per GPU, held from the library's first use on that GPU until the
 * process ends (64 MiB: enough for 1024x436 frames with 5 FP32 channels,
 * whose workspace is 58.8 MB).  Parameters whose msgpm_layout_query
 * total_bytes exceeds it are rejected with MSGPM_E_INVALID and nothing is
 * enqueued.  Frames, initial NNF and outputs are as for msgpm_solve; d_planes
 * (may be NULL) receives the plane table, layout.n_planes records, by a
 * device-to-device copy.  Everything runs on `stream`, in order (the two
 * launches of a restricted half-sweep one after the other, with the results
 * of msgpm_solve bit for bit); no stream, event, graph or memory is created
 * and kernel timing does not see these launches.  All calls on one GPU share
 * its array, and the array keeps the last call's state: calls that overlap on
 * one GPU (two streams, two threads) race and corrupt each other, so callers
 * must order them. */
#define MSGPM_STATIC_WS_BYTES (64ull << 20)
msgpm_status msgpm_solve_static(const msgpm_params* p, const float* d_rgb1, const float* d_rgb2,
                                const int32_t* d_init_nnf0, const int32_t* d_init_nnf1, float* d_flow0,
                                float* d_flow1, uint8_t* d_occ0, uint8_t* d_occ1, msgpm_plane* d_planes,
                                void* stream);

/* ---------------------------------------------------------------------------
 * Batched solves: the pipeline of msgpm_solve for n frame pairs at once, one
 * launch per phase covering every pair (pairs of different sizes share the
 * launches; small pairs then fill the GPU together).  Each pair has its own
 * parameters, workspace (layout from msgpm_layout_query on its parameters),
 * frames, optional initial NNF and outputs, exactly as for msgpm_solve, and its
 * results are identical to a msgpm_solve of that pair alone.  All pairs must
 * share patch_radius, channels, the FP16 flag, pm_iters and n_levels.
 *   params:          n parameter sets (host array).
 *   d_rgb1 .. d_occ1: host arrays of n device pointers each; d_init_nnf0/1 may
 *                    be NULL (random initial NNF for every pair) or hold NULL
 *                    entries.
 *   d_scratch:       device buffer of the size msgpm_batch_query returns,
 *                    256-byte aligned, for the launch tables; it must stay
 *                    untouched until the work enqueued here has run.
 * The launch tables are copied to d_scratch through a pinned host buffer that
 * the library keeps (and reuses once the previous upload has completed).
 * Work is enqueued on `stream`; errors as for msgpm_solve.
 * ------------------------------------------------------------------------- */
msgpm_status msgpm_batch_query(int n, const msgpm_params* params, uint64_t* scratch_bytes);
msgpm_status msgpm_solve_batch(int n, const msgpm_params* params, const float* const* d_rgb1,
                               const float* const* d_rgb2, const int32_t* const* d_init_nnf0,
                               const int32_t* const* d_init_nnf1, void* const* d_ws, float* const* d_flow0,
                               float* const* d_flow1, uint8_t* const* d_occ0, uint8_t* const* d_occ1,
                               void* d_scratch, void* stream);
/* msgpm_solve_batch as one HIP graph launch.  Every pair-dependent value
   (descriptors, item lists, launch sizes) is in the table in d_scratch, which
   is uploaded on each call, and every batched kernel is persistent (a fixed
   grid per kernel class, see msgpm_tuning), so the graph depends only on the
   sequence of phases (the shared parameters), the kernel instantiation, the
   tuning and d_scratch's address (and, for classes tuned one-shot, the
   pairs' work-item counts): one graph, captured on first use, serves every
   later batch with that schedule.  Results are
   identical to msgpm_solve_batch; kernel timing does not see graph launches.
   msgpm_graph_cache_clear drops these graphs too. */
msgpm_status msgpm_solve_batch_graph(int n, const msgpm_params* params, const float* const* d_rgb1,
                                     const float* const* d_rgb2, const int32_t* const* d_init_nnf0,
                                     const int32_t* const* d_init_nnf1, void* const* d_ws, float* const* d_flow0,
                                     float* const* d_flow1, uint8_t* const* d_occ0, uint8_t* const* d_occ1,
                                     void* d_scratch, void* stream);

/* Launch shape of the batched and served forms.  Their kernels can run
   persistent: a launch then runs wg_per_cu[class] x (compute units) resident
   workgroups of 256 threads, which take the launch's work items (tiles of a
   pair's pixels, windows of a level) in turn; 0 gives one workgroup per work
   item instead (for the PatchMatch classes a separate form of the kernel
   without the loop).  Classes: identity-patch PatchMatch (and its cost
   refresh), distorted-patch PatchMatch, RANSAC, every other per-pixel kernel.
   Values 0..64; defaults {0, 0, 0, 16}.  Results do not depend on them
   (every work item is computed the same way wherever it runs).  With every
   class persistent a batched graph depends only on the schedule (see
   msgpm_solve_batch_graph); a one-shot class makes it depend on the pairs'
   work-item counts as well.  A setting applies to one kernel instantiation (patch radius,
   channel count, storage) or, with 0 / 0 / -1 there, to all that have none
   of their own; paper_1804_03787_amd/autotune.py measures them per
   instantiation and the Python binding installs its stored choices.
   Process-wide; graphs already captured keep the shape they were captured
   with. */
enum { MSGPM_TUNE_PM_IDENTITY = 0, MSGPM_TUNE_PM_DISTORTED = 1, MSGPM_TUNE_RANSAC = 2, MSGPM_TUNE_PIXEL = 3,
       MSGPM_TUNE_CLASSES = 4 };
typedef struct msgpm_tuning {
  int32_t patch_radius;  /* 1..4, or 0: any */
  int32_t channels;      /* 3 or 5, or 0: any */
  int32_t fp16;          /* 0 or 1, or -1: either storage */
  int32_t wg_per_cu[MSGPM_TUNE_CLASSES];
} msgpm_tuning;
/* Stores t's shape for its instantiation (replacing an earlier one). */
msgpm_status msgpm_tuning_set(const msgpm_tuning* t);
/* Fills t->wg_per_cu with the shape that applies to t's instantiation. */
msgpm_status msgpm_tuning_get(msgpm_tuning* t);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of pairs that arrive at different times.  A
 * server queues submitted pairs and admits them, first come first served,
 * while the sum of the admitted pairs' workspace bytes stays within
 * hbm_budget and at most max_active are in flight.  Each msgpm_server_step
 * first retires the cohorts whose work has completed, then admits the queued
 * pairs that fit (those sharing the oldest pair's schedule, as a batch must)
 * as one cohort and enqueues the cohort's whole pipeline: its table is
 * uploaded and the batched pipeline of msgpm_solve_batch_graph runs as one
 * graph launch (one graph per schedule and region, captured once), on one of
 * the server's own streams, ordered after the work already on `stream`.  Up to
 * four cohorts (msgpm_server_set_cohorts) run on the device side by side, so
 * pairs that arrive while others are on the GPU start at once and share it
 * with them.  A pair's
 * results (as msgpm_solve, and identical to them) are complete once
 * msgpm_server_poll reports it done or msgpm_server_wait returns; its ticket
 * is then retired.  All pairs of a server share patch_radius, channels and the
 * FP16 flag; a pipeline of more than 4096 launches (very long fillings or
 * iteration counts) is not served (MSGPM_E_UNSUPPORTED).  Buffers are
 * caller-owned and must stay valid until the pair is done; d_scratch
 * (msgpm_server_scratch_bytes for max_active, 256-byte aligned) holds the
 * cohorts' tables, in four regions.  One host thread at a time per server
 * (calls are serialised by a lock).
 * ------------------------------------------------------------------------- */
typedef struct msgpm_server msgpm_server;
msgpm_status msgpm_server_create(uint64_t hbm_budget, int max_active, msgpm_server** out);
msgpm_status msgpm_server_destroy(msgpm_server* server);
msgpm_status msgpm_server_scratch_bytes(int max_active, uint64_t* bytes);
/* Queues a pair.  MSGPM_E_OOM: its workspace (layout.total_bytes) exceeds
   hbm_budget, so it could never be admitted.  MSGPM_E_BUSY: the queue already
   holds the limit set by msgpm_server_set_queue_limit (a transient refusal:
   submit again once pairs have been admitted).  Nothing is queued on an error. */
msgpm_status msgpm_server_submit(msgpm_server* server, const msgpm_params* p, const float* d_rgb1,
                                 const float* d_rgb2, const int32_t* d_init_nnf0, const int32_t* d_init_nnf1,
                                 void* d_ws, float* d_flow0, float* d_flow1, uint8_t* d_occ0, uint8_t* d_occ1,
                                 uint64_t* ticket);
/* Largest number of pairs waiting for admission (0 = no limit, the default). */
msgpm_status msgpm_server_set_queue_limit(msgpm_server* server, int max_queued);
/* Largest number of cohorts in flight, 1..MSGPM_SERVER_MAX_COHORTS (the
   default); MSGPM_E_INVALID outside that range.  It trades the median latency
   for the tail: with one cohort at a time, pairs that arrive in a burst queue
   for the GPU instead of sharing it, and the p99 latency is lowest; with four,
   the median is.  The throughput at capacity does not depend on it (a cohort
   of several pairs fills the GPU).  Takes effect at the next step; cohorts
   already in flight run to their end. */
#define MSGPM_SERVER_MAX_COHORTS 4
msgpm_status msgpm_server_set_cohorts(msgpm_server* server, int cohorts);
/* *pending: pairs queued or not yet done after this step. */
msgpm_status msgpm_server_step(msgpm_server* server, void* d_scratch, void* stream, int* pending);
msgpm_status msgpm_server_poll(msgpm_server* server, uint64_t ticket, int* done);
/* Waits until the pair's work has completed on the device, then retires the
   ticket as msgpm_server_poll does: MSGPM_OK when its results are complete,
   MSGPM_E_CANCELLED when it was cancelled in flight (its outputs are then
   undefined).  MSGPM_E_TIMEOUT after timeout_us microseconds (0: check once;
   negative: no limit) if it is not done; the ticket then stays valid.  A pair
   is done only after the msgpm_server_step calls that launch its last step,
   so a caller that waits with no limit must step the server from another
   thread.  Unknown ticket: MSGPM_E_INVALID. */
msgpm_status msgpm_server_wait(msgpm_server* server, uint64_t ticket, int64_t timeout_us);
/* Cancels a pair.  Queued: removed at once, its ticket retired (*retired = 1,
   may be NULL).  In flight: its cohort's work is already enqueued and runs to
   its end (the buffers are written until the pair is done); it is then
   reported done by msgpm_server_poll and cancelled by msgpm_server_wait, and
   its budget is released with its cohort's. */
msgpm_status msgpm_server_cancel(msgpm_server* server, uint64_t ticket, int* retired);

/* Test hook for the failure paths: the next n allocations the library itself
   makes (pinned host staging buffers, HIP events of the batched and serving
   forms) fail as if out of memory, and the call that needed one returns
   MSGPM_E_OOM with nothing enqueued.  0 switches the injection off. */
msgpm_status msgpm_debug_fail_allocations(int n);

/* ---------------------------------------------------------------------------
 * Kernel timing.  While enabled, the library records a pair of HIP events on
 * the launch stream around every kernel it launches (from any entry point) and
 * attributes the elapsed time to one of the kinds below.  msgpm_timing_read
 * waits for the recorded events, writes the total milliseconds and launch count
 * per kind since the last read (arrays of MSGPM_TIMER_KINDS elements, either
 * may be NULL) and starts a new accumulation.  Event objects are created on
 * first use and reused; no device memory is allocated.
 * ------------------------------------------------------------------------- */
enum {
  MSGPM_T_FEATURES = 0,
  MSGPM_T_INIT = 1,
  MSGPM_T_EVAL_COST = 2,
  MSGPM_T_PM_INIT = 3,       /* PatchMatch half-sweeps of the initial pass (identity patches) */
  MSGPM_T_PM_RESTRICTED = 4, /* restricted half-sweeps, pixels with a region plane (distorted patches) */
  MSGPM_T_RANSAC = 5,
  MSGPM_T_ASSIGN = 6,
  MSGPM_T_SYMMETRY = 7,
  MSGPM_T_FB = 8,
  MSGPM_T_NNF_UPDATE = 9,
  MSGPM_T_FINALIZE = 10,
  MSGPM_T_PM_LIST = 11,            /* pixel lists of the restricted half-sweeps */
  MSGPM_T_PM_RESTRICTED_IDENT = 12, /* restricted half-sweeps, pixels without one (identity patches) */
  MSGPM_T_FILL = 13,               /* filling by model propagation */
  MSGPM_TIMER_KINDS = 14
};
msgpm_status msgpm_timing_enable(int on);
msgpm_status msgpm_timing_read(double* ms, int64_t* launches);

/* Self-check of the FP16-storage arithmetic on the current device (R30: the
   FP16 form computes on the widened values).  The FP16 kernels widen halves
   inside mixed-precision multiply-adds; this compares every such form with an
   exact conversion followed by FP32 arithmetic, over all 65536 FP16 patterns
   in both halves of a word and `rounds` partner operands per pattern (12
   comparisons each).  Enqueued on `stream`; *d_mismatches, a device uint64,
   receives the number of differing results (results that are both NaN are
   not compared): 0 means the FP16 form's values are those of widening first.
   rounds: 1..4096, else MSGPM_E_INVALID. */
msgpm_status msgpm_check_fp16_arith(int32_t rounds, uint64_t* d_mismatches, void* stream);

/* Counters in the workspace (uint64[16][64] at layout.counters: 16 counters,
   each kept as 64 partial sums to be added by the reader), per direction
   d = 0, 1, reset by msgpm_init_state:
     [0 + d] candidates evaluated by the initial PatchMatch pass,
     [2 + d] cost refreshes (also those computed by MSGPM_PM_FRESH
     half-sweeps), [4 + d] candidates of the restricted passes at
     pixels with a region plane, [10 + d] at pixels without one,
     [6 + d], [8 + d], [12 + d] patch rows (2r+1 taps each) actually computed
     by the initial pass and the two restricted kinds (a candidate rejected
     early by its partial sum computes fewer rows). */

#ifdef __cplusplus
}
#endif
#endif /* MSGPM_H */
