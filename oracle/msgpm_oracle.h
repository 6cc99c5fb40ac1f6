/*
 * FP64 CPU oracle for the multi-scale generalized plane match (MSGPM) hot path
 * of Choi & Banerjee, "Multi-Scale Generalized Plane Match for Optical Flow"
 * (arXiv 1804.03787).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this library: only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the GPU
 * library; both follow the same written definitions (the paper plus the readings
 * listed in the design notes), each in its own code.
 *
 * Plain, slow C; every floating-point step is FP64 (features are FP32 or FP16
 * values widened to FP64).  Built with -O2 -ffp-contract=off, single-threaded
 * (the parity authority) and, from the same source, with -fopenmp: the loops
 * over the pixels of a phase and over the windows of a level are then shared
 * among threads.  Each such loop writes only its own element's state and reads
 * only state no iteration of the loop writes, and every floating-point value
 * is computed by one thread in the written order, so both builds give the same
 * bits (asserted by a test).
 *
 * Every phase function also reports per-element near-tie flags: a bit is set when
 * a discrete decision taken for that element (an argmin, a threshold test, a
 * rounding) was closer to its boundary than the band stated below, so that a
 * lower-precision or differently-ordered implementation may legitimately decide
 * the other way there.
 *
 * Near-tie bands (relative):
 *   PatchMatch cost comparisons   |a-b| <= 1e-5*max(a,b) + 1e-7*(2r+1)^2*C
 *   colour inlier e vs eps^2      |e-eps^2| <= 1e-9*eps^2
 *   plane loss comparisons        |L1-L2| <= 1e-9*max(L1,L2)  (planes with H differing by >1e-6)
 *   RANSAC inlier test            |e2 - tau^2 w^2| <= 1e-9*tau^2 w^2
 *   FB distance                   |d2 - tau_fb^2| <= 1e-9*tau_fb^2
 *   rounding                      |frac - 0.5| <= 1e-9
 *   image-bounds tests            |q - bound| <= 1e-9
 */
#ifndef MSGPM_ORACLE_H
#define MSGPM_ORACLE_H
#include <stdint.h>

#define ORC_MAX_LEVELS 8

/* Columns of the per-plane integer record (pinfo[P][ORC_PI_N]). */
enum {
  ORC_PI_DIR = 0, ORC_PI_LEVEL, ORC_PI_STAGE, ORC_PI_BLOCK,
  ORC_PI_X0, ORC_PI_Y0, ORC_PI_BW, ORC_PI_BH,
  ORC_PI_SUPPORT,   /* number of points handed to RANSAC */
  ORC_PI_COUNT,     /* final inlier count (after the refit decision) */
  ORC_PI_HYP,       /* index of the winning hypothesis, -1 if none */
  ORC_PI_HYPCOUNT,  /* its inlier count */
  ORC_PI_REFIT,     /* 1 if the least-squares refit was kept */
  ORC_PI_DETECTED,  /* count >= m_min */
  ORC_PI_RK,        /* |r_k|: colour-consistent pixels of the plane in its input set */
  ORC_PI_PASS,      /* pixels of r_k passing the forward-backward test */
  ORC_PI_VALID,     /* detected and kept by the symmetry test (and, with ORC_CUE_OVERLAP, the overlap test) */
  ORC_PI_RIN,       /* pixels of r_k that are also RANSAC inliers of the plane (occlusion cue 3) */
  ORC_PI_N
};

/* Near-tie flag bits. */
enum {
  ORC_F_COST = 1,     /* PatchMatch cost comparison */
  ORC_F_ROUND = 2,    /* rounding to the pixel grid */
  ORC_F_COLOUR = 4,   /* colour-consistency threshold or plane-loss argmin */
  ORC_F_FB = 8,       /* forward-backward distance threshold */
  ORC_F_BOUNDS = 16,  /* image-bounds test */
  ORC_F_RANSAC = 32,  /* RANSAC hypothesis choice / inlier count */
  ORC_F_TWOBEST = 64  /* PatchMatch: the two best costs over distinct targets of one update are
                         within the PatchMatch cost band (a narrower test than ORC_F_COST, which
                         compares every candidate with the running best) */
};

typedef struct orc_pair {
  /* geometry and cost */
  int32_t W, H, C, r;
  double wc[5];                 /* channel weights (1,1,1,gamma,gamma) */
  const float* F[2];            /* features of frame 1 and frame 2, HWC, C channels */
  /* method parameters */
  int32_t n_levels;
  int32_t block[ORC_MAX_LEVELS];
  int32_t iters, hyps, R0, m_min_abs, eta_num, eta_den;
  double tau, eps, tau_fb, mu;
  uint64_t seed;
  /* per-direction pixel state (dir 0: frame 1 -> frame 2, dir 1: frame 2 -> frame 1) */
  int32_t* nnf[2];              /* packed offset: (dx & 0xffff) | (dy << 16) */
  double* cost[2];
  int32_t* win[2];              /* assigned plane index, -1, or -2 - plane if filled */
  double* loss[2];              /* its loss L */
  int32_t* hlabel[2];           /* region plane index for the patch distortion, -1 = identity */
  int32_t* twin[2];             /* tentative / snapshot assignment */
  double* tloss[2];
  uint8_t* pflag[2];            /* per-pixel near-tie flags (OR-ed) */
  /* plane table */
  int32_t P;                    /* capacity = 2 dirs * 2 stages * sum of block counts */
  double* pH;                   /* P x 9 */
  int32_t* pinfo;               /* P x ORC_PI_N */
  uint8_t* bflag;               /* per-plane near-tie flags */
  /* statistics */
  int64_t evals;                /* warped-cost evaluations performed */
  /* optional occlusion cues of Sec. 3.4 beyond the forward-backward symmetry */
  int32_t cues;                 /* ORC_CUE_* bits */
  /* filling by homography-model propagation (Sec. 3.4.1): red-black
     half-sweeps, 0 = no filling */
  int32_t fill_sweeps;
  /* level priority of Sec. 3.3 taken strictly: an assigned pixel is no
     candidate of a later level (only unassigned pixels are assigned there);
     0 = the lexicographic key (L, level, stage, block) over every pixel */
  int32_t merge_strict;
} orc_pair;

enum {
  ORC_CUE_OVERLAP = 1,  /* cue 3: a plane must agree with its colour-consistent region */
  ORC_CUE_UNIQUE = 2    /* cue 2: of several pixels matched to one target, the higher-loss ones are occluded */
};

#ifdef __cplusplus
extern "C" {
#endif

/* Threads of the phase loops when the library is built with OpenMP (the
   result does not depend on it: every parallel loop writes disjoint elements
   and reads nothing written in the same loop); returns the count in use, 1 in
   the plain build. */
int orc_set_threads(int n);

/* Counter-based RNG: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
/* Integer draw in [0, n) from the top 32 bits of a 64-bit word (multiply-shift). */
uint32_t orc_draw(uint64_t word, uint32_t n);

/* Features (O1): rgb is HWC FP32; feat gets C (3 or 5) FP32 channels per pixel.
   fp16 != 0 rounds every feature to binary16 (nearest even) and back. */
void orc_features(const float* rgb, int W, int H, int C, int fp16, float* feat);
/* Histogram equalisation of the HSV value channel (Sec. 4.2): rgb and out are
   HWC FP32 (3 channels), out may not alias rgb.  See the definition above
   orc_histeq in the source. */
void orc_histeq(const float* rgb, int W, int H, float* out);
float orc_round_fp16(float x);

/* Homography projection; returns 0 when the homogeneous w is not positive. */
int orc_project(const double* Hm, double x, double y, double* qx, double* qy);

/* Warped-patch SSD C(p, t, H) (O3).  Hm may be NULL for the identity. */
double orc_cost(const orc_pair* S, int dir, int px, int py, int tx, int ty, const double* Hm);
/* Brute force for tests: cost of every pixel against every target with H = I,
   out[(p * W * H) + t]. */
void orc_cost_all(const orc_pair* S, int dir, double* out);

/* Number of block origins along an axis of length n for block side B (O6). */
int orc_block_count(int n, int B);
int orc_block_origin(int n, int B, int i);
int orc_plane_capacity(const orc_pair* S);
int orc_plane_index(const orc_pair* S, int dir, int level, int stage, int block);
int orc_m_min(const orc_pair* S, int bw, int bh);
/* Fills the static columns (dir, level, stage, block, rectangle) of every plane
   and clears the rest. */
void orc_planes_init(orc_pair* S);

/* O4: random initial NNF of one direction. */
void orc_nnf_init(orc_pair* S, int dir);
/* Cost refresh: cost[p] = C(p, p+v_p, H) for the pixels selected by mode:
   mode 0 = all pixels with H = identity,
   mode 1 = unassigned pixels with H = region plane (hlabel),
   mode 2 = assigned pixels with H = their assigned plane. */
void orc_eval_cost(orc_pair* S, int dir, int mode);
/* O5: one red-black half-sweep of one direction.  restricted = 0 for the init
   pass (all pixels active, H = identity); 1 for a restricted pass (active =
   unassigned, H = region plane, plus the plane candidate). */
void orc_pm_halfsweep(orc_pair* S, int dir, int colour, int iter, int slot, int restricted);

/* O7 / O11: RANSAC over every block of one level and stage for one direction. */
void orc_ransac(orc_pair* S, int dir, int level, int stage);
/* Hypothesis generator used by RANSAC, exposed for tests: the 4-point DLT with
   Hartley normalisation.  Returns 0 when rejected. */
int orc_dlt4(const double* sx, const double* sy, const double* dx, const double* dy, double* Hout);
/* Least-squares homography from n >= 4 correspondences (normal equations). */
int orc_refit(const double* sx, const double* sy, const double* dx, const double* dy, int n, double* Hout);
/* Solves A x = b (n <= 8, A row-major n x n) by Gaussian elimination with
   partial pivoting; returns 0 if a pivot magnitude falls below 1e-10. */
int orc_gauss_solve(double* A, double* b, int n, double* x);

/* Colour-consistency error e(p, H) (O8); +inf when q leaves the image. */
double orc_colour_err(const orc_pair* S, int dir, int px, int py, const double* Hm, int* near_bounds);

/* O9: assignment for one level/stage and direction.
   tentative = 1: candidates are detected planes, result written to twin/tloss;
   tentative = 0: candidates are valid planes, result written in place to win/loss. */
void orc_assign(orc_pair* S, int dir, int level, int stage, int tentative);
/* O10 counting step: for every detected plane of (level, stage) in both
   directions, count r_k and FB passes against the other direction's tentative
   winners (twin) and set the valid column. */
void orc_symmetry(orc_pair* S, int level, int stage);
/* Occlusion cue 2 (many-to-one matches), both directions: every assigned pixel
   whose plane sends it (rounded to the grid) to a target inside the frame
   competes with the other assigned pixels sent to that target; the one with
   the smallest loss keeps its plane (ties: the smallest pixel index), the
   others are unassigned. */
void orc_unique(orc_pair* S);
/* Filling by homography-model propagation (Sec. 3.4.1), both directions, after
   the last level: fill_sweeps red-black half-sweeps over the unassigned pixels
   (colour (x + y) % 2 == t % 2 in half-sweep t).  An unassigned pixel takes,
   of the planes held by its four neighbours (assigned or already filled), the
   one with the smallest colour error (ties: the smallest plane index) if that
   error is below eps^2; it is then marked filled: win = -2 - plane,
   loss = the error.  Stops early after two half-sweeps that fill nothing
   (nothing can change after them). */
void orc_fill(orc_pair* S);
/* Forward-backward test FB(p, H) of direction dir against the other direction's
   assignment array `other_win`. */
int orc_fb_test(const orc_pair* S, int dir, int px, int py, const double* Hm, const int32_t* other_win, uint8_t* flag);
/* O12: Jacobi end-of-level FB; assigned pixels failing FB become unassigned. */
void orc_fb_unassign(orc_pair* S);
/* O13 + O14: NNF update from assigned planes and region plane choice. */
void orc_nnf_update(orc_pair* S, int dir, int level);
/* O15 outputs: flow (H*W*2, FP32; a plane's flow where the pixel has one, else
   its NNF offset), occlusion mask (0 = assigned, 1 = no plane: occluded,
   2 = filled by model propagation). Costs of assigned pixels are refreshed
   under their plane. */
void orc_finalize(orc_pair* S, int dir, float* flow, uint8_t* occ);

/* Whole pipeline (O15) for both directions: init pass, then per level the two
   plane stages, FB, NNF update and the restricted pass.  init_nnf may be NULL
   (random init). */
void orc_solve(orc_pair* S, const int32_t* init_nnf0, const int32_t* init_nnf1,
               float* flow0, float* flow1, uint8_t* occ0, uint8_t* occ1);

#ifdef __cplusplus
}
#endif
#endif
