// Internal declarations shared by the HIP translation units of libmsgpm.
// Written for gfx950 (CDNA4): wave64, 256-thread workgroups.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/msgpm.h"

namespace msgpm {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kXcds = 8;  // MI355X: 8 accelerator complex dies, each with its own L2
constexpr int kCounterKinds = 16;
constexpr int kCounterStripes = 64;  // copies of every counter, summed by the reader

// Parameters as kernels see them (passed by value).
struct DevParams {
  int W, H, C, r;
  int iters, hyps, R0, nk;   // nk: number of random-search radii
  int m_min_abs, eta_num, eta_den, fp16;
  int cues;                          // MSGPM_FLAG_CUE_* bits
  int fill_sweeps;                   // half-sweeps of the filling, 0 = none
  int histeq;                        // equalise the frames' HSV value channel
  int merge_strict;                  // strict level priority: only unassigned pixels are candidates
  int n_levels;
  int block[MSGPM_MAX_LEVELS];
  int nbx[MSGPM_MAX_LEVELS], nby[MSGPM_MAX_LEVELS];
  int plane_off[MSGPM_MAX_LEVELS];  // 2 * windows of the levels before
  int planes_per_dir;
  float gw;                          // gradient-channel weight
  double tau2, eps2, fb2, mu;
  uint64_t seed;
};

// Typed views of the workspace.
struct Ws {
  const void* feat[2];  // float4 plane (+ float plane) or 8-half records
  int32_t* nnf[2];
  float* cost[2];
  int32_t* win[2];
  double* loss[2];
  int32_t* hlabel[2];
  int32_t* twin[2];
  double* tloss[2];
  msgpm_plane* planes;
  unsigned long long* counters;
  unsigned* heq;          // histograms [2][256], then FP32 maps [2][256], then flags [2]
  int32_t* act[4];        // pixels a restricted half-sweep updates, [direction][colour]
  unsigned* act_count;    // list lengths [direction][colour][with region plane, without], then
                          // the filling's ring of 4 counts per direction
};

// Batched launches: one launch covers the same phase of several frame pairs.
// A pair is described by a PairDesc (its parameters, workspace and buffers);
// its share of a launch is an Item: virtual workgroups [start, start + nb) of
// the launch (start a multiple of kXcds, so that XCD-aware remaps within a
// pair stay valid; the virtual workgroups up to the next item's start do
// nothing).  The phase's arguments are the same for every pair of a launch
// and are passed by value (BArgs).  Launches are persistent: gridDim.x
// resident workgroups (a multiple of kXcds) take the `total` virtual
// workgroups in turn, so one launch per phase serves every window, tile and
// pair whatever their number.
//
// Everything that depends on the pairs (their number, descriptors, items and
// the launch totals) lives in a table in device memory, so that a kernel's
// arguments (the table, the launch's index in it, the phase arguments) and
// its grid depend only on the sequence of phases: a captured graph of a
// sequence serves any set of pairs that follows it.  Table layout (byte
// offsets from its base): BatchHead, then LaunchTab[n_launches], then the
// PairDesc array at desc_off, then the item lists.
struct PairDesc {
  DevParams P;
  Ws w;
  const float* rgb[2];
  const int32_t* init[2];
  float* flow[2];
  uint8_t* occ[2];
};
struct Item {
  int pair, start, nb;
};
struct BArgs {
  int a[5];
};
struct BatchHead {
  int n_launches, n_pairs;
  uint32_t desc_off;
  int pad;
};
struct LaunchTab {
  int total;       // virtual workgroups
  uint32_t items;  // byte offset of the launch's item list (n_pairs items)
};
// A launch's view of its table.
struct BatchView {
  const PairDesc* pd;
  const Item* it;
  int n, total;
};
__device__ inline BatchView batch_view(const uint8_t* __restrict__ tab, int k) {
  const BatchHead* h = reinterpret_cast<const BatchHead*>(tab);
  const LaunchTab* L = reinterpret_cast<const LaunchTab*>(tab + sizeof(BatchHead)) + k;
  return BatchView{reinterpret_cast<const PairDesc*>(tab + h->desc_off),
                   reinterpret_cast<const Item*>(tab + L->items), h->n_pairs, L->total};
}

// Workgroup coordinates within its pair's part of a launch.
struct Blk {
  int x, nx, y;
};
__device__ inline Blk blk_here() { return Blk{(int)blockIdx.x, (int)gridDim.x, (int)blockIdx.y}; }

// The item owning virtual workgroup b (items sorted by start; n >= 1).
__device__ inline int find_item(const Item* __restrict__ it, int n, int b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (it[mid].start <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Runs body(item, Blk) for every virtual workgroup of a batched launch that
// belongs to an item, this workgroup taking blockIdx.x, blockIdx.x +
// gridDim.x, ...  With gridDim.x a multiple of kXcds every virtual workgroup
// keeps the XCD its index names.  The virtual workgroups of one workgroup
// come in increasing order, so the owning item is found once and then
// advanced.  LDS: the whole workgroup synchronises between two virtual
// workgroups, so a body may use LDS as in a one-shot launch.
// LOOP = false: the one-shot form, one virtual workgroup per workgroup
// (gridDim.x >= total), for kernels whose registers the loop would crowd.
template <bool LDS = false, bool LOOP = true, class F>
__device__ __forceinline__ void for_each_item(const Item* __restrict__ it, int n, int total, F&& body) {
  int vb = blockIdx.x;
  if (vb >= total) return;
  int i = find_item(it, n, vb);
  if constexpr (!LOOP) {
    const int lb = vb - it[i].start;
    if (lb < it[i].nb) body(i, Blk{lb, it[i].nb, (int)blockIdx.y});
    return;
  }
  for (; vb < total; vb += gridDim.x) {
    while (i + 1 < n && it[i + 1].start <= vb) ++i;
    const int lb = vb - it[i].start;
    if (lb < it[i].nb) body(i, Blk{lb, it[i].nb, (int)blockIdx.y});
    if (LDS && vb + (int)gridDim.x < total) __syncthreads();
  }
}

__host__ __device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__host__ __device__ inline int32_t pack_off(int dx, int dy) {
  return (int32_t)(((uint32_t)dx & 0xffffu) | ((uint32_t)dy << 16));
}
__host__ __device__ inline int off_dx(int32_t v) { return (int16_t)((uint32_t)v & 0xffffu); }
__host__ __device__ inline int off_dy(int32_t v) { return (int16_t)((uint32_t)v >> 16); }

// Workgroup index remapped so that each XCD (which receives every 8th
// workgroup in dispatch order) works on one contiguous range of tiles, keeping
// neighbouring tiles in the same L2.
__device__ inline int xcd_remap(int bid, int nb) {
  const int q = nb / kXcds, rem = nb % kXcds;
  const int xcd = bid % kXcds, k = bid / kXcds;
  const int base = xcd < rem ? xcd * (q + 1) : rem * (q + 1) + (xcd - rem) * q;
  return base + k;
}

// Full 128-bit product of two 64-bit words from four 32 x 32 -> 64-bit
// multiply-adds (v_mad_u64_u32); no partial sum overflows, since
// (2^32 - 1)^2 + 2 (2^32 - 1) < 2^64.  The compiler's own lowering of a 64-bit
// product plus its high half recomputes the cross terms with separate 32-bit
// multiplies (seven quarter-rate instructions instead of four).
__device__ inline void mul64_wide(uint64_t a, uint64_t m, uint64_t& lo, uint64_t& hi) {
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
  const uint32_t m0 = (uint32_t)m, m1 = (uint32_t)(m >> 32);
  const uint64_t p00 = (uint64_t)a0 * m0;
  const uint64_t t = (uint64_t)a0 * m1 + (p00 >> 32);
  const uint64_t u = (uint64_t)a1 * m0 + (uint32_t)t;
  lo = (u << 32) | (uint32_t)p00;
  hi = (uint64_t)a1 * m1 + (t >> 32) + (u >> 32);
}

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter c, key (k0, k1).
__device__ inline void philox4x64(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t lo0, hi0, lo1, hi1;
    mul64_wide(c[0], M0, lo0, hi0);
    mul64_wide(c[2], M1, lo1, hi1);
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// Integer in [0, n) from the top 32 bits of a word (multiply-shift).
__device__ inline int draw_below(uint64_t w, uint32_t n) { return (int)(((w >> 32) * (uint64_t)n) >> 32); }

__device__ inline uint64_t rng_word3(int phase, int dir, int slot, int stage) {
  return ((uint64_t)phase << 24) | ((uint64_t)dir << 16) | ((uint64_t)slot << 8) | (uint64_t)stage;
}

// Plane record index (see msgpm_plane).
__host__ __device__ inline int plane_index(const DevParams& P, int dir, int level, int stage, int block) {
  return dir * P.planes_per_dir + P.plane_off[level] + (stage - 1) * P.nbx[level] * P.nby[level] + block;
}

// Window origin along an axis (windows overlap by half, the last is flush).
__host__ __device__ inline int block_origin(int n, int B, int i) {
  if (n <= B) return 0;
  const int o = i * (B / 2);
  return o > n - B ? n - B : o;
}

// Contiguous range [lo, hi] of windows covering coordinate c.
__host__ __device__ inline void cover_range(int n, int B, int nb, int c, int& lo, int& hi) {
  const int bw = B < n ? B : n;
  const int S = B / 2;
  if (n <= B) {
    lo = hi = 0;
    return;
  }
  lo = (c - bw < 0) ? 0 : ((c - bw) / S + 1);
  if (lo > nb - 1) lo = nb - 1;
  hi = (c >= n - bw) ? nb - 1 : (c / S);
  if (hi > nb - 1) hi = nb - 1;
}

// ---- launch wrappers (defined in the .hip files) ---------------------------
hipError_t launch_histeq(const DevParams& P, const Ws& w, const float* rgb1, const float* rgb2, hipStream_t s);
int heq_hist_blocks(const DevParams& P);
hipError_t launch_features(const DevParams& P, const Ws& w, const float* rgb, int frame, hipStream_t s);
hipError_t launch_init_state(const DevParams& P, const Ws& w, const int32_t* init0, const int32_t* init1,
                             hipStream_t s);
hipError_t launch_eval_cost(const DevParams& P, const Ws& w, int mode, hipStream_t s);
// initial pass (identity patches over every pixel of the colour); fresh: the
// pixels' current costs are computed in the sweep (the mode-0 cost refresh)
hipError_t launch_pm_halfsweep(const DevParams& P, const Ws& w, int colour, int iter, int slot, int fresh,
                               hipStream_t s);
// restricted pass: the pixel lists, then one kernel per list; fresh: the
// listed pixels' current costs are computed in the sweep (the mode-1 refresh)
hipError_t launch_pm_lists(const DevParams& P, const Ws& w, hipStream_t s);
hipError_t launch_pm_restricted(const DevParams& P, const Ws& w, int colour, int iter, int slot, int ident,
                                int fresh, hipStream_t s);
hipError_t launch_ransac(const DevParams& P, const Ws& w, int level, int stage, hipStream_t s);
hipError_t launch_assign(const DevParams& P, const Ws& w, int level, int stage, int tentative, hipStream_t s);
hipError_t launch_symmetry(const DevParams& P, const Ws& w, int level, int stage, hipStream_t s);
hipError_t launch_fb_unassign(const DevParams& P, const Ws& w, hipStream_t s);
hipError_t launch_nnf_update(const DevParams& P, const Ws& w, int level, hipStream_t s);
hipError_t launch_unique(const DevParams& P, const Ws& w, hipStream_t s);
hipError_t launch_fill(const DevParams& P, const Ws& w, hipStream_t s);
hipError_t launch_finalize(const DevParams& P, const Ws& w, float* flow0, float* flow1, uint8_t* occ0,
                           uint8_t* occ1, hipStream_t s);
hipError_t launch_check_fp16_arith(int rounds, unsigned long long* out, hipStream_t s);

// ---- batched launches -------------------------------------------------------
enum BatchKind {
  BK_HEQ_CLEAR,     // equalisation: histograms to zero
  BK_HEQ_HIST,      // grid.y = frame
  BK_HEQ_MAP,       // grid.y = frame
  BK_FEATURES,      // grid.y = frame
  BK_INIT_PIXELS,
  BK_INIT_PLANES,   // grid.y = 1
  BK_EVAL_COST_IDENT,  // a = {0}: identity-patch cost refresh
  BK_EVAL_COST_PLANE,  // a = {mode 1 or 2}: region-plane cost refresh
  BK_ZERO_ACTIVE,   // one workgroup per item, grid.y = 1
  BK_ACTIVE_LIST,   // a = {colour}
  BK_PM_INIT,       // a = {colour, iter, slot, 0 | 2 (fresh: cost computed in the sweep)}
  BK_PM_RESTRICTED, // a = {colour, iter, slot, 1 | 2 (fresh)}: pixels with a region plane
  BK_PM_RESTRICTED_IDENT,  // the same, pixels without one
  BK_RANSAC,        // a = {level, stage}
  BK_ASSIGN,        // a = {level, stage, tentative}
  BK_SYMMETRY,      // a = {level, stage}
  BK_FB,
  BK_COMMIT,
  BK_NNF_UPDATE,    // a = {level}
  BK_FINALIZE,
  BK_UNIQUE,        // a = {phase 0..3}: occlusion cue 2
  BK_FILL_CLEAR,
  BK_FILL,          // a = {half-sweep}
  BK_KINDS
};
// Workgroups (x) one pair needs for kernel `kind` with arguments a; grid.y.
int batch_blocks(int kind, const DevParams& P, const int* a);
int batch_grid_y(int kind);
// Launch k of the table at `tab`, run by `grid` resident workgroups (a
// multiple of kXcds); `lds`: dynamic LDS (RANSAC).  P0 selects the kernel
// instantiation (r, C, storage), equal for every pair.  persist = false (the
// PatchMatch kernels only): the one-shot form, grid >= the launch's total.
hipError_t launch_batched(int kind, const DevParams& P0, const uint8_t* tab, int k, int grid, size_t lds, BArgs A,
                          bool persist, hipStream_t s);
hipError_t launch_batched_init(int kind, const uint8_t* tab, int k, int grid, BArgs A, hipStream_t s);
hipError_t launch_batched_pm(int kind, const DevParams& P0, const uint8_t* tab, int k, int grid, BArgs A,
                             bool persist, hipStream_t s);
hipError_t launch_batched_planes(int kind, const uint8_t* tab, int k, int grid, size_t lds, BArgs A, hipStream_t s);
size_t ransac_smem_bytes(const DevParams& P, int level);
// The same for a full B x B window (any frame of at least that size).
size_t ransac_smem_bytes_window(int B);

}  // namespace msgpm
