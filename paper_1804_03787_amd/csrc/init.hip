// Feature preparation and state initialisation.
//
// Features: the patch cost of the paper compares colours (Sec. 3.1.3); the cost
// here may add luma gradients.  Luma Y = (0.299 R + 0.587 G) + 0.114 B in FP32
// without contraction; gx = 0.5 (Y(x+1) - Y(x-1)), gy likewise, with replicate
// borders.  Stored interleaved per pixel: C floats (R, G, B[, gx, gy]), or in
// the FP16 form 4 halves (R, G, B, 0) / 6 halves (R, G, B, gx, gy, 0).  One zero
// pixel follows the last one so that a horizontal pair load at the last pixel
// stays inside the buffer.
#include "common.h"

#include <hip/hip_fp16.h>

#pragma clang fp contract(off)

namespace msgpm {

// ---------------------------------------------------------------------------
// Equalisation of the HSV value channel (illumination experiment, Sec. 4.2).
// Histogram: workgroups of kHeqSpan pixels, privatised in LDS, then one global
// atomic per occupied bin.  Map: one workgroup per frame, inclusive scan of the
// 256 bins.  The features kernel applies the map to every pixel it reads.
// ---------------------------------------------------------------------------
constexpr int kHeqSpan = 16 * kBlock;

__device__ inline int v_level(float V) {
  const float t = V * 255.0f + 0.5f;
  if (!(t >= 0.0f)) return 0;
  if (t >= 255.0f) return 255;
  return (int)t;
}

__device__ __forceinline__ void heq_clear_body(const Ws& w) {
  w.heq[threadIdx.x] = 0;
  w.heq[kBlock + threadIdx.x] = 0;
}

__device__ __forceinline__ void heq_hist_body(const float* __restrict__ rgb, int n, unsigned* __restrict__ hist,
                                              Blk bk) {
  __shared__ unsigned h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int p0 = bk.x * kHeqSpan;
  for (int k = 0; k < kHeqSpan / kBlock; ++k) {
    const int p = p0 + k * kBlock + threadIdx.x;
    if (p < n) atomicAdd(&h[v_level(fmaxf(fmaxf(rgb[3 * p], rgb[3 * p + 1]), rgb[3 * p + 2]))], 1u);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

__device__ __forceinline__ void heq_map_body(const unsigned* __restrict__ hist, float* __restrict__ map, int* flag,
                                             unsigned n) {
  __shared__ unsigned cdf[256];
  __shared__ unsigned cmin;
  const int q = threadIdx.x;
  const unsigned hq = hist[q];
  cdf[q] = hq;
  __syncthreads();
  for (int d = 1; d < 256; d <<= 1) {  // inclusive scan (Hillis-Steele)
    const unsigned v = q >= d ? cdf[q - d] : 0u;
    __syncthreads();
    cdf[q] += v;
    __syncthreads();
  }
  if (hq && cdf[q] == hq) cmin = hq;  // the lowest occupied level: nothing below it
  __syncthreads();
  const unsigned c = cdf[q], m = cmin;
  map[q] = c < m ? 0.0f : (float)((double)(c - m) / (double)(n - m));
  if (q == 0) *flag = m == n ? 1 : 0;
}

// One pixel of the frame as the method sees it: equalised when map != null.
__device__ inline void frame_rgb(const float* __restrict__ rgb, int p, const float* __restrict__ map, int flat,
                                 float out[3]) {
  const float R = rgb[3 * p], G = rgb[3 * p + 1], B = rgb[3 * p + 2];
  if (!map || flat) {
    out[0] = R;
    out[1] = G;
    out[2] = B;
    return;
  }
  const float V = fmaxf(fmaxf(R, G), B);
  const float Vn = map[v_level(V)];
  if (V > 0.0f) {
    const float s = Vn / V;
    out[0] = R * s;
    out[1] = G * s;
    out[2] = B * s;
  } else {
    out[0] = out[1] = out[2] = Vn;
  }
}

__device__ inline float luma(const float* rgb, int p, const float* map, int flat) {
  float c[3];
  frame_rgb(rgb, p, map, flat, c);
  const float t = 0.299f * c[0];
  const float u = 0.587f * c[1];
  const float v = 0.114f * c[2];
  return (t + u) + v;
}

__device__ __forceinline__ void features_body(const float* __restrict__ rgb, int W, int H, int C, int fp16,
                                              const float* __restrict__ map, int flat, void* __restrict__ feat,
                                              Blk bk) {
  const int p = bk.x * kBlock + threadIdx.x;
  const int n = W * H;
  if (p > n) return;
  float v[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
  if (p < n) {
    const int x = p % W, y = p / W;
    frame_rgb(rgb, p, map, flat, v);
    if (C == 5) {
      const int xl = x > 0 ? x - 1 : 0, xr = x < W - 1 ? x + 1 : W - 1;
      const int yu = y > 0 ? y - 1 : 0, yd = y < H - 1 ? y + 1 : H - 1;
      v[3] = 0.5f * (luma(rgb, y * W + xr, map, flat) - luma(rgb, y * W + xl, map, flat));
      v[4] = 0.5f * (luma(rgb, yd * W + x, map, flat) - luma(rgb, yu * W + x, map, flat));
    }
  }
  if (fp16) {
    const int S = C == 3 ? 4 : 6;
    __half* h = reinterpret_cast<__half*>(feat) + (size_t)S * p;
    for (int k = 0; k < S; ++k) h[k] = __float2half_rn(k < C ? v[k] : 0.f);
  } else {
    float* f = reinterpret_cast<float*>(feat) + (size_t)C * p;
    for (int k = 0; k < C; ++k) f[k] = v[k];
  }
}

__device__ inline const float* heq_map(const DevParams& P, const Ws& w, int frame) {
  return P.histeq ? reinterpret_cast<const float*>(w.heq + 512) + 256 * frame : nullptr;
}
__device__ inline int heq_flat(const DevParams& P, const Ws& w, int frame) {
  return P.histeq ? (int)w.heq[1024 + frame] : 0;
}

__global__ __launch_bounds__(kBlock) void k_heq_clear(Ws w) { heq_clear_body(w); }

__global__ __launch_bounds__(kBlock) void k_heq_hist(DevParams P, Ws w, const float* __restrict__ rgb1,
                                                    const float* __restrict__ rgb2) {
  const Blk bk = blk_here();
  heq_hist_body(bk.y ? rgb2 : rgb1, P.W * P.H, w.heq + 256 * bk.y, bk);
}

__global__ __launch_bounds__(kBlock) void k_heq_map(DevParams P, Ws w) {
  const int f = blockIdx.y;
  heq_map_body(w.heq + 256 * f, reinterpret_cast<float*>(w.heq + 512) + 256 * f, reinterpret_cast<int*>(w.heq + 1024 + f),
               (unsigned)(P.W * P.H));
}

__global__ __launch_bounds__(kBlock) void k_features(DevParams P, Ws w, const float* __restrict__ rgb, int frame) {
  features_body(rgb, P.W, P.H, P.C, P.fp16, heq_map(P, w, frame), heq_flat(P, w, frame),
                const_cast<void*>(w.feat[frame]), blk_here());
}

// batched: grid.y = frame
__global__ __launch_bounds__(kBlock) void kb_heq_clear(const uint8_t* __restrict__ tab, int k, BArgs A) {
  const BatchView V = batch_view(tab, k);
  const PairDesc* __restrict__ pd = V.pd;
  const Item* __restrict__ it = V.it;
  const int n = V.n, total = V.total;
  for_each_item(it, n, total, [&](int i, Blk bk) {
    heq_clear_body(pd[it[i].pair].w);
  });
}

__global__ __launch_bounds__(kBlock) void kb_heq_hist(const uint8_t* __restrict__ tab, int k, BArgs A) {
  const BatchView V = batch_view(tab, k);
  const PairDesc* __restrict__ pd = V.pd;
  const Item* __restrict__ it = V.it;
  const int n = V.n, total = V.total;
  for_each_item<true>(it, n, total, [&](int i, Blk bk) {
    const PairDesc& D = pd[it[i].pair];
    heq_hist_body(D.rgb[bk.y], D.P.W * D.P.H, D.w.heq + 256 * bk.y, bk);
  });
}

__global__ __launch_bounds__(kBlock) void kb_heq_map(const uint8_t* __restrict__ tab, int k, BArgs A) {
  const BatchView V = batch_view(tab, k);
  const PairDesc* __restrict__ pd = V.pd;
  const Item* __restrict__ it = V.it;
  const int n = V.n, total = V.total;
  for_each_item<true>(it, n, total, [&](int i, Blk bk) {
    const PairDesc& D = pd[it[i].pair];
    const int f = bk.y;
    heq_map_body(D.w.heq + 256 * f, reinterpret_cast<float*>(D.w.heq + 512) + 256 * f,
                 reinterpret_cast<int*>(D.w.heq + 1024 + f), (unsigned)(D.P.W * D.P.H));
  });
}

__global__ __launch_bounds__(kBlock) void kb_features(const uint8_t* __restrict__ tab, int k, BArgs A) {
  const BatchView V = batch_view(tab, k);
  const PairDesc* __restrict__ pd = V.pd;
  const Item* __restrict__ it = V.it;
  const int n = V.n, total = V.total;
  for_each_item(it, n, total, [&](int i, Blk bk) {
    const PairDesc& D = pd[it[i].pair];
    features_body(D.rgb[bk.y], D.P.W, D.P.H, D.P.C, D.P.fp16, heq_map(D.P, D.w, bk.y), heq_flat(D.P, D.w, bk.y),
                  const_cast<void*>(D.w.feat[bk.y]), bk);
  });
}

int heq_hist_blocks(const DevParams& P) { return (P.W * P.H + kHeqSpan - 1) / kHeqSpan; }

hipError_t launch_histeq(const DevParams& P, const Ws& w, const float* rgb1, const float* rgb2, hipStream_t s) {
  hipLaunchKernelGGL(k_heq_clear, dim3(1), dim3(kBlock), 0, s, w);
  hipLaunchKernelGGL(k_heq_hist, dim3(heq_hist_blocks(P), 2), dim3(kBlock), 0, s, P, w, rgb1, rgb2);
  hipLaunchKernelGGL(k_heq_map, dim3(1, 2), dim3(kBlock), 0, s, P, w);
  return hipGetLastError();
}

hipError_t launch_features(const DevParams& P, const Ws& w, const float* rgb, int frame, hipStream_t s) {
  const int n = P.W * P.H + 1;  // pixels plus the zero pad pixel
  hipLaunchKernelGGL(k_features, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, P, w, rgb, frame);
  return hipGetLastError();
}

// Initial NNF: caller's offsets with targets clamped into the frame, or a
// uniform random target per pixel from the Philox stream (phase 1, draw 0).
__device__ __forceinline__ void init_pixels_body(const DevParams& P, const Ws& w, const int32_t* __restrict__ init0,
                                                 const int32_t* __restrict__ init1, Blk bk) {
  const int p = bk.x * kBlock + threadIdx.x;
  const int dir = bk.y;
  const int W = P.W, H = P.H;
  if (p >= W * H) return;
  const int x = p % W, y = p / W;
  const int32_t* init = dir ? init1 : init0;
  int tx, ty;
  if (init) {
    const int32_t v = init[p];
    tx = clampi(x + off_dx(v), 0, W - 1);
    ty = clampi(y + off_dy(v), 0, H - 1);
  } else {
    uint64_t c[4] = {(uint64_t)(uint32_t)p, 0, 0, rng_word3(1, dir, 0, 0)};
    philox4x64(c, P.seed, 0);
    tx = draw_below(c[0], (uint32_t)W);
    ty = draw_below(c[1], (uint32_t)H);
  }
  w.nnf[dir][p] = pack_off(tx - x, ty - y);
  w.win[dir][p] = -1;
  w.loss[dir][p] = __builtin_huge_val();
  w.hlabel[dir][p] = -1;
  w.twin[dir][p] = -1;
  w.tloss[dir][p] = __builtin_huge_val();
  w.cost[dir][p] = 0.f;
}

__global__ __launch_bounds__(kBlock) void k_init_pixels(DevParams P, Ws w, const int32_t* __restrict__ init0,
                                                       const int32_t* __restrict__ init1) {
  init_pixels_body(P, w, init0, init1, blk_here());
}

__global__ __launch_bounds__(kBlock) void kb_init_pixels(const uint8_t* __restrict__ tab, int k, BArgs A) {
  const BatchView V = batch_view(tab, k);
  const PairDesc* __restrict__ pd = V.pd;
  const Item* __restrict__ it = V.it;
  const int n = V.n, total = V.total;
  for_each_item(it, n, total, [&](int i, Blk bk) {
    const PairDesc& D = pd[it[i].pair];
    init_pixels_body(D.P, D.w, D.init[0], D.init[1], bk);
  });
}

__device__ __forceinline__ void init_planes_body(const DevParams& P, const Ws& w, Blk bk) {
  const int k = bk.x * kBlock + threadIdx.x;
  for (int c = k; c < kCounterKinds * kCounterStripes; c += bk.nx * kBlock) w.counters[c] = 0;
  if (k >= 2 * P.planes_per_dir) return;
  const int dir = k / P.planes_per_dir;
  int r = k - dir * P.planes_per_dir;
  int level = 0;
  while (level + 1 < P.n_levels && r >= P.plane_off[level + 1]) ++level;
  r -= P.plane_off[level];
  const int nb = P.nbx[level] * P.nby[level];
  const int stage = r / nb + 1;
  const int b = r % nb;
  const int B = P.block[level];
  msgpm_plane pl;
  for (int i = 0; i < 9; ++i) pl.H[i] = 0.0;
  pl.dir = dir;
  pl.level = level;
  pl.stage = stage;
  pl.block = b;
  pl.x0 = block_origin(P.W, B, b % P.nbx[level]);
  pl.y0 = block_origin(P.H, B, b / P.nbx[level]);
  pl.bw = B < P.W ? B : P.W;
  pl.bh = B < P.H ? B : P.H;
  pl.support = pl.count = 0;
  pl.hyp = -1;
  pl.hyp_count = 0;
  pl.refit = pl.detected = pl.rk = pl.pass = pl.valid = pl.rin = 0;
  w.planes[k] = pl;
}

__global__ __launch_bounds__(kBlock) void k_init_planes(DevParams P, Ws w) { init_planes_body(P, w, blk_here()); }

__global__ __launch_bounds__(kBlock) void kb_init_planes(const uint8_t* __restrict__ tab, int k, BArgs A) {
  const BatchView V = batch_view(tab, k);
  const PairDesc* __restrict__ pd = V.pd;
  const Item* __restrict__ it = V.it;
  const int n = V.n, total = V.total;
  for_each_item(it, n, total, [&](int i, Blk bk) {
    const PairDesc& D = pd[it[i].pair];
    init_planes_body(D.P, D.w, bk);
  });
}

hipError_t launch_init_state(const DevParams& P, const Ws& w, const int32_t* init0, const int32_t* init1,
                             hipStream_t s) {
  const int n = P.W * P.H;
  hipLaunchKernelGGL(k_init_pixels, dim3((n + kBlock - 1) / kBlock, 2), dim3(kBlock), 0, s, P, w, init0, init1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int np = 2 * P.planes_per_dir;
  const int nblk = np > kBlock ? np : kBlock;
  hipLaunchKernelGGL(k_init_planes, dim3((nblk + kBlock - 1) / kBlock), dim3(kBlock), 0, s, P, w);
  return hipGetLastError();
}

hipError_t launch_batched_init(int kind, const uint8_t* tab, int k, int grid, BArgs A, hipStream_t s) {
  switch (kind) {
    case BK_HEQ_CLEAR:
      hipLaunchKernelGGL(kb_heq_clear, dim3(grid, 1), dim3(kBlock), 0, s, tab, k, A);
      break;
    case BK_HEQ_HIST:
      hipLaunchKernelGGL(kb_heq_hist, dim3(grid, 2), dim3(kBlock), 0, s, tab, k, A);
      break;
    case BK_HEQ_MAP:
      hipLaunchKernelGGL(kb_heq_map, dim3(grid, 2), dim3(kBlock), 0, s, tab, k, A);
      break;
    case BK_FEATURES:
      hipLaunchKernelGGL(kb_features, dim3(grid, 2), dim3(kBlock), 0, s, tab, k, A);
      break;
    case BK_INIT_PIXELS:
      hipLaunchKernelGGL(kb_init_pixels, dim3(grid, 2), dim3(kBlock), 0, s, tab, k, A);
      break;
    case BK_INIT_PLANES:
      hipLaunchKernelGGL(kb_init_planes, dim3(grid, 1), dim3(kBlock), 0, s, tab, k, A);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace msgpm
