// Warped-patch SSD and PatchMatch half-sweeps (the per-pixel hot loop).
//
// Cost C(p, t, H): sum over the (2r+1)^2 taps d of the square patch of p of
//   sum_c w_c (F1_c(clamp(p + d)) - bilinear F2_c(t + Delta(d)))^2,
// Delta(d) = pi(H(p + d)) - pi(H p): the patch in the other frame is the square
// patch distorted by the plane's local motion around p (Sec. 3.1.3 compensates
// the plane distortion instead of enumerating distortions, Sec. 1).  The
// integer part of t + Delta is formed in integers, the fraction separately;
// bases below 0 or at/after the last pixel clamp with fraction 0.
//
// Work mapping (gfx950, wave64): a pixel is handled by 2r+1 adjacent lanes, lane
// j owning patch column dx = j - r for every candidate.  Each lane keeps its
// column's source features and tap geometry in registers; a candidate costs
// each lane 2r+1 gathers (4 bilinear corners in the distorted form, 1 for the
// identity form) and the column partial sums are combined across the group in a
// fixed order, so every lane of the group takes the same decisions.  Costs are
// accumulated in FP32.
//
// PatchMatch (propagation + random search, as used by the paper for its NNF,
// Sec. 3.1) runs as red-black Jacobi half-sweeps: a pixel reads only the other
// colour's offsets, so a half-sweep is order-free.
#include "common.h"

#include <hip/hip_fp16.h>

#pragma clang fp contract(off)

namespace msgpm {

template <int C, bool FP16>
__device__ inline void load_px(const void* __restrict__ F, int npix, int idx, float* v) {
  if constexpr (FP16) {
    const uint4 u = reinterpret_cast<const uint4*>(F)[idx];
    const float2 a = __half22float2(__builtin_bit_cast(__half2, u.x));
    const float2 b = __half22float2(__builtin_bit_cast(__half2, u.y));
    v[0] = a.x;
    v[1] = a.y;
    v[2] = b.x;
    if constexpr (C == 5) {
      const float2 c = __half22float2(__builtin_bit_cast(__half2, u.z));
      v[3] = b.y;
      v[4] = c.x;
    }
  } else {
    const float4 a = reinterpret_cast<const float4*>(F)[idx];
    v[0] = a.x;
    v[1] = a.y;
    v[2] = a.z;
    if constexpr (C == 5) {
      v[3] = a.w;
      v[4] = reinterpret_cast<const float*>(reinterpret_cast<const float4*>(F) + npix)[idx];
    }
  }
}

// Per-lane state of one pixel: the lane's patch column of source features and
// the tap geometry (integer offset + fraction of Delta(d)) of that column.
template <int R, int C, bool IDENT>
struct LaneCol {
  static constexpr int T = 2 * R + 1;
  float f1[T][C];
  int ox[T], oy[T];
  float fx[IDENT ? 1 : T], fy[IDENT ? 1 : T];
};

// Tap geometry of column dx for plane H at pixel (x, y).  Returns false when
// the homogeneous coordinate is not positive somewhere (cost = +inf).
template <int R, int C, bool IDENT>
__device__ inline bool setup_geometry(LaneCol<R, C, IDENT>& L, const double* H, int x, int y, int dx, float lim) {
  if constexpr (IDENT) {
#pragma unroll
    for (int t = 0; t < 2 * R + 1; ++t) {
      L.ox[t] = dx;
      L.oy[t] = t - R;
    }
    return true;
  } else {
    if (H == nullptr) {
#pragma unroll
      for (int t = 0; t < 2 * R + 1; ++t) {
        L.ox[t] = dx;
        L.oy[t] = t - R;
        L.fx[t] = 0.f;
        L.fy[t] = 0.f;
      }
      return true;
    }
    // Delta(d) = (A/w - q g^T) d / (1 + g.d) with q = pi(Hp), g = (h6, h7)/w.
    const double w = H[6] * x + H[7] * y + H[8];
    if (!(w > 0)) return false;
    const double qx = (H[0] * x + H[1] * y + H[2]) / w;
    const double qy = (H[3] * x + H[4] * y + H[5]) / w;
    const double g0 = H[6] / w, g1 = H[7] / w;
    const float m00 = (float)(H[0] / w - qx * g0), m01 = (float)(H[1] / w - qx * g1);
    const float m10 = (float)(H[3] / w - qy * g0), m11 = (float)(H[4] / w - qy * g1);
    const float fg0 = (float)g0, fg1 = (float)g1;
    bool ok = true;
    const float fdx = (float)dx;
#pragma unroll
    for (int t = 0; t < 2 * R + 1; ++t) {
      const float fdy = (float)(t - R);
      const float den = fmaf(fg1, fdy, fmaf(fg0, fdx, 1.0f));
      ok = ok && (den > 0.f);
      const float inv = 1.0f / den;
      float Dx = fmaf(m01, fdy, m00 * fdx) * inv;
      float Dy = fmaf(m11, fdy, m10 * fdx) * inv;
      Dx = fminf(fmaxf(Dx, -lim), lim);
      Dy = fminf(fmaxf(Dy, -lim), lim);
      const float flx = floorf(Dx), fly = floorf(Dy);
      L.ox[t] = (int)flx;
      L.oy[t] = (int)fly;
      L.fx[t] = Dx - flx;
      L.fy[t] = Dy - fly;
    }
    return ok;
  }
}

template <int R, int C, bool FP16, bool IDENT>
__device__ inline void load_column(LaneCol<R, C, IDENT>& L, const void* F1, int W, int H, int x, int y, int dx) {
  const int cx = clampi(x + dx, 0, W - 1);
#pragma unroll
  for (int t = 0; t < 2 * R + 1; ++t) {
    const int cy = clampi(y + t - R, 0, H - 1);
    load_px<C, FP16>(F1, W * H, cy * W + cx, L.f1[t]);
  }
}

// Column partial of the cost for target (tx, ty).
template <int R, int C, bool FP16, bool IDENT>
__device__ inline float column_cost(const LaneCol<R, C, IDENT>& L, const void* __restrict__ F2, int W, int H, int tx,
                                    int ty, float gw) {
  float acc = 0.f;
  const int npix = W * H;
#pragma unroll
  for (int t = 0; t < 2 * R + 1; ++t) {
    float v[C];
    int bx = tx + L.ox[t], by = ty + L.oy[t];
    if constexpr (IDENT) {
      bx = clampi(bx, 0, W - 1);
      by = clampi(by, 0, H - 1);
      load_px<C, FP16>(F2, npix, by * W + bx, v);
    } else {
      float fx = L.fx[t], fy = L.fy[t];
      if (bx < 0) {
        bx = 0;
        fx = 0.f;
      } else if (bx >= W - 1) {
        bx = W - 1;
        fx = 0.f;
      }
      if (by < 0) {
        by = 0;
        fy = 0.f;
      } else if (by >= H - 1) {
        by = H - 1;
        fy = 0.f;
      }
      const int i00 = by * W + bx;
      const int i01 = i00 + (bx < W - 1 ? 1 : 0);
      const int i10 = i00 + (by < H - 1 ? W : 0);
      const int i11 = i10 + (bx < W - 1 ? 1 : 0);
      float a[C], b[C], c[C], d[C];
      load_px<C, FP16>(F2, npix, i00, a);
      load_px<C, FP16>(F2, npix, i01, b);
      load_px<C, FP16>(F2, npix, i10, c);
      load_px<C, FP16>(F2, npix, i11, d);
#pragma unroll
      for (int k = 0; k < C; ++k) {
        const float top = fmaf(fx, b[k] - a[k], a[k]);
        const float bot = fmaf(fx, d[k] - c[k], c[k]);
        v[k] = fmaf(fy, bot - top, top);
      }
    }
    float row = 0.f;
#pragma unroll
    for (int k = 0; k < C; ++k) {
      const float e = L.f1[t][k] - v[k];
      row = (k < 3) ? fmaf(e, e, row) : fmaf(gw * e, e, row);
    }
    acc += row;
  }
  return acc;
}

// Sum of the group's column partials in lane order; identical on every lane.
template <int G>
__device__ inline float group_sum(float v, int base) {
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < G; ++k) s += __shfl(v, base + k);
  return s;
}

__device__ inline const double* plane_H(const Ws& w, int label) {
  return label >= 0 ? w.planes[label].H : nullptr;
}

// Adds each group's evaluation count into counters[dir] with one atomic per
// wave; called by every lane of the wave (outside divergent code).
__device__ inline void count_evals(unsigned long long* ctr, unsigned v) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & (kWave - 1)) == 0 && v) atomicAdd(ctr, (unsigned long long)v);
}

// ---------------------------------------------------------------------------
// Cost refresh: cost[p] = C(p, p + v_p, H_p) for the selected pixels.
// ---------------------------------------------------------------------------
template <int R, int C, bool FP16, bool IDENT>
__global__ __launch_bounds__(kBlock) void k_eval_cost(DevParams P, Ws w, int mode) {
  constexpr int G = 2 * R + 1, NG = kWave / G;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int g = lane / G, j = lane - g * G, base = g * G;
  const int dir = blockIdx.y;
  const int W = P.W, H = P.H;
  const long long i = ((long long)xcd_remap(blockIdx.x, gridDim.x) * (kBlock / kWave) + wave) * NG + g;
  bool act = g < NG && i < (long long)W * H;
  const int p = act ? (int)i : 0, x = p % W, y = p / W;
  int label = -1;
  if (act && mode == 1) {
    act = w.win[dir][p] < 0;
    label = w.hlabel[dir][p];
  } else if (act && mode == 2) {
    label = w.win[dir][p];
    act = label >= 0;
  }
  unsigned evals = 0;
  if (act) {
    const float lim = 4.0f * (float)(W > H ? W : H);
    LaneCol<R, C, IDENT> L;
    const bool ok = setup_geometry<R, C, IDENT>(L, plane_H(w, label), x, y, j - R, lim);
    const bool all_ok = group_sum<G>(ok ? 0.f : 1.f, base) == 0.f;
    const int32_t v = w.nnf[dir][p];
    float c = __builtin_huge_valf();
    if (all_ok) {
      load_column<R, C, FP16, IDENT>(L, w.feat[dir], W, H, x, y, j - R);
      c = group_sum<G>(
          column_cost<R, C, FP16, IDENT>(L, w.feat[1 - dir], W, H, x + off_dx(v), y + off_dy(v), P.gw), base);
    }
    if (j == 0) {
      w.cost[dir][p] = c;
      evals = 1;
    }
  }
  count_evals(&w.counters[2 + dir], evals);
}

// ---------------------------------------------------------------------------
// One red-black half-sweep over the pixels of one colour, both directions.
// ---------------------------------------------------------------------------
template <int R, int C, bool FP16, bool IDENT>
__global__ __launch_bounds__(kBlock) void k_pm_halfsweep(DevParams P, Ws w, int colour, int iter, int slot,
                                                        int restricted) {
  constexpr int G = 2 * R + 1, NG = kWave / G;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int g = lane / G, j = lane - g * G, base = g * G;
  const int dir = blockIdx.y;
  const int W = P.W, H = P.H, Wh = (W + 1) >> 1;
  const long long i = ((long long)xcd_remap(blockIdx.x, gridDim.x) * (kBlock / kWave) + wave) * NG + g;
  bool act = g < NG && i < (long long)Wh * H;
  const int y = act ? (int)(i / Wh) : 0;
  const int x = act ? 2 * (int)(i - (long long)y * Wh) + ((y + colour) & 1) : 0;
  act = act && x < W;
  const int p = y * W + x;
  if (act && restricted) act = w.win[dir][p] < 0;
  unsigned evals = 0;
  if (act) {
    const int label = restricted ? w.hlabel[dir][p] : -1;
    const double* Hp = plane_H(w, label);
    const float lim = 4.0f * (float)(W > H ? W : H);

    // random-search draws of this pixel, computed by the lanes of the group:
    // lane j holds radii k = j, j + G, j + 2G, ... (up to 16 radii)
    constexpr int NH = (16 + G - 1) / G;
    const uint64_t w3 = rng_word3(2, dir, slot, 0);
    int rox[NH], roy[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const int k = j + h * G;
      rox[h] = roy[h] = 0;
      if (k < P.nk) {
        const int Rk = P.R0 >> k;
        uint64_t c[4] = {(uint64_t)p, (uint64_t)k, (uint64_t)iter, w3};
        philox4x64(c, P.seed, 0);
        rox[h] = draw_below(c[0], (uint32_t)(2 * Rk + 1)) - Rk;
        roy[h] = draw_below(c[1], (uint32_t)(2 * Rk + 1)) - Rk;
      }
    }

    LaneCol<R, C, IDENT> L;
    const bool ok = setup_geometry<R, C, IDENT>(L, Hp, x, y, j - R, lim);
    // a non-positive homogeneous coordinate makes every candidate +inf: no update
    if (group_sum<G>(ok ? 0.f : 1.f, base) == 0.f) {
      load_column<R, C, FP16, IDENT>(L, w.feat[dir], W, H, x, y, j - R);
      const void* F2 = w.feat[1 - dir];
      const int32_t* nnf = w.nnf[dir];

      const int32_t v0 = nnf[p];
      int btx = x + off_dx(v0), bty = y + off_dy(v0);
      float bc = w.cost[dir][p];
      auto consider = [&](int tx, int ty) {
        if (tx == btx && ty == bty) return;  // same target: same cost, never strictly better
        const float c = group_sum<G>(column_cost<R, C, FP16, IDENT>(L, F2, W, H, tx, ty, P.gw), base);
        ++evals;
        if (c < bc) {
          bc = c;
          btx = tx;
          bty = ty;
        }
      };
      // propagation: left, right, up, down
      if (x > 0) {
        const int32_t v = nnf[p - 1];
        consider(clampi(x + off_dx(v), 0, W - 1), clampi(y + off_dy(v), 0, H - 1));
      }
      if (x < W - 1) {
        const int32_t v = nnf[p + 1];
        consider(clampi(x + off_dx(v), 0, W - 1), clampi(y + off_dy(v), 0, H - 1));
      }
      if (y > 0) {
        const int32_t v = nnf[p - W];
        consider(clampi(x + off_dx(v), 0, W - 1), clampi(y + off_dy(v), 0, H - 1));
      }
      if (y < H - 1) {
        const int32_t v = nnf[p + W];
        consider(clampi(x + off_dx(v), 0, W - 1), clampi(y + off_dy(v), 0, H - 1));
      }
      // plane candidate: where the region plane sends p, rounded to the grid
      if (restricted && Hp) {
        const double ww = Hp[6] * x + Hp[7] * y + Hp[8];
        if (ww > 0) {
          const double qx = (Hp[0] * x + Hp[1] * y + Hp[2]) / ww;
          const double qy = (Hp[3] * x + Hp[4] * y + Hp[5]) / ww;
          double rx = floor(qx + 0.5), ry = floor(qy + 0.5);
          const double dl = (double)lim;
          rx = rx < -dl ? -dl : (rx > dl ? dl : rx);
          ry = ry < -dl ? -dl : (ry > dl ? dl : ry);
          consider(clampi((int)rx, 0, W - 1), clampi((int)ry, 0, H - 1));
        }
      }
      // random search around the best offset after propagation
      const int cdx = btx - x, cdy = bty - y;
      for (int k = 0; k < P.nk; ++k) {
        const int src = base + (k % G), slot_k = k / G;
        int mx = rox[0], my = roy[0];
#pragma unroll
        for (int h = 1; h < NH; ++h) {
          mx = slot_k == h ? rox[h] : mx;
          my = slot_k == h ? roy[h] : my;
        }
        const int ox = __shfl(mx, src);
        const int oy = __shfl(my, src);
        consider(clampi(x + cdx + ox, 0, W - 1), clampi(y + cdy + oy, 0, H - 1));
      }
      if (j == 0) {
        w.nnf[dir][p] = pack_off(btx - x, bty - y);
        w.cost[dir][p] = bc;
      }
    }
    if (j != 0) evals = 0;
  }
  count_evals(&w.counters[(restricted ? 4 : 0) + dir], evals);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <int R, int C, bool FP16, bool IDENT>
static hipError_t pm_launch(const DevParams& P, const Ws& w, int colour, int iter, int slot, int restricted,
                            hipStream_t s) {
  constexpr int G = 2 * R + 1, NG = kWave / G;
  const long long n = (long long)((P.W + 1) >> 1) * P.H;
  const long long per = (long long)NG * (kBlock / kWave);
  const int nb = (int)((n + per - 1) / per);
  hipLaunchKernelGGL((k_pm_halfsweep<R, C, FP16, IDENT>), dim3(nb, 2), dim3(kBlock), 0, s, P, w, colour, iter, slot,
                     restricted);
  return hipGetLastError();
}

template <int R, int C, bool FP16, bool IDENT>
static hipError_t ec_launch(const DevParams& P, const Ws& w, int mode, hipStream_t s) {
  constexpr int G = 2 * R + 1, NG = kWave / G;
  const long long n = (long long)P.W * P.H;
  const long long per = (long long)NG * (kBlock / kWave);
  const int nb = (int)((n + per - 1) / per);
  hipLaunchKernelGGL((k_eval_cost<R, C, FP16, IDENT>), dim3(nb, 2), dim3(kBlock), 0, s, P, w, mode);
  return hipGetLastError();
}

template <int R, int C, bool FP16>
static hipError_t dispatch_pm(const DevParams& P, const Ws& w, int colour, int iter, int slot, int restricted,
                              hipStream_t s) {
  if (restricted) return pm_launch<R, C, FP16, false>(P, w, colour, iter, slot, restricted, s);
  return pm_launch<R, C, FP16, true>(P, w, colour, iter, slot, restricted, s);
}

template <int R, int C, bool FP16>
static hipError_t dispatch_ec(const DevParams& P, const Ws& w, int mode, hipStream_t s) {
  if (mode == 0) return ec_launch<R, C, FP16, true>(P, w, mode, s);
  return ec_launch<R, C, FP16, false>(P, w, mode, s);
}

#define MSGPM_DISPATCH(FN, ...)                                                       \
  do {                                                                                \
    const bool h = P.fp16 != 0;                                                       \
    switch (P.r * 10 + P.C) {                                                         \
      case 13: return h ? FN<1, 3, true>(__VA_ARGS__) : FN<1, 3, false>(__VA_ARGS__); \
      case 15: return h ? FN<1, 5, true>(__VA_ARGS__) : FN<1, 5, false>(__VA_ARGS__); \
      case 23: return h ? FN<2, 3, true>(__VA_ARGS__) : FN<2, 3, false>(__VA_ARGS__); \
      case 25: return h ? FN<2, 5, true>(__VA_ARGS__) : FN<2, 5, false>(__VA_ARGS__); \
      case 33: return h ? FN<3, 3, true>(__VA_ARGS__) : FN<3, 3, false>(__VA_ARGS__); \
      case 35: return h ? FN<3, 5, true>(__VA_ARGS__) : FN<3, 5, false>(__VA_ARGS__); \
      case 43: return h ? FN<4, 3, true>(__VA_ARGS__) : FN<4, 3, false>(__VA_ARGS__); \
      case 45: return h ? FN<4, 5, true>(__VA_ARGS__) : FN<4, 5, false>(__VA_ARGS__); \
      default: return hipErrorInvalidValue;                                           \
    }                                                                                 \
  } while (0)

hipError_t launch_pm_halfsweep(const DevParams& P, const Ws& w, int colour, int iter, int slot, int restricted,
                               hipStream_t s) {
  MSGPM_DISPATCH(dispatch_pm, P, w, colour, iter, slot, restricted, s);
}

hipError_t launch_eval_cost(const DevParams& P, const Ws& w, int mode, hipStream_t s) {
  MSGPM_DISPATCH(dispatch_ec, P, w, mode, s);
}

}  // namespace msgpm
