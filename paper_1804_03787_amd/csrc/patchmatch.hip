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
// column's source features and tap geometry in registers.  A distorted tap
// needs the horizontal corner pairs of two rows, each fetched as one
// contiguous load (features are stored interleaved per pixel); integral
// geometries (identity, integer translations) fetch one pixel per tap.  Column
// partials are combined across the group in a fixed order, so every lane of the
// group takes the same decisions.  Identity-patch candidates are evaluated in
// batches whose first rows are gathered together, each then finished on its
// own; distorted-patch candidates one at a time; both with exact early
// rejections on partial sums (every schedule takes the decisions of a
// one-at-a-time loop).  Costs are accumulated in FP32; FP16 records are
// widened inside mixed-precision multiply-adds.
//
// PatchMatch (propagation + random search, as used by the paper for its NNF,
// Sec. 3.1) runs as red-black Jacobi half-sweeps: a pixel reads only the other
// colour's offsets, so a half-sweep is order-free.
#include "common.h"

#include <hip/hip_fp16.h>

#pragma clang fp contract(off)

namespace msgpm {

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x3 __attribute__((ext_vector_type(3)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ inline float2 h2f(uint32_t u) { return __half22float2(__builtin_bit_cast(__half2, u)); }
__device__ inline float uf(uint32_t u) { return __uint_as_float(u); }

// Feature buffer of one frame, read through a buffer resource: offsets are
// 32-bit byte offsets (the host rejects frames whose features exceed 2 GiB), so
// an address costs one integer multiply-add instead of 64-bit arithmetic.
struct Feat {
  __amdgpu_buffer_rsrc_t r;
};
template <int C, bool FP16>
__device__ inline Feat feat_buf(const void* F, int W, int H) {
  constexpr int kBytes = FP16 ? (C == 3 ? 8 : 12) : 4 * C;
  // word 3 = 0x00020000: 32-bit data format, as raw dword buffer loads need on gfx9
  return Feat{__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(F), (short)0, (W * H + 1) * kBytes, 0x00020000)};
}

// Feature access.  FP32: C floats per pixel; FP16: C=3 -> 4 halves, C=5 -> 6
// halves per pixel.  load1 reads pixel idx, load2 pixels idx and idx + 1 with
// one contiguous access (the buffer is padded so idx + 1 always exists).
template <int C, bool FP16>
struct Px {
  static constexpr int kBytes = FP16 ? (C == 3 ? 8 : 12) : 4 * C;
  static __device__ inline void load1(Feat F, int idx, float* v) {
    const int o = idx * kBytes;
    if constexpr (!FP16) {
      if constexpr (C == 3) {
        const u32x3 a = __builtin_amdgcn_raw_buffer_load_b96(F.r, o, 0, 0);
        v[0] = uf(a.x); v[1] = uf(a.y); v[2] = uf(a.z);
      } else {
        const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(F.r, o, 0, 0);
        const uint32_t e = __builtin_amdgcn_raw_buffer_load_b32(F.r, o + 16, 0, 0);
        v[0] = uf(a.x); v[1] = uf(a.y); v[2] = uf(a.z); v[3] = uf(a.w); v[4] = uf(e);
      }
    } else {
      if constexpr (C == 3) {
        const u32x2 u = __builtin_amdgcn_raw_buffer_load_b64(F.r, o, 0, 0);
        const float2 a = h2f(u.x), b = h2f(u.y);
        v[0] = a.x; v[1] = a.y; v[2] = b.x;
      } else {
        const u32x3 u = __builtin_amdgcn_raw_buffer_load_b96(F.r, o, 0, 0);
        const float2 a = h2f(u.x), b = h2f(u.y), c = h2f(u.z);
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y; v[4] = c.x;
      }
    }
  }
  // The record of pixel idx as raw words (kWords of them), for tap_sq_raw.
  static constexpr int kWords = kBytes / 4;
  static __device__ inline void raw1(Feat F, int idx, uint32_t* u) { raw1_at(F, idx * kBytes, u); }
  // The same from the record's byte offset o.
  static __device__ inline void raw1_at(Feat F, int o, uint32_t* u) {
    if constexpr (kWords == 5) {
      const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(F.r, o, 0, 0);
      u[0] = a.x; u[1] = a.y; u[2] = a.z; u[3] = a.w;
      u[4] = __builtin_amdgcn_raw_buffer_load_b32(F.r, o + 16, 0, 0);
    } else if constexpr (kWords == 3) {
      const u32x3 a = __builtin_amdgcn_raw_buffer_load_b96(F.r, o, 0, 0);
      u[0] = a.x; u[1] = a.y; u[2] = a.z;
    } else {
      const u32x2 a = __builtin_amdgcn_raw_buffer_load_b64(F.r, o, 0, 0);
      u[0] = a.x; u[1] = a.y;
    }
  }
  // Records of pixels idx and idx + 1 as raw words (2 kWords), one access.
  static __device__ inline void raw2(Feat F, int idx, uint32_t* u) {
    const int o = idx * kBytes;
    if constexpr (kWords == 5) {
      const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(F.r, o, 0, 0);
      const u32x4 b = __builtin_amdgcn_raw_buffer_load_b128(F.r, o + 16, 0, 0);
      const u32x2 c = __builtin_amdgcn_raw_buffer_load_b64(F.r, o + 32, 0, 0);
      u[0] = a.x; u[1] = a.y; u[2] = a.z; u[3] = a.w; u[4] = b.x;
      u[5] = b.y; u[6] = b.z; u[7] = b.w; u[8] = c.x; u[9] = c.y;
    } else if constexpr (kWords == 3) {
      const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(F.r, o, 0, 0);
      const u32x2 b = __builtin_amdgcn_raw_buffer_load_b64(F.r, o + 16, 0, 0);
      u[0] = a.x; u[1] = a.y; u[2] = a.z; u[3] = a.w; u[4] = b.x; u[5] = b.y;
    } else {
      const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(F.r, o, 0, 0);
      u[0] = a.x; u[1] = a.y; u[2] = a.z; u[3] = a.w;
    }
  }
  static __device__ inline void load2(Feat F, int idx, float* v, float* w) {
    const int o = idx * kBytes;
    if constexpr (!FP16) {
      if constexpr (C == 3) {
        const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(F.r, o, 0, 0);
        const u32x2 b = __builtin_amdgcn_raw_buffer_load_b64(F.r, o + 16, 0, 0);
        v[0] = uf(a.x); v[1] = uf(a.y); v[2] = uf(a.z); w[0] = uf(a.w); w[1] = uf(b.x); w[2] = uf(b.y);
      } else {
        const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(F.r, o, 0, 0);
        const u32x4 b = __builtin_amdgcn_raw_buffer_load_b128(F.r, o + 16, 0, 0);
        const u32x2 c = __builtin_amdgcn_raw_buffer_load_b64(F.r, o + 32, 0, 0);
        v[0] = uf(a.x); v[1] = uf(a.y); v[2] = uf(a.z); v[3] = uf(a.w); v[4] = uf(b.x);
        w[0] = uf(b.y); w[1] = uf(b.z); w[2] = uf(b.w); w[3] = uf(c.x); w[4] = uf(c.y);
      }
    } else {
      if constexpr (C == 3) {
        const u32x4 u = __builtin_amdgcn_raw_buffer_load_b128(F.r, o, 0, 0);
        const float2 a = h2f(u.x), b = h2f(u.y), c = h2f(u.z), d = h2f(u.w);
        v[0] = a.x; v[1] = a.y; v[2] = b.x; w[0] = c.x; w[1] = c.y; w[2] = d.x;
      } else {
        const u32x4 u = __builtin_amdgcn_raw_buffer_load_b128(F.r, o, 0, 0);
        const u32x2 t = __builtin_amdgcn_raw_buffer_load_b64(F.r, o + 16, 0, 0);
        const float2 a = h2f(u.x), b = h2f(u.y), c = h2f(u.z), d = h2f(u.w), e = h2f(t.x), f = h2f(t.y);
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y; v[4] = c.x;
        w[0] = d.x; w[1] = d.y; w[2] = e.x; w[3] = e.y; w[4] = f.x;
      }
    }
  }
};

// Per-lane state of one pixel: the lane's patch column of source features and,
// for distorted patches, the tap geometry (integer offset + fraction of
// Delta(d)) of that column, all in registers for every candidate.  FP16
// records keep the column packed (the record's words in the first slots of
// each f1[t]; 27 registers instead of 45 for C = 5), which takes the
// distorted-patch kernel to 4 waves per SIMD without spills.
template <int R, int C, bool IDENT>
struct LaneCol {
  static constexpr int T = 2 * R + 1;
  static constexpr int TG = IDENT ? 1 : T;
  float f1[T][C];
  int dx;
  int o[TG];  // integer part of Delta: x in the low, y in the high 16 bits
  __device__ int ox(int t) const { return (int)(short)(o[t] & 0xffff); }
  __device__ int oy(int t) const { return o[t] >> 16; }
  float fx[TG], fy[TG];
};

// Tap geometry of column dx for plane H at pixel (x, y) (H == nullptr: the
// identity).  Returns false when the homogeneous coordinate is not positive at
// some tap (cost = +inf); sets integral when every fraction of the column is 0.
template <int R, int C, bool IDENT>
__device__ inline bool setup_geometry(LaneCol<R, C, IDENT>& L, const double* H, int x, int y, int dx, float lim,
                                      bool& integral) {
  L.dx = dx;
  integral = true;
  if constexpr (IDENT) {
    return true;
  } else {
    if (H == nullptr) {
#pragma unroll
      for (int t = 0; t < 2 * R + 1; ++t) {
        L.o[t] = pack_off(dx, t - R);
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
      // integer parts beyond +-32767 (frames are at most 32767 pixels) select
      // the same clamped border pixel with fraction 0, so they are cut there
      L.o[t] = pack_off((int)fminf(fmaxf(flx, -32767.f), 32767.f), (int)fminf(fmaxf(fly, -32767.f), 32767.f));
      L.fx[t] = Dx - flx;
      L.fy[t] = Dy - fly;
      integral = integral && (L.fx[t] == 0.f) && (L.fy[t] == 0.f);
    }
    return ok;
  }
}

template <int R, int C, bool FP16, bool IDENT>
__device__ inline void load_column(LaneCol<R, C, IDENT>& L, Feat F1, int W, int H, int x, int y, int dx) {
  const int cx = clampi(x + dx, 0, W - 1);
#pragma unroll
  for (int t = 0; t < 2 * R + 1; ++t) {
    const int cy = clampi(y + t - R, 0, H - 1);
    if constexpr (FP16) {
      // FP16 records stay packed: the column's words in the first slots of
      // f1[t] (bit copies), widened inside the tap arithmetic
      uint32_t u[Px<C, FP16>::kWords];
      Px<C, FP16>::raw1(F1, cy * W + cx, u);
#pragma unroll
      for (int k = 0; k < Px<C, FP16>::kWords; ++k) L.f1[t][k] = __builtin_bit_cast(float, u[k]);
    } else {
      Px<C, FP16>::load1(F1, cy * W + cx, L.f1[t]);
    }
  }
}

template <int C>
__device__ inline float tap_sq(const float* f1, const float* v, float gw) {
  float row = 0.f;
#pragma unroll
  for (int k = 0; k < C; ++k) {
    const float e = f1[k] - v[k];
    row = (k < 3) ? fmaf(e, e, row) : fmaf(gw * e, e, row);
  }
  return row;
}

// f - h for the FP16 value h in the low (HI = false) or high half of u: the
// half is widened exactly and the difference rounded once, as a conversion
// followed by an FP32 subtraction gives, but in one mixed-precision
// multiply-add (h * -1 + f) instead of two instructions.
template <bool HI>
__device__ inline float sub_half(float f, uint32_t u) {
  float e;
  if constexpr (HI)
    asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(e) : "v"(u), "v"(f));
  else
    asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel_hi:[1,0,0]" : "=v"(e) : "v"(u), "v"(f));
  return e;
}

// a - b for FP16 values a (half HA of ua) and b (half HB of ub), both widened
// exactly and the difference rounded once (b * -1 + a).
template <bool HA, bool HB>
__device__ inline float sub_halves(uint32_t ua, uint32_t ub) {
  float e;
  if constexpr (HA && HB)
    asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel:[1,0,1] op_sel_hi:[1,0,1]" : "=v"(e) : "v"(ub), "v"(ua));
  else if constexpr (HA)
    asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel:[0,0,1] op_sel_hi:[1,0,1]" : "=v"(e) : "v"(ub), "v"(ua));
  else if constexpr (HB)
    asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,1]" : "=v"(e) : "v"(ub), "v"(ua));
  else
    asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel_hi:[1,0,1]" : "=v"(e) : "v"(ub), "v"(ua));
  return e;
}

// a - v for the FP16 value a (half HA of ua) and an FP32 v: a widened exactly,
// the difference rounded once (v * -1 + a).
template <bool HA>
__device__ inline float sub_half_f32(uint32_t ua, float v) {
  float e;
  if constexpr (HA)
    asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel:[0,0,1] op_sel_hi:[0,0,1]" : "=v"(e) : "v"(v), "v"(ua));
  else
    asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel_hi:[0,0,1]" : "=v"(e) : "v"(v), "v"(ua));
  return e;
}

// h * w + acc and h * w + 0 for the FP16 value h in the low or high half of u,
// rounded once, with h widened exactly: the values a conversion followed by
// an FP32 multiply-add (or multiply) gives, up to the sign of an exact zero
// product, which no tap cost can tell apart (it only ever reaches a square).
template <bool HI>
__device__ inline float fma_half(uint32_t u, float w, float acc) {
  float r;
  if constexpr (HI)
    asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(u), "v"(w), "v"(acc));
  else
    asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel_hi:[1,0,0]" : "=v"(r) : "v"(u), "v"(w), "v"(acc));
  return r;
}
template <bool HI>
__device__ inline float mul_half(uint32_t u, float w) {
  float r;
  if constexpr (HI)
    asm("v_fma_mix_f32 %0, %1, %2, 0 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(u), "v"(w));
  else
    asm("v_fma_mix_f32 %0, %1, %2, 0 op_sel_hi:[1,0,0]" : "=v"(r) : "v"(u), "v"(w));
  return r;
}

// Channel k of the record whose raw words start at u (FP16: widened).
template <int C, bool FP16>
__device__ inline float chan(const uint32_t* u, int k) {
  if constexpr (FP16) {
    const uint32_t x = u[k >> 1];
    return (float)__builtin_bit_cast(_Float16, (uint16_t)((k & 1) ? (x >> 16) : (x & 0xffffu)));
  } else {
    return uf(u[k]);
  }
}

// tap_sq of a record in its raw words (Px::raw1): the same value.
template <int C, bool FP16>
__device__ inline float tap_sq_raw(const float* f1, const uint32_t* u, float gw) {
  float row = 0.f;
#pragma unroll
  for (int k = 0; k < C; ++k) {
    float e;
    if constexpr (FP16) {
      const uint32_t a = __builtin_bit_cast(uint32_t, f1[k >> 1]);
      e = (k & 1) ? sub_halves<true, true>(a, u[k >> 1]) : sub_halves<false, false>(a, u[k >> 1]);
    } else
      e = f1[k] - uf(u[k]);
    row = (k < 3) ? fmaf(e, e, row) : fmaf(gw * e, e, row);
  }
  return row;
}

// tap_sq with the source record packed (FP16 words, as load_column keeps them)
// and the target values in FP32: the same value as with the source widened first.
template <int C>
__device__ inline float tap_sq_packed(const float* f1, const float* v, float gw) {
  float row = 0.f;
#pragma unroll
  for (int k = 0; k < C; ++k) {
    const uint32_t a = __builtin_bit_cast(uint32_t, f1[k >> 1]);
    const float e = (k & 1) ? sub_half_f32<true>(a, v[k]) : sub_half_f32<false>(a, v[k]);
    row = (k < 3) ? fmaf(e, e, row) : fmaf(gw * e, e, row);
  }
  return row;
}

// G - 1 adds with the wave shifted right by one lane leave at lane l the sum
// ((v[l-G+1] + v[l-G+2]) + ...) + v[l]; at the group's last lane that is the
// group's G column partials in lane order.  Groups never straddle inactive
// lanes: a group is active or inactive as a whole.
template <int G>
__device__ inline float group_chain(float v) {
  float s = v;
#pragma unroll
  for (int k = 1; k < G; ++k) {
    const float sh =
        __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, s), 0x138, 0xf, 0xf, false));
    s = sh + v;
  }
  return s;
}

// Sum of the group's column partials in lane order, identical on every lane
// of the group: group_chain's value at the last lane, broadcast (by lane reads
// for up to nine groups: measured on MI355X, faster than a permute through
// LDS by 0.1 ms per pair with FP32 records and 1.6 ms with FP16 records).
template <int G>
__device__ inline float group_sum(float v, int base) {
  const float s = group_chain<G>(v);
  constexpr int NG = kWave / G;
  if constexpr (NG <= 9) {
    // few groups: read each group's last lane and select, no LDS round trip
    float r = 0.f;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const float t = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, s), g * G + G - 1));
      r = base == g * G ? t : r;
    }
    return r;
  } else {
    return __shfl(s, base + G - 1);
  }
}

// A decision taken at the group's last lane (where group_chain leaves the
// group's sum), handed to every lane of the group through one wave ballot:
// what a comparison of the broadcast sum would give on every lane, without
// the broadcast.  Values compared with such a sum (the running best cost of
// the identity-patch search) then need to be right only at the last lane.
template <int G>
__device__ inline bool group_flag(bool at_last, int base) {
  const unsigned long long m = __ballot(at_last);
  return (m >> (base + G - 1)) & 1ull;
}

__device__ inline const double* plane_H(const Ws& w, int label) {
  return label >= 0 ? w.planes[label].H : nullptr;
}

// Adds each group's count into counter `kind` with one atomic per wave;
// called by every lane of the wave (outside divergent code).  Spread over
// kCounterStripes copies (STRIPED) so that the waves of a launch do not
// serialise on one address, or all on copy 0: measured on MI355X, striping
// speeds the identity-patch and cost kernels (14.2 vs 14.4 ms and 1.4 vs 4.0
// ms per pipeline) while the distorted-patch kernel runs faster with one
// address (40.4 vs 51.3 ms); results are identical either way.
template <bool STRIPED>
__device__ inline void count_evals(unsigned long long* counters, int kind, unsigned v) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) v += __shfl_xor(v, o);
  const int stripe = STRIPED ? (blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave) & (kCounterStripes - 1) : 0;
  if ((threadIdx.x & (kWave - 1)) == 0 && v) atomicAdd(&counters[kind * kCounterStripes + stripe], (unsigned long long)v);
}

// Group-wide geometry status: 0 = usable, fractional taps; 1 = usable, all
// taps integral; 2 = some homogeneous coordinate not positive (cost +inf).
template <int G>
__device__ inline int group_geometry(bool ok, bool integral, int base) {
  const float bad = group_sum<G>(ok ? 0.f : 1.f, base);
  const float frac = group_sum<G>(integral ? 0.f : 1.f, base);
  return bad != 0.f ? 2 : (frac == 0.f ? 1 : 0);
}

// Adds the lane's taps of rows [T0, T1) for target (tx, ty) to acc, in row
// order.  Integral geometry: one pixel per tap.  Otherwise bilinear: the
// corner pairs of the tap's two rows, each one contiguous load.  Rows are
// taken three at a time: all their loads are issued first and a scheduling
// barrier keeps them ahead of the arithmetic, so a wave has the gathers of
// three rows in flight instead of waiting on each row in turn.
template <int R, int C, bool FP16, bool IDENT, bool INTEGRAL, int T0, int T1>
__device__ inline float add_rows(float acc, const LaneCol<R, C, IDENT>& L, Feat F2, int W, int H,
                                 int tx, int ty, float gw) {
  if constexpr (T1 - T0 > 3) {
    acc = add_rows<R, C, FP16, IDENT, INTEGRAL, T0, T0 + 3>(acc, L, F2, W, H, tx, ty, gw);
    return add_rows<R, C, FP16, IDENT, INTEGRAL, T0 + 3, T1>(acc, L, F2, W, H, tx, ty, gw);
  } else if constexpr (IDENT || INTEGRAL) {
    constexpr int N = T1 - T0;
    uint32_t v[N][Px<C, FP16>::kWords];
#pragma unroll
    for (int n = 0; n < N; ++n) {
      const int t = T0 + n;
      int bx, by;
      if constexpr (IDENT) {
        bx = clampi(tx + L.dx, 0, W - 1);
        by = clampi(ty + t - R, 0, H - 1);
      } else {
        bx = clampi(tx + L.ox(t), 0, W - 1);
        by = clampi(ty + L.oy(t), 0, H - 1);
      }
      Px<C, FP16>::raw1(F2, by * W + bx, v[n]);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int n = 0; n < N; ++n) acc += tap_sq_raw<C, FP16>(L.f1[T0 + n], v[n], gw);
    return acc;
  } else {
    constexpr int N = T1 - T0, KW = Px<C, FP16>::kWords;
    uint32_t top[N][2 * KW], bot[N][2 * KW];
    float fx[N], fy[N];
#pragma unroll
    for (int n = 0; n < N; ++n) {
      const int t = T0 + n;
      // base pixel clamped into the frame; a fraction survives only where the
      // base and its right (lower) neighbour are both inside
      const int ux = tx + L.ox(t), uy = ty + L.oy(t);
      const int bx = min(max(ux, 0), W - 1), by = min(max(uy, 0), H - 1);
      fx[n] = (unsigned)ux < (unsigned)(W - 1) ? L.fx[t] : 0.f;
      fy[n] = (unsigned)uy < (unsigned)(H - 1) ? L.fy[t] : 0.f;
      const int i0 = by * W + bx;
      const int i1 = i0 + (by < H - 1 ? W : 0);
      Px<C, FP16>::raw2(F2, i0, top[n]);
      Px<C, FP16>::raw2(F2, i1, bot[n]);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int n = 0; n < N; ++n) {
      const float gx = 1.f - fx[n], gy = 1.f - fy[n];
      const float w00 = gx * gy, w01 = fx[n] * gy, w10 = gx * fy[n], w11 = fx[n] * fy[n];
      float v[C];
#pragma unroll
      for (int k = 0; k < C; ++k) {
        if constexpr (FP16) {
          // corners a, b (top pair) and c, d (bottom pair), widened inside the FMAs
          const int wi = k >> 1;
          if (k & 1)
            v[k] = fma_half<true>(bot[n][KW + wi], w11, fma_half<true>(bot[n][wi], w10,
                   fma_half<true>(top[n][KW + wi], w01, mul_half<true>(top[n][wi], w00))));
          else
            v[k] = fma_half<false>(bot[n][KW + wi], w11, fma_half<false>(bot[n][wi], w10,
                   fma_half<false>(top[n][KW + wi], w01, mul_half<false>(top[n][wi], w00))));
        } else {
          v[k] = fmaf(w11, chan<C, FP16>(bot[n] + KW, k),
                      fmaf(w10, chan<C, FP16>(bot[n], k),
                           fmaf(w01, chan<C, FP16>(top[n] + KW, k), w00 * chan<C, FP16>(top[n], k))));
        }
      }
      if constexpr (FP16)
        acc += tap_sq_packed<C>(L.f1[T0 + n], v, gw);
      else
        acc += tap_sq<C>(L.f1[T0 + n], v, gw);
    }
    return acc;
  }
}

// Group cost of target (tx, ty).  With EE the running group sum is compared
// with `bound` (the current best cost) after the first and second third of the
// rows: every tap adds a non-negative term and FP32 addition is monotone, so a
// prefix >= bound proves the full cost >= bound, and the candidate, which could
// never be strictly better, is dropped (rejected = true).  An accepted
// candidate is summed in the same order as without the checks.  rows returns
// the tap rows computed.
template <int R, int C, bool FP16, bool IDENT, bool INTEGRAL, bool EE>
__device__ inline float group_cost(const LaneCol<R, C, IDENT>& L, Feat F2, int W, int H, int tx,
                                   int ty, float gw, int base, float bound, bool& rejected, unsigned& rows) {
  constexpr int T = 2 * R + 1, T1 = T / 3, T2 = (2 * T) / 3;
  rejected = false;
  if constexpr (!EE) {
    rows += T;
    return group_sum<T>(add_rows<R, C, FP16, IDENT, INTEGRAL, 0, T>(0.f, L, F2, W, H, tx, ty, gw), base);
  } else {
    float acc = add_rows<R, C, FP16, IDENT, INTEGRAL, 0, T1>(0.f, L, F2, W, H, tx, ty, gw);
    rows += T1;
    rejected = true;
    if (group_sum<T>(acc, base) >= bound) return 0.f;
    acc = add_rows<R, C, FP16, IDENT, INTEGRAL, T1, T2>(acc, L, F2, W, H, tx, ty, gw);
    rows += T2 - T1;
    if (group_sum<T>(acc, base) >= bound) return 0.f;
    acc = add_rows<R, C, FP16, IDENT, INTEGRAL, T2, T>(acc, L, F2, W, H, tx, ty, gw);
    rows += T - T2;
    rejected = false;
    return group_sum<T>(acc, base);
  }
}

// ---------------------------------------------------------------------------
// Cost refresh: cost[p] = C(p, p + v_p, H_p) for the selected pixels.
// ---------------------------------------------------------------------------
template <int R, int C, bool FP16, bool IDENT>
__device__ __forceinline__ void eval_cost_body(const DevParams& P, const Ws& w, Blk bk, int mode) {
  constexpr int G = 2 * R + 1, NG = kWave / G;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int g = lane / G, j = lane - g * G, base = g * G;
  const int dir = bk.y;
  const int W = P.W, H = P.H;
  bool act;
  int p;
  int label = -1;
  if (mode == 1) {
    // the unassigned pixels, from the restricted pass's lists (both colours):
    // identity patches over the back lists (no region plane), distorted ones
    // over the front lists; each colour takes its own run of workgroups
    constexpr unsigned per = NG * (kBlock / kWave);
    const unsigned c0 = w.act_count[2 * (2 * dir) + (IDENT ? 1 : 0)];
    const unsigned c1 = w.act_count[2 * (2 * dir + 1) + (IDENT ? 1 : 0)];
    const int nb0 = (int)((c0 + per - 1) / per), nb1 = (int)((c1 + per - 1) / per);
    if (bk.x >= nb0 + nb1) return;
    const int colour = bk.x < nb0 ? 0 : 1;
    const int b = colour ? bk.x - nb0 : bk.x, nb = colour ? nb1 : nb0;
    const unsigned cnt = colour ? c1 : c0;
    const long long i = ((long long)xcd_remap(b, nb) * (kBlock / kWave) + wave) * NG + g;
    act = g < NG && i < (long long)cnt;
    const unsigned cap = (unsigned)((W + 1) >> 1) * (unsigned)H;
    p = act ? w.act[2 * dir + colour][IDENT ? cap - 1u - (unsigned)i : (unsigned)i] : 0;
    label = act && !IDENT ? w.hlabel[dir][p] : -1;
  } else {
    const long long i = ((long long)xcd_remap(bk.x, bk.nx) * (kBlock / kWave) + wave) * NG + g;
    act = g < NG && i < (long long)W * H;
    p = act ? (int)i : 0;
  }
  const int x = p % W, y = p / W;
  if (act && mode == 2) {
    label = w.win[dir][p];
    act = label >= 0;
  }
  unsigned evals = 0;
  if (act) {
    const float lim = 4.0f * (float)(W > H ? W : H);
    LaneCol<R, C, IDENT> L;
    bool integral;
    const bool ok = setup_geometry<R, C, IDENT>(L, plane_H(w, label), x, y, j - R, lim, integral);
    const int geo = group_geometry<G>(ok, integral, base);
    const int32_t v = w.nnf[dir][p];
    float c = __builtin_huge_valf();
    if (geo != 2) {
      load_column<R, C, FP16, IDENT>(L, feat_buf<C, FP16>(w.feat[dir], W, H), W, H, x, y, j - R);
      const int tx = x + off_dx(v), ty = y + off_dy(v);
      bool rejected;
      unsigned rows = 0;
      if (IDENT || geo == 1)
        c = group_cost<R, C, FP16, IDENT, true, false>(L, feat_buf<C, FP16>(w.feat[1 - dir], W, H), W, H, tx, ty, P.gw, base, 0.f, rejected,
                                                       rows);
      else
        c = group_cost<R, C, FP16, IDENT, IDENT, false>(L, feat_buf<C, FP16>(w.feat[1 - dir], W, H), W, H, tx, ty, P.gw, base, 0.f, rejected,
                                                        rows);
    }
    if (j == 0) {
      w.cost[dir][p] = c;
      evals = 1;
    }
  }
  count_evals<true>(w.counters, 2 + dir, evals);
}

template <int R, int C, bool FP16, bool IDENT>
__global__ __launch_bounds__(kBlock) void k_eval_cost(DevParams P, Ws w, int mode) {
  eval_cost_body<R, C, FP16, IDENT>(P, w, blk_here(), mode);
}

template <int R, int C, bool FP16, bool IDENT, bool LOOP>
__global__ __launch_bounds__(kBlock) void kb_eval_cost(const uint8_t* __restrict__ tab, int k, BArgs A) {
  const BatchView V = batch_view(tab, k);
  const PairDesc* __restrict__ pd = V.pd;
  const Item* __restrict__ it = V.it;
  const int n = V.n, total = V.total;
  for_each_item<false, LOOP>(it, n, total, [&](int i, Blk bk) {
    eval_cost_body<R, C, FP16, IDENT>(pd[it[i].pair].P, pd[it[i].pair].w, bk, A.a[0]);
  });
}

// Candidate loops of one pixel: the four neighbours' offsets (left, right, up,
// down), the plane candidate (restricted passes), then random search centred on
// the best offset after those; a candidate replaces the best only if strictly
// better.  Two schedules with identical decisions:
//  * identity patches (short per-candidate chain): candidates in batches of
//    NB; the first third of the rows of the batch is gathered together, then
//    each candidate still in the running is finished on its own, with exact
//    early rejections per lane group;
//  * distorted patches (long chain, register-heavy): one candidate at a time
//    with the exact early rejection of group_cost.

// Byte offsets of the records of an identity-patch target (tx, ty) in a lane's
// column dx: record (clamp(tx + dx), clamp(ty + t - R)) of row t.  The row
// clamp commutes with the multiplication by the row pitch (positive), and a
// clamp commutes with adding the column's offset, so that a row costs one add
// of a wave-uniform term and one three-way median on a per-target base and
// bounds, instead of a clamp, a multiply-add and a multiply.
template <int R, int KB>
struct IdentAddr {
  int base, lo, hi, pitch;
  IdentAddr() = default;
  __device__ inline IdentAddr(int tx, int ty, int dx, int W, int H) {
    pitch = W * KB;
    lo = clampi(tx + dx, 0, W - 1) * KB;
    hi = lo + (H - 1) * pitch;
    base = lo + (ty - R) * pitch;
  }
  __device__ inline int at(int t) const {
    int o;
    asm("v_med3_i32 %0, %1, %2, %3" : "=v"(o) : "v"(base + t * pitch), "v"(lo), "v"(hi));
    return o;
  }
};

// Tap rows per load chunk of identity-patch batches: one (measured on MI355X, two
// or three rows per chunk take the kernel to 256 VGPRs and lose more than the
// longer chunks gain).
constexpr int kIdentRows = 1;
// Rows per step when one identity-patch candidate is finished, with an
// early-rejection check before each step.  Measured on MI355X at 1024x436
// (whole pipeline, r = 4, FP32 records): checks at rows 3 and 6 take 33.1 ms per
// pair, a check at row 3 only 33.9 ms, checks at rows 3, 5 and 7 33.8 ms,
// one at every row 38.2 ms; the batch-wide check this replaced took 37.3 ms.
constexpr int kIdentStep = 3;

// Rows [T0, T) of NB identity-patch targets added to acc, in chunks of
// kIdentRows: each lane walks its column once, and the loads of a chunk (all
// candidates) are issued ahead of its arithmetic.
template <int R, int C, bool FP16, int NB, int T0, int T>
__device__ inline void ident_rows(float* acc, const LaneCol<R, C, true>& L, Feat F2, int W, int H, const int* tx,
                                  const int* ty, float gw) {
  IdentAddr<R, Px<C, FP16>::kBytes> A[NB] = {};
#pragma unroll
  for (int b = 0; b < NB; ++b) A[b] = IdentAddr<R, Px<C, FP16>::kBytes>(tx[b], ty[b], L.dx, W, H);
#pragma unroll
  for (int t0 = T0; t0 < T; t0 += kIdentRows) {
    constexpr int TC = kIdentRows;
    uint32_t v[TC][NB][Px<C, FP16>::kWords];
#pragma unroll
    for (int u = 0; u < TC; ++u)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        if (t0 + u < T) Px<C, FP16>::raw1_at(F2, A[b].at(t0 + u), v[u][b]);
      }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < TC; ++u)
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if (t0 + u < T) acc[b] += tap_sq_raw<C, FP16>(L.f1[t0 + u], v[u][b], gw);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Rows [T0, T) of one identity-patch target added to acc: the loads of all
// rows are issued ahead of their arithmetic.
template <int R, int C, bool FP16, int T0, int T>
__device__ inline float ident_rows1(float acc, const LaneCol<R, C, true>& L, Feat F2, int W, int H, int tx, int ty,
                                    float gw) {
  constexpr int N = T - T0;
  uint32_t v[N][Px<C, FP16>::kWords];
  const IdentAddr<R, Px<C, FP16>::kBytes> A(tx, ty, L.dx, W, H);
#pragma unroll
  for (int n = 0; n < N; ++n) Px<C, FP16>::raw1_at(F2, A.at(T0 + n), v[n]);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int n = 0; n < N; ++n) acc += tap_sq_raw<C, FP16>(L.f1[T0 + n], v[n], gw);
  return acc;
}

// Rows [T0, T) of one identity-patch target in steps of kIdentStep rows, the
// group sum checked against bound before each step: false (and the rows
// computed added to rows) as soon as a partial sum is >= bound; otherwise a =
// the full lane partial and rows += T.
template <int R, int C, bool FP16, int T0>
__device__ inline bool ident_finish(float& a, float acc, const LaneCol<R, C, true>& L, Feat F2, int W, int H,
                                    int tx, int ty, float gw, int base, float bound, unsigned& rows) {
  constexpr int T = 2 * R + 1, T1 = T0 + kIdentStep < T ? T0 + kIdentStep : T;
  acc = ident_rows1<R, C, FP16, T0, T1>(acc, L, F2, W, H, tx, ty, gw);
  if constexpr (T1 == T) {
    a = acc;
    rows += T;
    return true;
  } else {
    if (!group_flag<T>(group_chain<T>(acc) < bound, base)) {
      rows += T1;
      return false;
    }
    return ident_finish<R, C, FP16, T1>(a, acc, L, F2, W, H, tx, ty, gw, base, bound, rows);
  }
}

// One identity-patch batch: NB targets, compared with the best in candidate
// order (a candidate replaces it only if strictly better), with the decisions
// of a one-at-a-time loop.  The first third of the rows of every target is
// gathered together; then each target still in the running is finished on its
// own, unless its partial sum is already >= the current best cost: taps are
// non-negative and FP32 addition is monotone, so its full cost could not be
// strictly lower, and its remaining rows are skipped.  The check is per lane
// group: the lanes of a dropped target sit out its remaining gathers, which
// is where the time goes (the cost of a gather scales with the lanes that
// take part in it).  A finished target is summed in the same order as a lone
// evaluation.  Every comparison is taken at the group's last lane, where the
// lane-order sum forms, and handed to the group by a ballot (group_flag), so
// the running best cost bc is exact at that lane only.  Both record formats
// use this form; with FP16 records (one load per tap) it was 3 % slower than
// gathering all rows of the batch and skipping the checks while the kernel's
// VALU work bound it, and after the per-target row offsets and the ballot
// decisions it is 7 % faster (measured on MI355X, 1024x436).
template <int R, int C, bool FP16, int NB>
__device__ inline void ident_batch(const LaneCol<R, C, true>& L, Feat F2, int W, int H, const int* tx,
                                   const int* ty, const bool* ok, float gw, int base, int& btx, int& bty, float& bc,
                                   unsigned& evals, unsigned& rows) {
  constexpr int T = 2 * R + 1, TE = T / 3;
  bool any = false;
#pragma unroll
  for (int b = 0; b < NB; ++b) any = any || ok[b];
  if (!any) return;
  float acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = 0.f;
  ident_rows<R, C, FP16, NB, 0, TE>(acc, L, F2, W, H, tx, ty, gw);
  float pre[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) pre[b] = group_chain<T>(acc[b]);
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if (!ok[b]) continue;
    ++evals;
    if ((tx[b] == btx && ty[b] == bty) || !group_flag<T>(pre[b] < bc, base)) {
      rows += TE;
      continue;
    }
    float a;
    if (!ident_finish<R, C, FP16, TE>(a, acc[b], L, F2, W, H, tx[b], ty[b], gw, base, bc, rows)) continue;
    const float c = group_chain<T>(a);
    if (group_flag<T>(c < bc, base)) {
      bc = c;
      btx = tx[b];
      bty = ty[b];
    }
  }
}

// Random-search candidates k0 .. k0 + NB - 1 around (x + cdx, y + cdy), as one
// identity-patch batch.
template <int R, int C, bool FP16, int NB>
__device__ inline void random_batch(const LaneCol<R, C, true>& L, const DevParams& P, Feat F2, int x, int y,
                                    int cdx, int cdy, int k0, int base, const int* rox, const int* roy, int& btx,
                                    int& bty, float& bc, unsigned& evals, unsigned& rows) {
  constexpr int G = 2 * R + 1, NH = (16 + G - 1) / G;
  const int W = P.W, H = P.H;
  int tx[NB], ty[NB];
  bool ok[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int kk = k0 + b;
    const int src = base + (kk % G), slot_k = kk / G;
    int mx = rox[0], my = roy[0];
#pragma unroll
    for (int h = 1; h < NH; ++h) {
      mx = slot_k == h ? rox[h] : mx;
      my = slot_k == h ? roy[h] : my;
    }
    tx[b] = clampi(x + cdx + __shfl(mx, src), 0, W - 1);
    ty[b] = clampi(y + cdy + __shfl(my, src), 0, H - 1);
    ok[b] = !(tx[b] == btx && ty[b] == bty);
  }
  ident_batch<R, C, FP16, NB>(L, F2, W, H, tx, ty, ok, P.gw, base, btx, bty, bc, evals, rows);
}

// The last random-search batch, of rest < NB candidates (rest is the same for
// every lane).
template <int R, int C, bool FP16, int N>
__device__ inline void random_rest(int rest, const LaneCol<R, C, true>& L, const DevParams& P, Feat F2, int x, int y,
                                   int cdx, int cdy, int k0, int base, const int* rox, const int* roy, int& btx,
                                   int& bty, float& bc, unsigned& evals, unsigned& rows) {
  if constexpr (N > 0) {
    if (rest == N)
      random_batch<R, C, FP16, N>(L, P, F2, x, y, cdx, cdy, k0, base, rox, roy, btx, bty, bc, evals, rows);
    else
      random_rest<R, C, FP16, N - 1>(rest, L, P, F2, x, y, cdx, cdy, k0, base, rox, roy, btx, bty, bc, evals, rows);
  }
}

template <int R, int C, bool FP16>
__device__ inline void pm_candidates_ident(const LaneCol<R, C, true>& L, const DevParams& P, const Ws& w, int dir,
                                           int x, int y, int base, bool fresh, const int* rox, const int* roy,
                                           unsigned& evals, unsigned& rows) {
  constexpr int NB = 4;
  const int W = P.W, H = P.H, p = y * W + x;
  const Feat F2 = feat_buf<C, FP16>(w.feat[1 - dir], W, H);
  const int32_t* nnf = w.nnf[dir];
  const int32_t v0 = nnf[p];
  int btx = x + off_dx(v0), bty = y + off_dy(v0);
  float bc;
  if (fresh) {
    bool rejected;
    unsigned r0 = 0;
    bc = group_cost<R, C, FP16, true, true, false>(L, F2, W, H, btx, bty, P.gw, base, 0.f, rejected, r0);
  } else {
    bc = w.cost[dir][p];
  }
  {
    int tx[4], ty[4];
    bool ok[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int nx = x + (k == 0 ? -1 : (k == 1 ? 1 : 0));
      const int ny = y + (k == 2 ? -1 : (k == 3 ? 1 : 0));
      const bool inside = nx >= 0 && nx < W && ny >= 0 && ny < H;
      const int32_t v = nnf[clampi(ny, 0, H - 1) * W + clampi(nx, 0, W - 1)];
      tx[k] = clampi(x + off_dx(v), 0, W - 1);
      ty[k] = clampi(y + off_dy(v), 0, H - 1);
      ok[k] = inside && !(tx[k] == btx && ty[k] == bty);
    }
    ident_batch<R, C, FP16, 4>(L, F2, W, H, tx, ty, ok, P.gw, base, btx, bty, bc, evals, rows);
  }
  // random search in full batches, then one batch of the remaining radii (a
  // wave-uniform size, so no slot loads a patch for a radius that is not there)
  const int cdx = btx - x, cdy = bty - y;
  int k0 = 0;
  for (; k0 + NB <= P.nk; k0 += NB)
    random_batch<R, C, FP16, NB>(L, P, F2, x, y, cdx, cdy, k0, base, rox, roy, btx, bty, bc, evals, rows);
  random_rest<R, C, FP16, NB - 1>(P.nk - k0, L, P, F2, x, y, cdx, cdy, k0, base, rox, roy, btx, bty, bc, evals,
                                  rows);
  // the running best cost is exact at the group's last lane (group_flag)
  if (base + 2 * R == (int)(threadIdx.x & (kWave - 1))) {
    w.nnf[dir][p] = pack_off(btx - x, bty - y);
    w.cost[dir][p] = bc;
  }
}

template <int R, int C, bool FP16, bool IDENT, bool INTEGRAL>
__device__ inline void pm_candidates_serial(const LaneCol<R, C, IDENT>& L, const DevParams& P, const Ws& w, int dir, int x,
                                     int y, int base, bool fresh, bool has_plane, int ptx, int pty, const int* rox,
                                     const int* roy, unsigned& evals, unsigned& rows) {
  constexpr int G = 2 * R + 1, NH = (16 + G - 1) / G;
  constexpr bool EE = true;
  const int W = P.W, H = P.H, p = y * W + x;
  const Feat F2 = feat_buf<C, FP16>(w.feat[1 - dir], W, H);
  const int32_t* nnf = w.nnf[dir];
  const int32_t v0 = nnf[p];
  int btx = x + off_dx(v0), bty = y + off_dy(v0);
  float bc;
  if (fresh) {
    bool rejected;
    unsigned r0 = 0;
    bc = group_cost<R, C, FP16, IDENT, INTEGRAL, false>(L, F2, W, H, btx, bty, P.gw, base, 0.f, rejected, r0);
  } else {
    bc = w.cost[dir][p];
  }
  int cdx = 0, cdy = 0;
  for (int k = 0; k < 5 + P.nk; ++k) {
    int tx, ty;
    if (k < 4) {
      const int nx = x + (k == 0 ? -1 : (k == 1 ? 1 : 0));
      const int ny = y + (k == 2 ? -1 : (k == 3 ? 1 : 0));
      if (nx < 0 || nx >= W || ny < 0 || ny >= H) continue;
      const int32_t v = nnf[ny * W + nx];
      tx = clampi(x + off_dx(v), 0, W - 1);
      ty = clampi(y + off_dy(v), 0, H - 1);
    } else if (k == 4) {
      if (!has_plane) continue;
      tx = ptx;
      ty = pty;
    } else {
      if (k == 5) {
        cdx = btx - x;
        cdy = bty - y;
      }
      const int kk = k - 5;
      const int src = base + (kk % G), slot_k = kk / G;
      int mx = rox[0], my = roy[0];
#pragma unroll
      for (int h = 1; h < NH; ++h) {
        mx = slot_k == h ? rox[h] : mx;
        my = slot_k == h ? roy[h] : my;
      }
      tx = clampi(x + cdx + __shfl(mx, src), 0, W - 1);
      ty = clampi(y + cdy + __shfl(my, src), 0, H - 1);
    }
    if (tx == btx && ty == bty) continue;  // same target: same cost, never strictly better
    bool rejected;
    const float c = group_cost<R, C, FP16, IDENT, INTEGRAL, EE>(L, F2, W, H, tx, ty, P.gw, base, bc, rejected, rows);
    ++evals;
    if (!rejected && c < bc) {
      bc = c;
      btx = tx;
      bty = ty;
    }
  }
  if (base == (int)(threadIdx.x & (kWave - 1))) {
    w.nnf[dir][p] = pack_off(btx - x, bty - y);
    w.cost[dir][p] = bc;
  }
}

// ---------------------------------------------------------------------------
// Restricted half-sweeps update only the unassigned pixels of one colour.
// They are listed first, so that every lane group of the sweep has a pixel,
// in two lists sharing one buffer per direction: pixels with a region plane
// from the front (distorted patches), pixels without one from the back
// (identity patches: the update of the initial pass, without a plane
// candidate).  Each workgroup appends the pixels of its span (row-major) at
// positions taken from the two counters; the order of the spans varies between
// runs, and the update of a pixel does not depend on it.
// ---------------------------------------------------------------------------
__global__ void k_zero_active(Ws w) {
  if (threadIdx.x < 8) w.act_count[threadIdx.x] = 0u;
}

// batched: each workgroup takes items blockIdx.x, blockIdx.x + gridDim.x, ...
__global__ void kb_zero_active(const uint8_t* __restrict__ tab, int k) {
  const BatchView V = batch_view(tab, k);
  for (int i = blockIdx.x; i < V.n; i += gridDim.x)
    if (threadIdx.x < 8) V.pd[V.it[i].pair].w.act_count[threadIdx.x] = 0u;
}

constexpr int kListSpan = 4;  // pixels of the colour per thread of k_active_list

__device__ __forceinline__ void active_list_body(const DevParams& P, const Ws& w, Blk bk, int colour) {
  constexpr int NS = kListSpan * (kBlock / kWave);
  __shared__ int s_cnt[2][NS];
  __shared__ unsigned s_base[2];
  const int dir = bk.y;
  const int W = P.W, H = P.H, Wh = (W + 1) >> 1;
  const unsigned cap = (unsigned)Wh * (unsigned)H;
  const int t = threadIdx.x, lane = t & (kWave - 1), wave = t / kWave;
  int pix[kListSpan];
  bool inA[kListSpan], inB[kListSpan];
  unsigned long long mA[kListSpan], mB[kListSpan];
#pragma unroll
  for (int k = 0; k < kListSpan; ++k) {
    const long long i = ((long long)bk.x * kListSpan + k) * kBlock + t;
    bool act = i < (long long)cap;
    pix[k] = 0;
    bool plane = false;
    if (act) {
      const int y = (int)(i / Wh);
      const int x = 2 * (int)(i - (long long)y * Wh) + ((y + colour) & 1);
      pix[k] = y * W + x;
      act = x < W && w.win[dir][pix[k]] < 0;
      plane = act && w.hlabel[dir][pix[k]] >= 0;
    }
    inA[k] = plane;
    inB[k] = act && !plane;
    mA[k] = __ballot(inA[k]);
    mB[k] = __ballot(inB[k]);
    if (lane == 0) {
      s_cnt[0][k * (kBlock / kWave) + wave] = __popcll(mA[k]);
      s_cnt[1][k * (kBlock / kWave) + wave] = __popcll(mB[k]);
    }
  }
  __syncthreads();
  if (t < 2) {
    unsigned total = 0u;
    for (int k = 0; k < NS; ++k) total += s_cnt[t][k];
    s_base[t] = total ? atomicAdd(&w.act_count[2 * (2 * dir + colour) + t], total) : 0u;
  }
  __syncthreads();
  unsigned posA = s_base[0], posB = s_base[1];
  int done = 0;
  const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
  for (int k = 0; k < kListSpan; ++k) {
    const int mine = k * (kBlock / kWave) + wave;
    for (; done < mine; ++done) {
      posA += s_cnt[0][done];
      posB += s_cnt[1][done];
    }
    int32_t* list = w.act[2 * dir + colour];
    if (inA[k]) list[posA + __popcll(mA[k] & lt)] = pix[k];
    if (inB[k]) list[cap - 1u - (posB + __popcll(mB[k] & lt))] = pix[k];
  }
}

__global__ __launch_bounds__(kBlock) void k_active_list(DevParams P, Ws w, int colour) {
  active_list_body(P, w, blk_here(), colour);
}

__global__ __launch_bounds__(kBlock) void kb_active_list(const uint8_t* __restrict__ tab, int k, BArgs A) {
  const BatchView V = batch_view(tab, k);
  const PairDesc* __restrict__ pd = V.pd;
  const Item* __restrict__ it = V.it;
  const int n = V.n, total = V.total;
  for_each_item<true>(it, n, total, [&](int i, Blk bk) {
    active_list_body(pd[it[i].pair].P, pd[it[i].pair].w, bk, A.a[0]);
  });
}

// ---------------------------------------------------------------------------
// One red-black half-sweep over the pixels of one colour, both directions
// (restricted: over the listed pixels).
// ---------------------------------------------------------------------------
// The distorted-patch form is held to 168 VGPRs (3 waves per SIMD): on MI355X
// the extra wave hides more gather latency than the few registers it costs.
// mode bit 0: restricted; bit 1 (fresh): the pixel's current cost is computed
// first, as the cost refresh of that pass computes it, instead of being read,
// so that the first half-sweep of each colour stands in for the refresh.
template <int R, int C, bool FP16, bool IDENT>
__device__ __forceinline__ void pm_halfsweep_body(const DevParams& P, const Ws& w, Blk bk, int colour, int iter,
                                                  int slot, int mode) {
  constexpr int G = 2 * R + 1, NG = kWave / G;
  const int restricted = mode & 1;
  const bool fresh = (mode & 2) != 0;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int g = lane / G, j = lane - g * G, base = g * G;
  const int dir = bk.y;
  const int W = P.W, H = P.H, Wh = (W + 1) >> 1;
  bool act;
  int x, y;
  if (restricted) {
    // only the workgroups covering the list work; each XCD takes a contiguous
    // part.  Distorted patches: the front list; identity patches: the back one.
    const unsigned cnt = w.act_count[2 * (2 * dir + colour) + (IDENT ? 1 : 0)];
    constexpr unsigned per = NG * (kBlock / kWave);
    const int nb = (int)((cnt + per - 1) / per);
    if (bk.x >= nb) return;
    const long long i = ((long long)xcd_remap(bk.x, nb) * (kBlock / kWave) + wave) * NG + g;
    act = g < NG && i < (long long)cnt;
    const unsigned cap = (unsigned)Wh * (unsigned)H;
    const int q = act ? w.act[2 * dir + colour][IDENT ? cap - 1u - (unsigned)i : (unsigned)i] : 0;
    y = q / W;
    x = q - y * W;
  } else {
    const long long i = ((long long)xcd_remap(bk.x, bk.nx) * (kBlock / kWave) + wave) * NG + g;
    act = g < NG && i < (long long)Wh * H;
    y = act ? (int)(i / Wh) : 0;
    x = act ? 2 * (int)(i - (long long)y * Wh) + ((y + colour) & 1) : 0;
    act = act && x < W;
  }
  const int p = y * W + x;
  unsigned evals = 0, rows = 0, refreshed = 0;
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
        uint64_t c[4] = {(uint64_t)(uint32_t)p, (uint64_t)k, (uint64_t)iter, w3};
        philox4x64(c, P.seed, 0);
        rox[h] = draw_below(c[0], (uint32_t)(2 * Rk + 1)) - Rk;
        roy[h] = draw_below(c[1], (uint32_t)(2 * Rk + 1)) - Rk;
      }
    }

    LaneCol<R, C, IDENT> L;
    bool integral;
    const bool ok = setup_geometry<R, C, IDENT>(L, Hp, x, y, j - R, lim, integral);
    const int geo = group_geometry<G>(ok, integral, base);
    // a non-positive homogeneous coordinate makes every candidate +inf: no update
    if (geo != 2) {
      load_column<R, C, FP16, IDENT>(L, feat_buf<C, FP16>(w.feat[dir], W, H), W, H, x, y, j - R);
      // plane candidate: where the region plane sends p, rounded to the grid
      bool has_plane = false;
      int ptx = 0, pty = 0;
      if (restricted && Hp) {
        const double ww = Hp[6] * x + Hp[7] * y + Hp[8];
        if (ww > 0) {
          const double qx = (Hp[0] * x + Hp[1] * y + Hp[2]) / ww;
          const double qy = (Hp[3] * x + Hp[4] * y + Hp[5]) / ww;
          double rx = floor(qx + 0.5), ry = floor(qy + 0.5);
          const double dl = (double)lim;
          rx = rx < -dl ? -dl : (rx > dl ? dl : rx);
          ry = ry < -dl ? -dl : (ry > dl ? dl : ry);
          ptx = clampi((int)rx, 0, W - 1);
          pty = clampi((int)ry, 0, H - 1);
          has_plane = true;
        }
      }
      if constexpr (IDENT)
        pm_candidates_ident<R, C, FP16>(L, P, w, dir, x, y, base, fresh, rox, roy, evals, rows);
      else if (geo == 1)
        pm_candidates_serial<R, C, FP16, IDENT, true>(L, P, w, dir, x, y, base, fresh, has_plane, ptx, pty, rox, roy,
                                                      evals, rows);
      else
        pm_candidates_serial<R, C, FP16, IDENT, false>(L, P, w, dir, x, y, base, fresh, has_plane, ptx, pty, rox,
                                                       roy, evals, rows);
    } else if (fresh && j == 0) {
      w.cost[dir][p] = __builtin_huge_valf();
    }
    if (j != 0) evals = rows = 0;
    refreshed = fresh && j == 0 ? 1 : 0;
  }
  count_evals<IDENT>(w.counters, (restricted ? (IDENT ? 10 : 4) : 0) + dir, evals);
  count_evals<IDENT>(w.counters, (restricted ? (IDENT ? 12 : 8) : 6) + dir, rows);
  if (fresh) count_evals<IDENT>(w.counters, 2 + dir, refreshed);
}

template <int R, int C, bool FP16, bool IDENT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(IDENT ? 4 : 3))) void k_pm_halfsweep(
    DevParams P, Ws w, int colour, int iter, int slot, int mode) {
  pm_halfsweep_body<R, C, FP16, IDENT>(P, w, blk_here(), colour, iter, slot, mode);
}

template <int R, int C, bool FP16, bool IDENT, bool LOOP>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(IDENT ? 4 : 3))) void kb_pm_halfsweep(
    const uint8_t* __restrict__ tab, int k, BArgs A) {
  const BatchView V = batch_view(tab, k);
  const PairDesc* __restrict__ pd = V.pd;
  const Item* __restrict__ it = V.it;
  const int n = V.n, total = V.total;
  for_each_item<false, LOOP>(it, n, total, [&](int i, Blk bk) {
    const Item& I = it[i];
    pm_halfsweep_body<R, C, FP16, IDENT>(pd[I.pair].P, pd[I.pair].w, bk, A.a[0], A.a[1], A.a[2], A.a[3]);
  });
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <int R, int C, bool FP16, bool IDENT>
static hipError_t pm_launch(const DevParams& P, const Ws& w, int colour, int iter, int slot, int mode,
                            hipStream_t s) {
  constexpr int G = 2 * R + 1, NG = kWave / G;
  const long long n = (long long)((P.W + 1) >> 1) * P.H;
  const long long per = (long long)NG * (kBlock / kWave);
  const int nb = (int)((n + per - 1) / per);
  hipLaunchKernelGGL((k_pm_halfsweep<R, C, FP16, IDENT>), dim3(nb, 2), dim3(kBlock), 0, s, P, w, colour, iter, slot,
                     mode);
  return hipGetLastError();
}

// Restricted half-sweep over the lists of launch_pm_lists: the distorted-patch
// kernel over the front list or the identity-patch kernel over the back one
// (both read only the other colour, so their order does not matter).
template <int R, int C, bool FP16>
static hipError_t dispatch_restricted(const DevParams& P, const Ws& w, int colour, int iter, int slot, int ident,
                                      int fresh, hipStream_t s) {
  const int mode = 1 | (fresh ? 2 : 0);
  if (ident) return pm_launch<R, C, FP16, true>(P, w, colour, iter, slot, mode, s);
  return pm_launch<R, C, FP16, false>(P, w, colour, iter, slot, mode, s);
}

// The lists of both colours; they hold for every half-sweep of a restricted
// pass (assignment and region planes do not change during it).
hipError_t launch_pm_lists(const DevParams& P, const Ws& w, hipStream_t s) {
  const long long n = (long long)((P.W + 1) >> 1) * P.H;
  hipLaunchKernelGGL(k_zero_active, dim3(1), dim3(kWave), 0, s, w);
  hipError_t e = hipGetLastError();
  const long long span = (long long)kListSpan * kBlock;
  for (int colour = 0; colour < 2 && e == hipSuccess; ++colour) {
    hipLaunchKernelGGL(k_active_list, dim3((unsigned)((n + span - 1) / span), 2), dim3(kBlock), 0, s, P, w, colour);
    e = hipGetLastError();
  }
  return e;
}

template <int R, int C, bool FP16, bool IDENT>
static hipError_t ec_launch(const DevParams& P, const Ws& w, int mode, hipStream_t s) {
  constexpr int G = 2 * R + 1, NG = kWave / G;
  const long long n = (long long)P.W * P.H, half = (long long)((P.W + 1) >> 1) * P.H;
  const long long per = (long long)NG * (kBlock / kWave);
  const int nb = mode == 1 ? (int)(2 * ((half + per - 1) / per)) : (int)((n + per - 1) / per);
  hipLaunchKernelGGL((k_eval_cost<R, C, FP16, IDENT>), dim3(nb, 2), dim3(kBlock), 0, s, P, w, mode);
  return hipGetLastError();
}

template <int R, int C, bool FP16>
static hipError_t dispatch_pm(const DevParams& P, const Ws& w, int colour, int iter, int slot, int fresh,
                              hipStream_t s) {
  return pm_launch<R, C, FP16, true>(P, w, colour, iter, slot, fresh ? 2 : 0, s);
}

template <int R, int C, bool FP16>
static hipError_t dispatch_ec(const DevParams& P, const Ws& w, int mode, hipStream_t s) {
  if (mode == 0) return ec_launch<R, C, FP16, true>(P, w, mode, s);
  if (mode == 1) {
    hipError_t e = ec_launch<R, C, FP16, true>(P, w, mode, s);
    if (e != hipSuccess) return e;
  }
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

hipError_t launch_pm_halfsweep(const DevParams& P, const Ws& w, int colour, int iter, int slot, int fresh,
                               hipStream_t s) {
  MSGPM_DISPATCH(dispatch_pm, P, w, colour, iter, slot, fresh, s);
}

hipError_t launch_pm_restricted(const DevParams& P, const Ws& w, int colour, int iter, int slot, int ident,
                                int fresh, hipStream_t s) {
  MSGPM_DISPATCH(dispatch_restricted, P, w, colour, iter, slot, ident, fresh, s);
}

hipError_t launch_eval_cost(const DevParams& P, const Ws& w, int mode, hipStream_t s) {
  MSGPM_DISPATCH(dispatch_ec, P, w, mode, s);
}

template <int R, int C, bool FP16, bool LOOP>
static void dispatch_batched_form(int kind, const uint8_t* tab, int k, dim3 grid, BArgs A, hipStream_t s) {
  const dim3 block(kBlock);
  switch (kind) {
    case BK_PM_INIT:
    case BK_PM_RESTRICTED_IDENT:
      hipLaunchKernelGGL((kb_pm_halfsweep<R, C, FP16, true, LOOP>), grid, block, 0, s, tab, k, A);
      break;
    case BK_PM_RESTRICTED:
      hipLaunchKernelGGL((kb_pm_halfsweep<R, C, FP16, false, LOOP>), grid, block, 0, s, tab, k, A);
      break;
    case BK_EVAL_COST_IDENT:
      hipLaunchKernelGGL((kb_eval_cost<R, C, FP16, true, LOOP>), grid, block, 0, s, tab, k, A);
      break;
    default:
      hipLaunchKernelGGL((kb_eval_cost<R, C, FP16, false, LOOP>), grid, block, 0, s, tab, k, A);
      break;
  }
}

// persistent (loop over the virtual workgroups) or one-shot (grid >= total)
template <int R, int C, bool FP16>
static hipError_t dispatch_batched(int kind, const uint8_t* tab, int k, int ngrid, BArgs A, bool persist,
                                   hipStream_t s) {
  if (kind != BK_PM_INIT && kind != BK_PM_RESTRICTED_IDENT && kind != BK_PM_RESTRICTED &&
      kind != BK_EVAL_COST_IDENT && kind != BK_EVAL_COST_PLANE)
    return hipErrorInvalidValue;
  if (persist)
    dispatch_batched_form<R, C, FP16, true>(kind, tab, k, dim3(ngrid, 2), A, s);
  else
    dispatch_batched_form<R, C, FP16, false>(kind, tab, k, dim3(ngrid, 2), A, s);
  return hipGetLastError();
}

hipError_t launch_batched_pm(int kind, const DevParams& P0, const uint8_t* tab, int k, int grid, BArgs A,
                             bool persist, hipStream_t s) {
  if (kind == BK_ZERO_ACTIVE) {
    hipLaunchKernelGGL(kb_zero_active, dim3(grid), dim3(kWave), 0, s, tab, k);
    return hipGetLastError();
  }
  if (kind == BK_ACTIVE_LIST) {
    hipLaunchKernelGGL(kb_active_list, dim3(grid, 2), dim3(kBlock), 0, s, tab, k, A);
    return hipGetLastError();
  }
  const DevParams& P = P0;
  MSGPM_DISPATCH(dispatch_batched, kind, tab, k, grid, A, persist, s);
}

// Workgroups of the PatchMatch-side kernels for one pair (the single-pair
// launchers' grids).
int pm_batch_blocks(int kind, const DevParams& P, const int* a) {
  const int G = 2 * P.r + 1, NG = kWave / G, per = NG * (kBlock / kWave);
  const long long half = (long long)((P.W + 1) >> 1) * P.H;
  switch (kind) {
    case BK_EVAL_COST_IDENT:
    case BK_EVAL_COST_PLANE:
      if (a && a[0] == 1) return (int)(2 * ((half + per - 1) / per));  // both colours' lists
      return (int)(((long long)P.W * P.H + per - 1) / per);
    case BK_ZERO_ACTIVE:
      return 1;
    case BK_ACTIVE_LIST: {
      const long long span = (long long)kListSpan * kBlock;
      return (int)((half + span - 1) / span);
    }
    default:
      return (int)((half + per - 1) / per);
  }
}

// ---------------------------------------------------------------------------
// Self-check of the mixed-precision helpers of the FP16 records against
// widening first: thread i takes a word whose low half is FP16 pattern i (all
// 65536 patterns over the grid) and whose high half is another pattern, and
// compares every helper with the plain conversion-then-FP32 arithmetic for
// `rounds` partner words and FP32 operands drawn by an integer hash.  Results
// differ only where both are NaN (payloads are not compared).
// ---------------------------------------------------------------------------
__device__ inline uint32_t check_mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

__device__ inline float widen(uint32_t u, bool hi) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)(hi ? (u >> 16) : (u & 0xffffu)));
}

__device__ inline unsigned differs(float a, float b) {
  return (__float_as_uint(a) != __float_as_uint(b) && !(a != a && b != b)) ? 1u : 0u;
}

__global__ __launch_bounds__(kBlock) void k_check_fp16_arith(int rounds, unsigned long long* out) {
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  const uint32_t ua = (i & 0xffffu) | ((check_mix32(i) & 0xffffu) << 16);
  unsigned bad = 0;
  for (int j = 0; j < rounds; ++j) {
    const uint32_t ub = check_mix32(i * 131u + (uint32_t)j * 2654435761u);
    const uint32_t r = check_mix32(ub ^ 0x9e3779b9u);
    // FP32 operands over many magnitudes: a 24-bit mantissa scaled by 2^(e - 24)
    const float f = ldexpf((float)(int)(r & 0xffffffu) - 8388608.f, (int)((r >> 24) & 31u) - 36);
    const float w = ldexpf((float)(int)(check_mix32(r) & 0xffffffu) - 8388608.f, -23);
    const float a0 = widen(ua, false), a1 = widen(ua, true), b0 = widen(ub, false), b1 = widen(ub, true);
    bad += differs(sub_half<false>(f, ua), f - a0) + differs(sub_half<true>(f, ua), f - a1);
    bad += differs(sub_halves<false, false>(ua, ub), a0 - b0) + differs(sub_halves<true, true>(ua, ub), a1 - b1);
    bad += differs(sub_halves<true, false>(ua, ub), a1 - b0) + differs(sub_halves<false, true>(ua, ub), a0 - b1);
    bad += differs(sub_half_f32<false>(ua, f), a0 - f) + differs(sub_half_f32<true>(ua, f), a1 - f);
    bad += differs(fma_half<false>(ua, w, f), fmaf(a0, w, f)) + differs(fma_half<true>(ua, w, f), fmaf(a1, w, f));
    bad += differs(mul_half<false>(ua, w), a0 * w + 0.f) + differs(mul_half<true>(ua, w), a1 * w + 0.f);
  }
  if (bad) atomicAdd(out, (unsigned long long)bad);
}

__global__ void k_check_clear(unsigned long long* out) {
  if (threadIdx.x == 0) *out = 0ull;
}

hipError_t launch_check_fp16_arith(int rounds, unsigned long long* out, hipStream_t s) {
  hipLaunchKernelGGL(k_check_clear, dim3(1), dim3(64), 0, s, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_check_fp16_arith, dim3(65536 / kBlock), dim3(kBlock), 0, s, rounds, out);
  return hipGetLastError();
}

}  // namespace msgpm
