// Gather ceiling of the PatchMatch kernels' access pattern (a measurement
// kernel for the benchmark, not part of the solver).
//
// The PatchMatch half-sweep kernels spend their time gathering patch rows of
// the other frame's features at candidate targets that are scattered over the
// frame; their arithmetic per tap is small.  This kernel performs the same
// gathers with none of the arithmetic: lanes grouped per pixel as in the
// solver (2r+1 adjacent lanes, lane j owning patch column j - r), each group
// gathering the (2r+1)^2-tap patches of one pixel's candidate stream, the
// four neighbour propagations near the pixel plus one target per random-search
// radius R0 >> k.  The loaded words are folded with XOR (one integer
// operation per word) into one word per lane, written out so that no load can
// be dropped.  Its rate, in patches per second, is the ceiling the solver's
// kernels are compared with: what the memory pipeline delivers for this
// pattern on this layout when nothing else runs.
//
//   identity (bilinear = 0): one record per tap, as the identity-patch kernel;
//   bilinear (bilinear = 1): two records of the tap's row and two of the row
//   below per tap, as the distorted-patch kernel (the row pitch is a run-time
//   value, so the lower pair is a load of its own, as in the solver).
#include <hip/hip_runtime.h>

#include <cstdint>

namespace msgpm_ceiling {

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x3 __attribute__((ext_vector_type(3)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;
constexpr int kBlock = 256;

__device__ inline uint32_t mix32(uint32_t x) {
  // integer finaliser (multiply-xorshift), used only to scatter targets
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

__device__ inline int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// One record (WORDS 32-bit words) at byte offset o, folded into acc.
template <int WORDS>
__device__ inline uint32_t fold1(__amdgpu_buffer_rsrc_t F, int o, uint32_t acc) {
  if constexpr (WORDS == 5) {
    const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(F, o, 0, 0);
    const uint32_t e = __builtin_amdgcn_raw_buffer_load_b32(F, o + 16, 0, 0);
    return acc ^ a.x ^ a.y ^ a.z ^ a.w ^ e;
  } else if constexpr (WORDS == 3) {
    const u32x3 a = __builtin_amdgcn_raw_buffer_load_b96(F, o, 0, 0);
    return acc ^ a.x ^ a.y ^ a.z;
  } else {
    const u32x2 a = __builtin_amdgcn_raw_buffer_load_b64(F, o, 0, 0);
    return acc ^ a.x ^ a.y;
  }
}

// Two adjacent records (2 WORDS words) at byte offset o, folded into acc.
template <int WORDS>
__device__ inline uint32_t fold2(__amdgpu_buffer_rsrc_t F, int o, uint32_t acc) {
  if constexpr (WORDS == 5) {
    const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(F, o, 0, 0);
    const u32x4 b = __builtin_amdgcn_raw_buffer_load_b128(F, o + 16, 0, 0);
    const u32x2 c = __builtin_amdgcn_raw_buffer_load_b64(F, o + 32, 0, 0);
    return acc ^ a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w ^ c.x ^ c.y;
  } else if constexpr (WORDS == 3) {
    const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(F, o, 0, 0);
    const u32x2 b = __builtin_amdgcn_raw_buffer_load_b64(F, o + 16, 0, 0);
    return acc ^ a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y;
  } else {
    const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(F, o, 0, 0);
    return acc ^ a.x ^ a.y ^ a.z ^ a.w;
  }
}

// Grid: one group per pixel of a W x H frame's one colour (as a half-sweep),
// kWave / (2R+1) groups per wave.  Each group gathers `patches` patches of the
// pixel's candidate stream; rows are issued three at a time, as the solver does.
template <int R, int WORDS, bool BILINEAR>
__global__ __launch_bounds__(kBlock) void k_gather(const void* feat, int W, int H, int pitch, int patches,
                                                   uint32_t seed, uint32_t* sink) {
  constexpr int G = 2 * R + 1, NG = kWave / G, T = 2 * R + 1;
  constexpr int kBytes = WORDS * 4;
  const __amdgpu_buffer_rsrc_t F =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(feat), (short)0, (W * H + 1) * kBytes, 0x00020000);
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int g = lane / G, j = lane - g * G;
  const long long i = ((long long)blockIdx.x * (kBlock / kWave) + wave) * NG + g;
  const int Wh = (W + 1) >> 1;
  uint32_t acc = 0u;
  if (g < NG && i < (long long)Wh * H) {
    const int y = (int)(i / Wh);
    const int x = min(2 * (int)(i - (long long)y * Wh) + (y & 1), W - 1);
    const int R0 = W > H ? W : H;
    for (int k = 0; k < patches; ++k) {
      const uint32_t h = mix32(seed ^ mix32((uint32_t)i * 2654435761u + (uint32_t)k));
      const int rad = k < 4 ? 1 : max(R0 >> min(k - 4, 30), 1);
      const int tx = clampi(x + (int)(h % (uint32_t)(2 * rad + 1)) - rad, 0, W - 1);
      const int ty = clampi(y + (int)((h >> 16) % (uint32_t)(2 * rad + 1)) - rad, 0, H - 1);
      const int bx = clampi(tx + j - R, 0, W - 1);
#pragma unroll
      for (int t0 = 0; t0 < T; t0 += 3) {
        uint32_t part = 0u;
#pragma unroll
        for (int t = t0; t < t0 + 3 && t < T; ++t) {
          const int by = clampi(ty + t - R, 0, H - 1);
          const int o = (by * W + bx) * kBytes;
          if constexpr (BILINEAR) {
            part = fold2<WORDS>(F, o, part);
            part = fold2<WORDS>(F, o + (by < H - 1 ? pitch : 0), part);
          } else {
            part = fold1<WORDS>(F, o, part);
          }
        }
        acc ^= part;
      }
    }
  }
  sink[(size_t)blockIdx.x * kBlock + threadIdx.x] = acc;
}

template <int R>
static hipError_t launch_r(const void* feat, int W, int H, int words, int bilinear, int patches, uint32_t seed,
                           uint32_t* sink, int nb, hipStream_t s) {
  const int pitch = W * words * 4;
  const dim3 grid(nb), block(kBlock);
  switch (words * 2 + (bilinear ? 1 : 0)) {
    case 10: hipLaunchKernelGGL((k_gather<R, 5, false>), grid, block, 0, s, feat, W, H, pitch, patches, seed, sink); break;
    case 11: hipLaunchKernelGGL((k_gather<R, 5, true>), grid, block, 0, s, feat, W, H, pitch, patches, seed, sink); break;
    case 6: hipLaunchKernelGGL((k_gather<R, 3, false>), grid, block, 0, s, feat, W, H, pitch, patches, seed, sink); break;
    case 7: hipLaunchKernelGGL((k_gather<R, 3, true>), grid, block, 0, s, feat, W, H, pitch, patches, seed, sink); break;
    case 4: hipLaunchKernelGGL((k_gather<R, 2, false>), grid, block, 0, s, feat, W, H, pitch, patches, seed, sink); break;
    case 5: hipLaunchKernelGGL((k_gather<R, 2, true>), grid, block, 0, s, feat, W, H, pitch, patches, seed, sink); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace msgpm_ceiling

extern "C" {

// Workgroups of one launch for a W x H frame and patch radius r: one lane
// group per pixel of one colour.  The sink must hold 256 words per workgroup.
int msgpm_ceiling_blocks(int W, int H, int r) {
  if (W < 2 || H < 2 || W > 32767 || H > 32767 || r < 1 || r > 4) return -1;
  const long long groups = (long long)((W + 1) >> 1) * H;
  const int per = (msgpm_ceiling::kWave / (2 * r + 1)) * (msgpm_ceiling::kBlock / msgpm_ceiling::kWave);
  return (int)((groups + per - 1) / per);
}

// One launch of the gather ceiling kernel on `stream`.  feat: device feature
// records of a W x H frame plus one padding record (record_words 32-bit words
// each: 5 = FP32 C=5, 3 = FP32 C=3 or FP16 C=5, 2 = FP16 C=3); sink: device
// buffer of msgpm_ceiling_blocks(W, H, r) * 256 words.  Returns 0, or -1 for
// arguments outside these ranges (nothing launched), or the launch error.
int msgpm_ceiling_gather(const void* feat, int W, int H, int record_words, int r, int bilinear, int patches,
                         unsigned seed, void* sink, void* stream) {
  const int nb = msgpm_ceiling_blocks(W, H, r);
  if (nb < 0 || feat == nullptr || sink == nullptr || patches < 1 || patches > 64) return -1;
  if (record_words != 5 && record_words != 3 && record_words != 2) return -1;
  if (((long long)W * H + 1) * record_words * 4 > 0x7fffffffll) return -1;
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint32_t* out = static_cast<uint32_t*>(sink);
  hipError_t e;
  switch (r) {
    case 1: e = msgpm_ceiling::launch_r<1>(feat, W, H, record_words, bilinear, patches, seed, out, nb, s); break;
    case 2: e = msgpm_ceiling::launch_r<2>(feat, W, H, record_words, bilinear, patches, seed, out, nb, s); break;
    case 3: e = msgpm_ceiling::launch_r<3>(feat, W, H, record_words, bilinear, patches, seed, out, nb, s); break;
    default: e = msgpm_ceiling::launch_r<4>(feat, W, H, record_words, bilinear, patches, seed, out, nb, s); break;
  }
  return (int)e;
}

}  // extern "C"
