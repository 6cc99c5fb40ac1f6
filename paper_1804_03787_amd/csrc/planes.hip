// Plane detection, assignment and forward-backward checks (FP64).
//
// Every floating-point decision here (RANSAC inlier tests, the DLT and its
// least-squares refit, colour-consistency losses, forward-backward distances,
// rounding to the pixel grid) is taken in FP64 with a fixed operation order and
// no contraction, so that identical inputs give identical decisions on any
// implementation that follows the same written steps:
//   * Hartley normalisation: centroid = sum / n, mean distance = sum of
//     sqrt(dx^2 + dy^2) / n, scale sqrt(2) / mean distance, coordinates
//     s * (x - centroid);
//   * 8x8 systems solved by Gaussian elimination with partial pivoting (first
//     largest pivot, rejected below 1e-10), back substitution;
//   * H = T_dst^-1 * Hn * T_src by plain 3x3 products, then divided by H[8];
//   * the refit's normal-equation sums run over the inliers in point-list
//     order, one accumulator per entry.
#include "common.h"

#include <hip/hip_fp16.h>

#pragma clang fp contract(off)

namespace msgpm {

// ---------------------------------------------------------------------------
// Shared FP64 helpers
// ---------------------------------------------------------------------------
__device__ inline bool project(const double* H, double x, double y, double& qx, double& qy) {
  const double w = H[6] * x + H[7] * y + H[8];
  if (!(w > 0)) return false;
  qx = (H[0] * x + H[1] * y + H[2]) / w;
  qy = (H[3] * x + H[4] * y + H[5]) / w;
  return true;
}

__device__ inline void rgb_at(const DevParams& P, const void* F, int idx, double* v) {
  if (P.fp16) {
    const __half* h = reinterpret_cast<const __half*>(F) + (size_t)(P.C == 3 ? 4 : 6) * idx;
    v[0] = __half2float(h[0]);
    v[1] = __half2float(h[1]);
    v[2] = __half2float(h[2]);
  } else {
    const float* f = reinterpret_cast<const float*>(F) + (size_t)P.C * idx;
    v[0] = f[0];
    v[1] = f[1];
    v[2] = f[2];
  }
}

// Colour-consistency error e(p, H): mean over RGB of the squared difference
// between F1 at p and F2 bilinearly sampled at pi(H p) (Eq. 3 in squared RMS
// form); +inf when pi(H p) is undefined or outside the frame.
__device__ double colour_err(const DevParams& P, const Ws& w, int dir, int px, int py, const double* H) {
  const int W = P.W, Hh = P.H;
  double qx, qy;
  if (!project(H, px, py, qx, qy)) return __builtin_huge_val();
  if (qx < 0 || qx > W - 1 || qy < 0 || qy > Hh - 1) return __builtin_huge_val();
  const double fx0 = floor(qx), fy0 = floor(qy);
  int bx = (int)fx0, by = (int)fy0;
  double fx = qx - fx0, fy = qy - fy0;
  if (bx < 0) {
    bx = 0;
    fx = 0;
  } else if (bx >= W - 1) {
    bx = W - 1;
    fx = 0;
  }
  if (by < 0) {
    by = 0;
    fy = 0;
  } else if (by >= Hh - 1) {
    by = Hh - 1;
    fy = 0;
  }
  const int x1 = bx + 1 < W - 1 ? bx + 1 : W - 1;
  const int y1 = by + 1 < Hh - 1 ? by + 1 : Hh - 1;
  const void* F2 = w.feat[1 - dir];
  double a[3], b[3], c[3], d[3], f1[3];
  rgb_at(P, F2, by * W + bx, a);
  rgb_at(P, F2, by * W + x1, b);
  rgb_at(P, F2, y1 * W + bx, c);
  rgb_at(P, F2, y1 * W + x1, d);
  rgb_at(P, w.feat[dir], py * W + px, f1);
  double e = 0;
  for (int k = 0; k < 3; ++k) {
    const double v = (1 - fy) * ((1 - fx) * a[k] + fx * b[k]) + fy * ((1 - fx) * c[k] + fx * d[k]);
    const double df = f1[k] - v;
    e += df * df;
  }
  return e / 3.0;
}

// Forward-backward test of pixel p of direction dir under plane H against the
// other direction's assignment `other`.
__device__ bool fb_test(const DevParams& P, const Ws& w, int px, int py, const double* H, const int32_t* other) {
  const int W = P.W, Hh = P.H;
  double qx, qy;
  if (!project(H, px, py, qx, qy)) return false;
  if (qx < 0 || qx > W - 1 || qy < 0 || qy > Hh - 1) return false;
  const int rx = clampi((int)floor(qx + 0.5), 0, W - 1);
  const int ry = clampi((int)floor(qy + 0.5), 0, Hh - 1);
  const int j = other[ry * W + rx];
  if (j < 0) return false;
  double bx, by;
  if (!project(w.planes[j].H, qx, qy, bx, by)) return false;
  const double d2 = (bx - px) * (bx - px) + (by - py) * (by - py);
  return d2 < P.fb2;
}

// ---------------------------------------------------------------------------
// Homography estimation
// ---------------------------------------------------------------------------
template <int N>
__device__ inline bool hartley_n(const double* x, const double* y, double& s, double& cx, double& cy) {
  double sx = 0, sy = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    sx += x[i];
    sy += y[i];
  }
  cx = sx / N;
  cy = sy / N;
  double md = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const double ex = x[i] - cx, ey = y[i] - cy;
    md += sqrt(ex * ex + ey * ey);
  }
  md = md / N;
  if (!(md > 0)) return false;
  s = sqrt(2.0) / md;
  return true;
}

// Gaussian elimination with partial pivoting on an 8x8 system held in
// registers; row exchanges are done with selects so indices stay static.
__device__ inline bool gauss8(double (&A)[8][8], double (&b)[8], double (&x)[8]) {
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    int piv = k;
    double best = fabs(A[k][k]);
#pragma unroll
    for (int i = k + 1; i < 8; ++i) {
      const double a = fabs(A[i][k]);
      if (a > best) {
        best = a;
        piv = i;
      }
    }
    if (best < 1e-10) return false;
#pragma unroll
    for (int i = k + 1; i < 8; ++i) {
      const bool sw = (i == piv);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const double t = A[k][j];
        A[k][j] = sw ? A[i][j] : A[k][j];
        A[i][j] = sw ? t : A[i][j];
      }
      const double t = b[k];
      b[k] = sw ? b[i] : b[k];
      b[i] = sw ? t : b[i];
    }
#pragma unroll
    for (int i = k + 1; i < 8; ++i) {
      const double f = A[i][k] / A[k][k];
#pragma unroll
      for (int j = k; j < 8; ++j) A[i][j] -= f * A[k][j];
      b[i] -= f * b[k];
    }
  }
#pragma unroll
  for (int i = 7; i >= 0; --i) {
    double s = b[i];
#pragma unroll
    for (int j = i + 1; j < 8; ++j) s -= A[i][j] * x[j];
    x[i] = s / A[i][i];
  }
  return true;
}

__device__ inline bool denormalise(const double (&h)[8], double s1, double c1x, double c1y, double s2, double c2x,
                                   double c2y, double* Hout) {
  const double Hn[9] = {h[0], h[1], h[2], h[3], h[4], h[5], h[6], h[7], 1.0};
  const double Ts[9] = {s1, 0, -s1 * c1x, 0, s1, -s1 * c1y, 0, 0, 1};
  const double Ti[9] = {1.0 / s2, 0, c2x, 0, 1.0 / s2, c2y, 0, 0, 1};
  double M[9], R[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double t = 0;
#pragma unroll
      for (int k = 0; k < 3; ++k) t += Hn[i * 3 + k] * Ts[k * 3 + j];
      M[i * 3 + j] = t;
    }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double t = 0;
#pragma unroll
      for (int k = 0; k < 3; ++k) t += Ti[i * 3 + k] * M[k * 3 + j];
      R[i * 3 + j] = t;
    }
  if (fabs(R[8]) < 1e-12) return false;
  const double d = R[8];
#pragma unroll
  for (int i = 0; i < 9; ++i) Hout[i] = R[i] / d;
  return true;
}

// Normalised 4-point DLT with H[8] = 1.
__device__ inline bool dlt4(const double (&sx)[4], const double (&sy)[4], const double (&dx)[4],
                            const double (&dy)[4], double* Hout) {
  double s1, c1x, c1y, s2, c2x, c2y;
  if (!hartley_n<4>(sx, sy, s1, c1x, c1y)) return false;
  if (!hartley_n<4>(dx, dy, s2, c2x, c2y)) return false;
  double A[8][8], b[8], h[8];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double x = s1 * (sx[i] - c1x), y = s1 * (sy[i] - c1y);
    const double u = s2 * (dx[i] - c2x), v = s2 * (dy[i] - c2y);
    A[2 * i][0] = x;
    A[2 * i][1] = y;
    A[2 * i][2] = 1;
    A[2 * i][3] = 0;
    A[2 * i][4] = 0;
    A[2 * i][5] = 0;
    A[2 * i][6] = -x * u;
    A[2 * i][7] = -y * u;
    A[2 * i + 1][0] = 0;
    A[2 * i + 1][1] = 0;
    A[2 * i + 1][2] = 0;
    A[2 * i + 1][3] = x;
    A[2 * i + 1][4] = y;
    A[2 * i + 1][5] = 1;
    A[2 * i + 1][6] = -x * v;
    A[2 * i + 1][7] = -y * v;
    b[2 * i] = u;
    b[2 * i + 1] = v;
  }
  if (!gauss8(A, b, h)) return false;
  return denormalise(h, s1, c1x, c1y, s2, c2x, c2y, Hout);
}

// Reprojection inlier test, division-free: w > 0 and |(u, v) - w q|^2 < tau^2 w^2,
// each product-plus-sum a fused multiply-add (rounded once).
__device__ inline bool ransac_inlier(const double* H, double x, double y, double qx, double qy, double tau2) {
  const double w = fma(H[6], x, fma(H[7], y, H[8]));
  if (!(w > 0)) return false;
  const double u = fma(H[0], x, fma(H[1], y, H[2]));
  const double v = fma(H[3], x, fma(H[4], y, H[5]));
  const double ex = fma(-w, qx, u), ey = fma(-w, qy, v);
  const double e2 = fma(ex, ex, ey * ey);
  const double t = tau2 * w * w;
  return e2 < t;
}

__device__ inline bool collinear(int ax, int ay, int bx, int by, int cx, int cy) {
  return (long long)(bx - ax) * (cy - ay) - (long long)(by - ay) * (cx - ax) == 0;
}

__device__ inline uint32_t pack_pt(int x, int y) { return (uint32_t)x | ((uint32_t)y << 16); }
__device__ inline int pt_x(uint32_t v) { return (int)(v & 0xffffu); }
__device__ inline int pt_y(uint32_t v) { return (int)(v >> 16); }

// ---------------------------------------------------------------------------
// RANSAC: one workgroup per (window, direction).
//
// 1. The window's point list (source pixel, NNF target; row-major, stage 2 only
//    the unassigned pixels) is compacted into LDS.
// 2. Hypotheses are made 256 at a time, one per thread: sample, degeneracy
//    test, normalised DLT; the batch's 8 coefficients per hypothesis go to LDS.
// 3. Scoring is point-major: each wave takes a strided share of the points,
//    4 per lane, converted to FP64 once, and tests them against every valid
//    hypothesis of the batch (coefficients broadcast from LDS); per-hypothesis
//    counts are ballot popcounts, gathered into lanes and added into LDS.
// 4. The winner (largest count, lowest index) is refitted by least squares on
//    its inliers.  The inliers are compacted in list order; the centroid sums
//    are integer sums (exact in any order); the mean-distance and
//    normal-equation sums keep the sequential order of the definition: the
//    per-inlier terms are produced by waves 1-3 into a double buffer while
//    wave 0 adds them, one lane per distinct sum, in list order.
// 5. The refit's support is recounted over the window (read again from the
//    NNF) and kept when it does not lose support.
// ---------------------------------------------------------------------------
constexpr int kMdChunk = 192;   // inliers per mean-distance chunk: one per producer thread
constexpr int kNeChunk = 32;    // inliers per normal-equation chunk: 6 producer threads each
// doubles per inlier in a normal-equation chunk: the 38 slots used, no padding,
// so that three workgroups of 64x64 windows (32 KB of points each) fit the
// 160 KB of LDS of a CU (measured on MI355X: the two stages of that level
// 6 and 13 % faster than with two workgroups per CU)
constexpr int kNeSlots = 38;
constexpr int kNeSums = 29;     // distinct normal-equation sums (below)
constexpr int kNeZero = 37;     // slot holding +0 (the second term of one-term sums)
constexpr int kAuxDoubles = 2 * kNeChunk * kNeSlots;
static_assert(kAuxDoubles >= kBlock * 8, "hypothesis batch must fit the aux area");
static_assert(kAuxDoubles >= 2 * 2 * kMdChunk, "mean-distance buffers must fit the aux area");
static_assert(kMdChunk == kBlock - kWave && kNeChunk * 6 == kBlock - kWave, "producers are waves 1-3");
static_assert(kNeSlots == kNeZero + 1, "slots 0-28, 32-36 and the zero slot");

// Inlier test against 8 coefficients with h8 = 1 (the DLT and the refit
// normalise to it), same operations as ransac_inlier.
__device__ inline bool inlier8(const double* H, double x, double y, double qx, double qy, double tau2) {
  const double w = fma(H[6], x, fma(H[7], y, 1.0));
  const double u = fma(H[0], x, fma(H[1], y, H[2]));
  const double v = fma(H[3], x, fma(H[4], y, H[5]));
  const double ex = fma(-w, qx, u), ey = fma(-w, qy, v);
  const double e2 = fma(ex, ex, ey * ey);
  const double t = tau2 * w * w;
  return (w > 0) && (e2 < t);
}

// Hypothesis h of window b: partial Fisher-Yates over a virtual identity
// permutation of the n points, degeneracy test, normalised DLT.
__device__ inline bool make_hypothesis(const DevParams& P, int b, int h, int n, uint64_t w3, const uint32_t* src,
                                       const uint32_t* dst, double* Hout) {
  uint64_t c[4] = {(uint64_t)(uint32_t)b, (uint64_t)h, 0, w3};
  philox4x64(c, P.seed, 0);
  int key[8], val[8], nm = 0, sel[4];
#pragma unroll
  for (int m = 0; m < 8; ++m) key[m] = val[m] = -1;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int rj = j + draw_below(c[j], (uint32_t)(n - j));
    int vj = j, vr = rj, fj = -1, fr = -1;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      if (m < nm && key[m] == j) {
        vj = val[m];
        fj = m;
      }
      if (m < nm && key[m] == rj) {
        vr = val[m];
        fr = m;
      }
    }
    if (fj < 0) fj = nm++;
    if (fr < 0) fr = nm++;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      if (m == fj) {
        key[m] = j;
        val[m] = vr;
      }
      if (m == fr) {
        key[m] = rj;
        val[m] = vj;
      }
    }
    sel[j] = vr;
  }
  int SX[4], SY[4], DX[4], DY[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t a = src[sel[j]], d = dst[sel[j]];
    SX[j] = pt_x(a);
    SY[j] = pt_y(a);
    DX[j] = pt_x(d);
    DY[j] = pt_y(d);
  }
  bool degen = false;
  degen = degen || collinear(SX[0], SY[0], SX[1], SY[1], SX[2], SY[2]);
  degen = degen || collinear(SX[0], SY[0], SX[1], SY[1], SX[3], SY[3]);
  degen = degen || collinear(SX[0], SY[0], SX[2], SY[2], SX[3], SY[3]);
  degen = degen || collinear(SX[1], SY[1], SX[2], SY[2], SX[3], SY[3]);
  degen = degen || collinear(DX[0], DY[0], DX[1], DY[1], DX[2], DY[2]);
  degen = degen || collinear(DX[0], DY[0], DX[1], DY[1], DX[3], DY[3]);
  degen = degen || collinear(DX[0], DY[0], DX[2], DY[2], DX[3], DY[3]);
  degen = degen || collinear(DX[1], DY[1], DX[2], DY[2], DX[3], DY[3]);
  if (degen) return false;
  const double sx[4] = {(double)SX[0], (double)SX[1], (double)SX[2], (double)SX[3]};
  const double sy[4] = {(double)SY[0], (double)SY[1], (double)SY[2], (double)SY[3]};
  const double ddx[4] = {(double)DX[0], (double)DX[1], (double)DX[2], (double)DX[3]};
  const double ddy[4] = {(double)DY[0], (double)DY[1], (double)DY[2], (double)DY[3]};
  return dlt4(sx, sy, ddx, ddy, Hout);
}

// Normal-equation terms of one inlier (normalised x, y, u, v).  With
// a0 = (x, y, 1, 0, 0, 0, -xu, -yu) and a1 = (0, 0, 0, x, y, 1, -xv, -yv), the
// sums N[j][k] += a0[j] a0[k]; N[j][k] += a1[j] a1[k]; rhs[j] += a0[j] u;
// rhs[j] += a1[j] v have, per inlier, at most two non-zero terms; the zero
// products leave a sum unchanged (it starts at +0 and cannot become -0), so
// only the non-zero terms are added.  29 distinct sums remain:
//   0-5   N00 N01 N02 N11 N12 N22 (= N33 N34 N35 N44 N45 N55)
//   6-11  N06 N07 N16 N17 N26 N27        12-14 rhs0 rhs1 rhs2
//   15-20 N36 N37 N46 N47 N56 N57        21-23 rhs3 rhs4 rhs5
//   24-28 N66 N67 N77 rhs6 rhs7 (two terms: the a0 one, then the a1 one)
// Slot s < 29 holds the first (or only) term of sum s; slots 32-36 the second
// term of sums 24-28; slot 37 is +0.  Each producer thread writes one part.
__device__ inline void ne_terms(double x, double y, double u, double v, int part, double* T) {
  const double p6 = -x * u, p7 = -y * u, q6 = -x * v, q7 = -y * v;
  switch (part) {
    case 0:
      T[0] = x * x;
      T[1] = x * y;
      T[2] = x * 1.0;
      T[3] = y * y;
      T[4] = y * 1.0;
      T[5] = 1.0;
      break;
    case 1:
      T[6] = x * p6;
      T[7] = x * p7;
      T[8] = y * p6;
      T[9] = y * p7;
      T[10] = 1.0 * p6;
      T[11] = 1.0 * p7;
      break;
    case 2:
      T[12] = x * u;
      T[13] = y * u;
      T[14] = 1.0 * u;
      T[21] = x * v;
      T[22] = y * v;
      T[23] = 1.0 * v;
      break;
    case 3:
      T[15] = x * q6;
      T[16] = x * q7;
      T[17] = y * q6;
      T[18] = y * q7;
      T[19] = 1.0 * q6;
      T[20] = 1.0 * q7;
      break;
    case 4:
      T[24] = p6 * p6;
      T[32] = q6 * q6;
      T[25] = p6 * p7;
      T[33] = q6 * q7;
      T[26] = p7 * p7;
      T[34] = q7 * q7;
      break;
    default:
      T[27] = p6 * u;
      T[35] = q6 * v;
      T[28] = p7 * u;
      T[36] = q7 * v;
      T[kNeZero] = 0.0;
      break;
  }
}

// Scores one batch of hypotheses.  Work items are (chunk of U * 64 points,
// group of 64 hypotheses) pairs dealt round-robin to the waves; a lane holds U
// points in FP64 and the per-hypothesis counts are popcounts of the ballots of
// the two conditions of inlier8 (same operations), gathered into lane j for
// hypothesis j of the group and added into s_cnt.
template <int U>
__device__ inline void score_batch(const double* aux, const unsigned long long* s_gmask, int* s_cnt, int ngroups,
                                   const uint32_t* src, const uint32_t* dst, int n, double tau2, int wave,
                                   int lane) {
  const int nchunks = (n + U * kWave - 1) / (U * kWave);
  const int nitems = nchunks * ngroups;
  for (int item = wave; item < nitems; item += kBlock / kWave) {
    const int chunk = item / ngroups, g = item - chunk * ngroups;
    unsigned long long m = s_gmask[g];
    m = ((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(m >> 32)) << 32) |
        (unsigned)__builtin_amdgcn_readfirstlane((int)(m & 0xffffffffull));
    if (!m) continue;
    double X[U], Y[U], QX[U], QY[U];
    unsigned long long vm[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = chunk * U * kWave + u * kWave + lane;
      const bool has = i < n;
      const uint32_t a = has ? src[i] : 0u, d = has ? dst[i] : 0u;
      X[u] = (double)pt_x(a);
      Y[u] = (double)pt_y(a);
      QX[u] = (double)pt_x(d);
      QY[u] = (double)pt_y(d);
      vm[u] = __ballot(has);
    }
    int tmp = 0;
    while (m) {
      const int j = __builtin_ctzll(m);
      m &= m - 1ull;
      const double* H = aux + (g * kWave + j) * 8;
      double Hc[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) Hc[k] = H[k];
      int c = 0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double w = fma(Hc[6], X[u], fma(Hc[7], Y[u], 1.0));
        const double uu = fma(Hc[0], X[u], fma(Hc[1], Y[u], Hc[2]));
        const double vv = fma(Hc[3], X[u], fma(Hc[4], Y[u], Hc[5]));
        const double ex = fma(-w, QX[u], uu), ey = fma(-w, QY[u], vv);
        const double e2 = fma(ex, ex, ey * ey);
        const double t = tau2 * w * w;
        const unsigned long long pos = __ballot(w > 0), close = __ballot(e2 < t);
        c += __popcll(pos & close & vm[u]);
      }
      tmp = lane == j ? c : tmp;
    }
    atomicAdd(&s_cnt[g * kWave + lane], tmp);
  }
}

// UMAX: points per lane of the scoring loop for the largest windows (8 for
// windows of more than 512 points, whose scoring dominates; 4 otherwise, which
// keeps the hypothesis generation of small windows from spilling more).
template <int UMAX>
__device__ __forceinline__ void ransac_body(const DevParams& P, const Ws& w, Blk bk, int level, int stage) {
  extern __shared__ double smem_d[];
  __shared__ int s_wave[kBlock / kWave];
  __shared__ int s_n, s_ni, s_ok, s_cnt_r;
  __shared__ int s_cnt[kBlock];
  __shared__ unsigned long long s_gmask[kBlock / kWave];
  __shared__ unsigned long long s_key[kBlock / kWave];
  __shared__ unsigned long long s_isum[4];
  __shared__ double s_H[8], s_Hr[9];
  __shared__ double s_md[2];
  __shared__ double s_ne[kNeSums];

  const int t = threadIdx.x, lane = t & (kWave - 1), wave = t / kWave;
  const int b = bk.x, dir = bk.y;
  const int W = P.W, Hh = P.H;
  const int B = P.block[level], nbx = P.nbx[level];
  const int bw = B < W ? B : W, bh = B < Hh ? B : Hh;
  const int x0 = block_origin(W, B, b % nbx), y0 = block_origin(Hh, B, b / nbx);
  const int nmax = bw * bh;
  double* aux = smem_d;
  uint32_t* src = reinterpret_cast<uint32_t*>(smem_d + kAuxDoubles);
  uint32_t* dst = src + nmax;
  msgpm_plane* pl = &w.planes[plane_index(P, dir, level, stage, b)];
  const int32_t* nnf = w.nnf[dir];
  const int32_t* win = w.win[dir];
  const unsigned long long lt_mask = (1ull << lane) - 1ull;

  // 1. point list
  if (t == 0) {
    s_n = 0;
    s_ni = 0;
    s_cnt_r = 0;
  }
  if (t < 4) s_isum[t] = 0ull;
  __syncthreads();
  for (int c0 = 0; c0 < nmax; c0 += kBlock) {
    const int i = c0 + t;
    int x = 0, y = 0, p = 0;
    bool keep = i < nmax;
    if (keep) {
      x = x0 + i % bw;
      y = y0 + i / bw;
      p = y * W + x;
      if (stage == 2) keep = win[p] < 0;
    }
    const unsigned long long m = __ballot(keep);
    const int before = __popcll(m & lt_mask);
    if (lane == 0) s_wave[wave] = __popcll(m);
    __syncthreads();
    int off = s_n;
    for (int k = 0; k < wave; ++k) off += s_wave[k];
    if (keep) {
      const int32_t v = nnf[p];
      src[off + before] = pack_pt(x, y);
      dst[off + before] = pack_pt(x + off_dx(v), y + off_dy(v));
    }
    __syncthreads();
    if (t == 0) s_n += s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
    __syncthreads();
  }
  const int n = s_n;
  const int mmin_frac = (int)ceil(P.mu * (double)bw * (double)bh);
  const int mmin = mmin_frac > P.m_min_abs ? mmin_frac : P.m_min_abs;

  msgpm_plane out;
  for (int i = 0; i < 9; ++i) out.H[i] = 0.0;
  out.dir = dir;
  out.level = level;
  out.stage = stage;
  out.block = b;
  out.x0 = x0;
  out.y0 = y0;
  out.bw = bw;
  out.bh = bh;
  out.support = n;
  out.count = 0;
  out.hyp = -1;
  out.hyp_count = 0;
  out.refit = out.detected = out.rk = out.pass = out.valid = out.rin = 0;
  if (n < mmin || n < 4) {
    if (t == 0) *pl = out;
    return;
  }

  // 2-3. hypotheses in batches of 256, point-major scoring
  const double tau2 = P.tau2;
  const uint64_t w3 = rng_word3(3, dir, level + 1, stage);
  unsigned long long best = 0ull;  // (count << 32) | ~h, 0 = none
  for (int base = 0; base < P.hyps; base += kBlock) {
    const int h = base + t;
    bool ok = false;
    if (h < P.hyps) {
      double Hx[9];
      ok = make_hypothesis(P, b, h, n, w3, src, dst, Hx);
      if (ok) {
#pragma unroll
        for (int j = 0; j < 8; ++j) aux[t * 8 + j] = Hx[j];
      }
    }
    s_cnt[t] = 0;
    const unsigned long long gm = __ballot(ok);
    if (lane == 0) s_gmask[wave] = gm;
    __syncthreads();
    const int left = P.hyps - base;
    const int ngroups = ((left < kBlock ? left : kBlock) + kWave - 1) / kWave;
    if (n <= kWave)
      score_batch<1>(aux, s_gmask, s_cnt, ngroups, src, dst, n, tau2, wave, lane);
    else if (n <= 2 * kWave)
      score_batch<2>(aux, s_gmask, s_cnt, ngroups, src, dst, n, tau2, wave, lane);
    else if (UMAX < 8 || n <= 8 * kWave)
      score_batch<4>(aux, s_gmask, s_cnt, ngroups, src, dst, n, tau2, wave, lane);
    else
      score_batch<UMAX>(aux, s_gmask, s_cnt, ngroups, src, dst, n, tau2, wave, lane);
    __syncthreads();
    unsigned long long key = ok ? (((unsigned long long)s_cnt[t] << 32) | (0xffffffffu - (unsigned)h)) : 0ull;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const unsigned long long other = __shfl_xor(key, o);
      key = other > key ? other : key;
    }
    if (lane == 0) s_key[wave] = key;
    __syncthreads();
    unsigned long long bk = s_key[0];
    for (int k = 1; k < kBlock / kWave; ++k) bk = s_key[k] > bk ? s_key[k] : bk;
    if (bk > best) {
      best = bk;
      const int bh_ = (int)(0xffffffffu - (unsigned)(bk & 0xffffffffull));
      if (bh_ == h) {
#pragma unroll
        for (int j = 0; j < 8; ++j) s_H[j] = aux[t * 8 + j];
      }
    }
    __syncthreads();
  }
  if (best == 0ull) {
    if (t == 0) *pl = out;
    return;
  }
  const int best_cnt = (int)(best >> 32);
  const int best_h = (int)(0xffffffffu - (unsigned)(best & 0xffffffffull));

  // 4. inliers of the winner, compacted in list order; integer centroid sums
  unsigned long long isum[4] = {0ull, 0ull, 0ull, 0ull};
  for (int c0 = 0; c0 < n; c0 += kBlock) {
    const int i = c0 + t;
    const bool has = i < n;
    const uint32_t a = has ? src[i] : 0u, d = has ? dst[i] : 0u;
    const bool in = has && inlier8(s_H, (double)pt_x(a), (double)pt_y(a), (double)pt_x(d), (double)pt_y(d), tau2);
    const unsigned long long m = __ballot(in);
    const int before = __popcll(m & lt_mask);
    if (lane == 0) s_wave[wave] = __popcll(m);
    if (in) {
      isum[0] += (unsigned)pt_x(a);
      isum[1] += (unsigned)pt_y(a);
      isum[2] += (unsigned)pt_x(d);
      isum[3] += (unsigned)pt_y(d);
    }
    __syncthreads();
    int off = s_ni;
    for (int k = 0; k < wave; ++k) off += s_wave[k];
    if (in) {
      src[off + before] = a;
      dst[off + before] = d;
    }
    __syncthreads();
    if (t == 0) s_ni += s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    unsigned long long v = isum[k];
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) v += __shfl_xor(v, o);
    if (lane == 0) atomicAdd(&s_isum[k], v);
  }
  __syncthreads();
  const int ni = s_ni;
  bool norm_ok = ni >= 4;
  // centroids: the sums are integers below 2^53, so FP64 sums in any order equal them
  const double c1x = (double)s_isum[0] / ni, c1y = (double)s_isum[1] / ni;
  const double c2x = (double)s_isum[2] / ni, c2y = (double)s_isum[3] / ni;
  double s1 = 0, s2 = 0;
  if (norm_ok) {
    // mean distances: lane 0 sums the source terms, lane 1 the target terms, in list order
    const int nch = (ni + kMdChunk - 1) / kMdChunk;
    const int tp = t - kWave;
    auto produce = [&](int k) {
      const int i = k * kMdChunk + tp;
      if (i < ni) {
        double* buf = aux + (k & 1) * 2 * kMdChunk;
        const uint32_t a = src[i], d = dst[i];
        const double ex = (double)pt_x(a) - c1x, ey = (double)pt_y(a) - c1y;
        const double fx = (double)pt_x(d) - c2x, fy = (double)pt_y(d) - c2y;
        buf[tp] = sqrt(ex * ex + ey * ey);
        buf[kMdChunk + tp] = sqrt(fx * fx + fy * fy);
      }
    };
    if (wave > 0) produce(0);
    __syncthreads();
    double acc = 0;
    for (int k = 0; k < nch; ++k) {
      if (wave == 0) {
        const double* col = aux + (k & 1) * 2 * kMdChunk + (lane & 1) * kMdChunk;
        const int cnt = ni - k * kMdChunk < kMdChunk ? ni - k * kMdChunk : kMdChunk;
        for (int j = 0; j < cnt; ++j) acc += col[j];
      } else if (k + 1 < nch) {
        produce(k + 1);
      }
      __syncthreads();
    }
    if (t < 2) s_md[t] = acc;
    __syncthreads();
    const double md1 = s_md[0] / ni, md2 = s_md[1] / ni;
    norm_ok = (md1 > 0) && (md2 > 0);
    s1 = sqrt(2.0) / md1;
    s2 = sqrt(2.0) / md2;
  }
  if (norm_ok) {
    // normal equations: lane s of wave 0 owns sum s
    const int nch = (ni + kNeChunk - 1) / kNeChunk;
    const int tp = t - kWave;
    auto produce = [&](int k) {
      const int i = k * kNeChunk + tp / 6;
      if (i < ni) {
        double* T = aux + ((k & 1) * kNeChunk + tp / 6) * kNeSlots;
        const uint32_t a = src[i], d = dst[i];
        const double x = s1 * ((double)pt_x(a) - c1x), y = s1 * ((double)pt_y(a) - c1y);
        const double u = s2 * ((double)pt_x(d) - c2x), v = s2 * ((double)pt_y(d) - c2y);
        ne_terms(x, y, u, v, tp % 6, T);
      }
    };
    if (wave > 0) produce(0);
    __syncthreads();
    const int s = lane < kNeSums ? lane : kNeSums - 1;
    const int s2nd = s >= 24 ? 32 + (s - 24) : kNeZero;
    double acc = 0;
    for (int k = 0; k < nch; ++k) {
      if (wave == 0) {
        const double* T = aux + (k & 1) * kNeChunk * kNeSlots;
        const int cnt = ni - k * kNeChunk < kNeChunk ? ni - k * kNeChunk : kNeChunk;
        for (int j = 0; j < cnt; ++j) {
          acc += T[j * kNeSlots + s];
          acc += T[j * kNeSlots + s2nd];
        }
      } else if (k + 1 < nch) {
        produce(k + 1);
      }
      __syncthreads();
    }
    if (t < kNeSums) s_ne[t] = acc;
    __syncthreads();
  }
  if (t == 0) {
    s_ok = 0;
    if (norm_ok) {
      const double* S = s_ne;
      double A[8][8], rhs[8], hsol[8];
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int q = 0; q < 8; ++q) A[r][q] = 0.0;
      const int tri[6][3] = {{0, 0, 0}, {0, 1, 1}, {0, 2, 2}, {1, 1, 3}, {1, 2, 4}, {2, 2, 5}};
#pragma unroll
      for (int e = 0; e < 6; ++e) {
        const int r = tri[e][0], q = tri[e][1];
        const double v = S[tri[e][2]];
        A[r][q] = A[q][r] = v;
        A[r + 3][q + 3] = A[q + 3][r + 3] = v;
      }
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        A[r][6] = A[6][r] = S[6 + 2 * r];
        A[r][7] = A[7][r] = S[7 + 2 * r];
        A[r + 3][6] = A[6][r + 3] = S[15 + 2 * r];
        A[r + 3][7] = A[7][r + 3] = S[16 + 2 * r];
        rhs[r] = S[12 + r];
        rhs[r + 3] = S[21 + r];
      }
      A[6][6] = S[24];
      A[6][7] = A[7][6] = S[25];
      A[7][7] = S[26];
      rhs[6] = S[27];
      rhs[7] = S[28];
      double Hr[9];
      if (gauss8(A, rhs, hsol) && denormalise(hsol, s1, c1x, c1y, s2, c2x, c2y, Hr)) {
        for (int i = 0; i < 9; ++i) s_Hr[i] = Hr[i];
        s_ok = 1;
      }
    }
  }
  __syncthreads();

  // 5. support of the refit over the whole window
  int final_cnt = best_cnt;
  bool use_refit = false;
  if (s_ok) {
    int local = 0;
    for (int i = t; i < nmax; i += kBlock) {
      const int x = x0 + i % bw, y = y0 + i / bw, p = y * W + x;
      if (stage == 2 && win[p] >= 0) continue;
      const int32_t v = nnf[p];
      local += ransac_inlier(s_Hr, (double)x, (double)y, (double)(x + off_dx(v)), (double)(y + off_dy(v)), tau2);
    }
    atomicAdd(&s_cnt_r, local);
    __syncthreads();
    if (s_cnt_r >= best_cnt) {
      use_refit = true;
      final_cnt = s_cnt_r;
    }
  }
  if (t == 0) {
    for (int i = 0; i < 8; ++i) out.H[i] = use_refit ? s_Hr[i] : s_H[i];
    out.H[8] = use_refit ? s_Hr[8] : 1.0;
    out.hyp = best_h;
    out.hyp_count = best_cnt;
    out.count = final_cnt;
    out.refit = use_refit ? 1 : 0;
    out.detected = final_cnt >= mmin ? 1 : 0;
    out.valid = out.detected;
    *pl = out;
  }
}

// Held to 168 VGPRs (3 waves per SIMD, a few registers of the DLT spilled): the
// scoring loop needs the waves to hide FP64 latency more than the hypothesis
// generation needs the registers.
template <int UMAX>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_ransac(DevParams P, Ws w, int level,
                                                                                         int stage) {
  ransac_body<UMAX>(P, w, blk_here(), level, stage);
}

template <int UMAX>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void kb_ransac(const uint8_t* __restrict__ tab, int k, BArgs A) {
  const BatchView V = batch_view(tab, k);
  const PairDesc* __restrict__ pd = V.pd;
  const Item* __restrict__ it = V.it;
  const int n = V.n, total = V.total;
  for_each_item<true>(it, n, total, [&](int i, Blk bk) {
    const Item& I = it[i];
    ransac_body<UMAX>(pd[I.pair].P, pd[I.pair].w, bk, A.a[0], A.a[1]);
  });
}

// Windows of more than this many points take the 8-points-per-lane scoring.
constexpr size_t kRansacWide = 8 * kWave;

template <class K>
static hipError_t ransac_lds(K kernel, size_t lds) {
  if (lds <= 64 * 1024) return hipSuccess;
  // windows above 64x64 keep their point list in more than 64 KB of LDS
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds);
}

// ---------------------------------------------------------------------------
// Assignment: per pixel, the minimum of the key (L, level, stage, window) over
// the incumbent and the inlier planes of (level, stage) whose window covers p.
// ---------------------------------------------------------------------------
__device__ inline bool key_less(double L1, const msgpm_plane& a, double L2, const msgpm_plane& b) {
  if (L1 != L2) return L1 < L2;
  if (a.level != b.level) return a.level < b.level;
  if (a.stage != b.stage) return a.stage < b.stage;
  return a.block < b.block;
}

__device__ __forceinline__ void assign_body(const DevParams& P, const Ws& w, Blk bk, int level, int stage, int tentative) {
  const int p = bk.x * kBlock + threadIdx.x, dir = bk.y;
  const int W = P.W, Hh = P.H;
  if (p >= W * Hh) return;
  const int x = p % W, y = p / W;
  int bwin = w.win[dir][p];
  double bl = w.loss[dir][p];
  // stage 2 offers only the residual pixels (Sec. 3.2); with the strict level
  // priority (Sec. 3.3) every stage does: an assigned pixel keeps its plane
  if ((stage == 1 && !P.merge_strict) || bwin < 0) {
    const int B = P.block[level], nbx = P.nbx[level], nby = P.nby[level];
    int xlo, xhi, ylo, yhi;
    cover_range(W, B, nbx, x, xlo, xhi);
    cover_range(Hh, B, nby, y, ylo, yhi);
    for (int by = ylo; by <= yhi; ++by)
      for (int bx = xlo; bx <= xhi; ++bx) {
        const int k = plane_index(P, dir, level, stage, by * nbx + bx);
        const msgpm_plane& pk = w.planes[k];
        if (!(tentative ? pk.detected : pk.valid)) continue;
        const double e = colour_err(P, w, dir, x, y, pk.H);
        if (!(e < P.eps2)) continue;
        if (bwin < 0 || key_less(e, pk, bl, w.planes[bwin])) {
          bwin = k;
          bl = e;
        }
      }
  }
  int32_t* ow = tentative ? w.twin[dir] : w.win[dir];
  double* ol = tentative ? w.tloss[dir] : w.loss[dir];
  ow[p] = bwin;
  ol[p] = bwin >= 0 ? bl : __builtin_huge_val();
}

__global__ __launch_bounds__(kBlock) void k_assign(DevParams P, Ws w, int level, int stage, int tentative) {
  assign_body(P, w, blk_here(), level, stage, tentative);
}

__global__ __launch_bounds__(kBlock) void kb_assign(const uint8_t* __restrict__ tab, int k, BArgs A) {
  const BatchView V = batch_view(tab, k);
  const PairDesc* __restrict__ pd = V.pd;
  const Item* __restrict__ it = V.it;
  const int n = V.n, total = V.total;
  for_each_item(it, n, total, [&](int i, Blk bk) {
    const Item& I = it[i];
    assign_body(pd[I.pair].P, pd[I.pair].w, bk, A.a[0], A.a[1], A.a[2]);
  });
}

// ---------------------------------------------------------------------------
// Plane symmetry: one workgroup per (window, direction).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void symmetry_body(const DevParams& P, const Ws& w, Blk bk, int level, int stage) {
  __shared__ int s_rk, s_pass, s_rin;
  const int t = threadIdx.x, b = bk.x, dir = bk.y;
  msgpm_plane* pl = &w.planes[plane_index(P, dir, level, stage, b)];
  if (t == 0) {
    s_rk = 0;
    s_pass = 0;
    s_rin = 0;
  }
  __syncthreads();
  if (!pl->detected) {
    if (t == 0) {
      pl->rk = 0;
      pl->pass = 0;
      pl->rin = 0;
      pl->valid = 0;
    }
    return;
  }
  const int W = P.W;
  const int x0 = pl->x0, y0 = pl->y0, bw = pl->bw, bh = pl->bh;
  double H[9];
  for (int i = 0; i < 9; ++i) H[i] = pl->H[i];
  const int32_t* other = w.twin[1 - dir];
  int rk = 0, pass = 0, rin = 0;
  for (int i = t; i < bw * bh; i += kBlock) {
    const int x = x0 + i % bw, y = y0 + i / bw;
    if (stage == 2 && w.win[dir][y * W + x] >= 0) continue;
    const double e = colour_err(P, w, dir, x, y, H);
    if (e < P.eps2) {
      ++rk;
      pass += fb_test(P, w, x, y, H, other) ? 1 : 0;
      // cue 3: the plane's own RANSAC test on the pixel's NNF match
      const int32_t v = w.nnf[dir][y * W + x];
      rin += ransac_inlier(H, (double)x, (double)y, (double)(x + off_dx(v)), (double)(y + off_dy(v)), P.tau2) ? 1 : 0;
    }
  }
  atomicAdd(&s_rk, rk);
  atomicAdd(&s_pass, pass);
  atomicAdd(&s_rin, rin);
  __syncthreads();
  if (t == 0) {
    const int mmin_frac = (int)ceil(P.mu * (double)bw * (double)bh);
    const int mmin = mmin_frac > P.m_min_abs ? mmin_frac : P.m_min_abs;
    pl->rk = s_rk;
    pl->pass = s_pass;
    pl->rin = s_rin;
    bool ok = s_rk >= mmin && (long long)s_pass * P.eta_den > (long long)P.eta_num * s_rk;
    if (P.cues & MSGPM_FLAG_CUE_OVERLAP) ok = ok && (long long)s_rin * P.eta_den > (long long)P.eta_num * s_rk;
    pl->valid = ok ? 1 : 0;
  }
}

__global__ __launch_bounds__(kBlock) void k_symmetry(DevParams P, Ws w, int level, int stage) {
  symmetry_body(P, w, blk_here(), level, stage);
}

__global__ __launch_bounds__(kBlock) void kb_symmetry(const uint8_t* __restrict__ tab, int k, BArgs A) {
  const BatchView V = batch_view(tab, k);
  const PairDesc* __restrict__ pd = V.pd;
  const Item* __restrict__ it = V.it;
  const int n = V.n, total = V.total;
  for_each_item<true>(it, n, total, [&](int i, Blk bk) {
    const Item& I = it[i];
    symmetry_body(pd[I.pair].P, pd[I.pair].w, bk, A.a[0], A.a[1]);
  });
}

// ---------------------------------------------------------------------------
// End-of-level forward-backward check (Jacobi over both directions).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void fb_body(const DevParams& P, const Ws& w, Blk bk) {
  const int p = bk.x * kBlock + threadIdx.x, dir = bk.y;
  if (p >= P.W * P.H) return;
  const int j = w.win[dir][p];
  int o = j;
  double l = w.loss[dir][p];
  if (j >= 0 && !fb_test(P, w, p % P.W, p / P.W, w.planes[j].H, w.win[1 - dir])) {
    o = -1;
    l = __builtin_huge_val();
  }
  w.twin[dir][p] = o;
  w.tloss[dir][p] = l;
}

__global__ __launch_bounds__(kBlock) void k_fb(DevParams P, Ws w) {
  fb_body(P, w, blk_here());
}

__global__ __launch_bounds__(kBlock) void kb_fb(const uint8_t* __restrict__ tab, int k, BArgs A) {
  const BatchView V = batch_view(tab, k);
  const PairDesc* __restrict__ pd = V.pd;
  const Item* __restrict__ it = V.it;
  const int n = V.n, total = V.total;
  for_each_item(it, n, total, [&](int i, Blk bk) {
    const Item& I = it[i];
    fb_body(pd[I.pair].P, pd[I.pair].w, bk);
  });
}

__device__ __forceinline__ void commit_body(const DevParams& P, const Ws& w, Blk bk) {
  const int p = bk.x * kBlock + threadIdx.x, dir = bk.y;
  if (p >= P.W * P.H) return;
  w.win[dir][p] = w.twin[dir][p];
  w.loss[dir][p] = w.tloss[dir][p];
}

__global__ __launch_bounds__(kBlock) void k_commit(DevParams P, Ws w) {
  commit_body(P, w, blk_here());
}

__global__ __launch_bounds__(kBlock) void kb_commit(const uint8_t* __restrict__ tab, int k, BArgs A) {
  const BatchView V = batch_view(tab, k);
  const PairDesc* __restrict__ pd = V.pd;
  const Item* __restrict__ it = V.it;
  const int n = V.n, total = V.total;
  for_each_item(it, n, total, [&](int i, Blk bk) {
    const Item& I = it[i];
    commit_body(pd[I.pair].P, pd[I.pair].w, bk);
  });
}

// ---------------------------------------------------------------------------
// NNF update from assigned planes and region plane choice.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Occlusion cue 2 (many-to-one matches): per in-frame target, the assigned
// pixel with the smallest loss keeps its plane, ties to the smallest index.
// Scratch (free between the FB check and the next assignment): tloss holds
// each target's smallest loss as its IEEE bits (losses are >= 0, so the
// unsigned order of the bits is the order of the values), twin the smallest
// index among the pixels with that loss.  Four launches: clear, minimum loss,
// minimum index, apply.
// ---------------------------------------------------------------------------
__device__ inline int unique_target(const DevParams& P, const Ws& w, int dir, int p) {
  const int j = w.win[dir][p];
  if (j < 0) return -1;
  const int W = P.W, Hh = P.H;
  double qx, qy;
  if (!project(w.planes[j].H, (double)(p % W), (double)(p / W), qx, qy)) return -1;
  const double rx = floor(qx + 0.5), ry = floor(qy + 0.5);
  if (!(rx >= 0 && rx <= W - 1 && ry >= 0 && ry <= Hh - 1)) return -1;
  return (int)ry * W + (int)rx;
}

__device__ __forceinline__ void uq_body(const DevParams& P, const Ws& w, Blk bk, int phase) {
  const int p = bk.x * kBlock + threadIdx.x, dir = bk.y;
  if (p >= P.W * P.H) return;
  unsigned long long* best_loss = reinterpret_cast<unsigned long long*>(w.tloss[dir]);
  int* best_p = w.twin[dir];
  if (phase == 0) {
    best_loss[p] = ~0ull;
    best_p[p] = 0x7fffffff;
    return;
  }
  const int q = unique_target(P, w, dir, p);
  if (q < 0) return;
  const unsigned long long key = __double_as_longlong(w.loss[dir][p]);
  if (phase == 1) {
    atomicMin(&best_loss[q], key);
  } else if (phase == 2) {
    if (best_loss[q] == key) atomicMin(&best_p[q], p);
  } else if (best_p[q] != p) {
    w.win[dir][p] = -1;
    w.loss[dir][p] = __builtin_huge_val();
  }
}

__global__ __launch_bounds__(kBlock) void k_unique(DevParams P, Ws w, int phase) { uq_body(P, w, blk_here(), phase); }

__global__ __launch_bounds__(kBlock) void kb_unique(const uint8_t* __restrict__ tab, int k, BArgs A) {
  const BatchView V = batch_view(tab, k);
  const PairDesc* __restrict__ pd = V.pd;
  const Item* __restrict__ it = V.it;
  const int n = V.n, total = V.total;
  for_each_item(it, n, total, [&](int i, Blk bk) {
    uq_body(pd[it[i].pair].P, pd[it[i].pair].w, bk, A.a[0]);
  });
}

// ---------------------------------------------------------------------------
// Filling by homography-model propagation: red-black half-sweeps over the
// unassigned pixels.  Half-sweep t updates colour t % 2 and reads only the
// other colour, so pixels update in place.  Each direction keeps a ring of
// four fill counts: half-sweep t adds into slot t, zeroes slot t + 1 (last
// written by half-sweep t - 3, read by nobody after t - 1) and exits at once
// when slots t - 1 and t - 2 are both zero: two half-sweeps in a row that
// filled nothing leave nothing to fill.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void fill_clear_body(const Ws& w) {
  if (threadIdx.x < 8) w.act_count[8 + threadIdx.x] = 0;
}

__device__ __forceinline__ void fill_body(const DevParams& P, const Ws& w, Blk bk, int t) {
  const int dir = bk.y, W = P.W, Hh = P.H;
  unsigned* ring = w.act_count + 8 + 4 * dir;
  if (bk.x == 0 && threadIdx.x == 0) ring[(t + 1) & 3] = 0;
  if (t >= 2 && ring[(t - 1) & 3] == 0 && ring[(t - 2) & 3] == 0) return;  // uniform over the workgroup
  const int p = bk.x * kBlock + threadIdx.x;
  int filled = 0;
  if (p < W * Hh) {
    const int x = p % W, y = p / W;
    int32_t* win = w.win[dir];
    if (((x + y) & 1) == (t & 1) && win[p] == -1) {
      int best = -1;
      double be = __builtin_huge_val();
      const int nx[4] = {x - 1, x + 1, x, x}, ny[4] = {y, y, y - 1, y + 1};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (nx[k] < 0 || nx[k] >= W || ny[k] < 0 || ny[k] >= Hh) continue;
        const int j = win[ny[k] * W + nx[k]];
        if (j == -1) continue;
        const int plane = j >= 0 ? j : -2 - j;
        const double e = colour_err(P, w, dir, x, y, w.planes[plane].H);
        if (e < be || (e == be && plane < best)) {
          be = e;
          best = plane;
        }
      }
      if (best >= 0 && be < P.eps2) {
        win[p] = -2 - best;
        w.loss[dir][p] = be;
        filled = 1;
      }
    }
  }
  const int n = __syncthreads_count(filled);
  if (threadIdx.x == 0 && n) atomicAdd(&ring[t & 3], (unsigned)n);
}

__global__ __launch_bounds__(kBlock) void k_fill_clear(Ws w) { fill_clear_body(w); }
__global__ __launch_bounds__(kBlock) void k_fill(DevParams P, Ws w, int t) { fill_body(P, w, blk_here(), t); }

__global__ __launch_bounds__(kBlock) void kb_fill_clear(const uint8_t* __restrict__ tab, int k, BArgs A) {
  const BatchView V = batch_view(tab, k);
  const PairDesc* __restrict__ pd = V.pd;
  const Item* __restrict__ it = V.it;
  const int n = V.n, total = V.total;
  for_each_item(it, n, total, [&](int i, Blk bk) {
    fill_clear_body(pd[it[i].pair].w);
  });
}

__global__ __launch_bounds__(kBlock) void kb_fill(const uint8_t* __restrict__ tab, int k, BArgs A) {
  const BatchView V = batch_view(tab, k);
  const PairDesc* __restrict__ pd = V.pd;
  const Item* __restrict__ it = V.it;
  const int n = V.n, total = V.total;
  for_each_item(it, n, total, [&](int i, Blk bk) {
    fill_body(pd[it[i].pair].P, pd[it[i].pair].w, bk, A.a[0]);
  });
}

__device__ __forceinline__ void nnf_update_body(const DevParams& P, const Ws& w, Blk bk, int level) {
  const int p = bk.x * kBlock + threadIdx.x, dir = bk.y;
  const int W = P.W, Hh = P.H;
  if (p >= W * Hh) return;
  const int x = p % W, y = p / W;
  const int j = w.win[dir][p];
  if (j >= 0) {
    double qx, qy;
    if (project(w.planes[j].H, x, y, qx, qy)) {
      // round, then clamp in FP64: no projection is converted to int out of range
      const double fx = fmin(fmax(floor(qx + 0.5), 0.0), (double)(W - 1));
      const double fy = fmin(fmax(floor(qy + 0.5), 0.0), (double)(Hh - 1));
      w.nnf[dir][p] = pack_off((int)fx - x, (int)fy - y);
    }
  }
  const int B = P.block[level], nbx = P.nbx[level], nby = P.nby[level];
  int xlo, xhi, ylo, yhi;
  cover_range(W, B, nbx, x, xlo, xhi);
  cover_range(Hh, B, nby, y, ylo, yhi);
  int best = -1, bestc = -1;
  for (int stage = 1; stage <= 2; ++stage)
    for (int by = ylo; by <= yhi; ++by)
      for (int bx = xlo; bx <= xhi; ++bx) {
        const int k = plane_index(P, dir, level, stage, by * nbx + bx);
        const msgpm_plane& pk = w.planes[k];
        if (!pk.valid) continue;
        if (pk.count > bestc) {
          bestc = pk.count;
          best = k;
        }
      }
  if (best >= 0) w.hlabel[dir][p] = best;
}

__global__ __launch_bounds__(kBlock) void k_nnf_update(DevParams P, Ws w, int level) {
  nnf_update_body(P, w, blk_here(), level);
}

__global__ __launch_bounds__(kBlock) void kb_nnf_update(const uint8_t* __restrict__ tab, int k, BArgs A) {
  const BatchView V = batch_view(tab, k);
  const PairDesc* __restrict__ pd = V.pd;
  const Item* __restrict__ it = V.it;
  const int n = V.n, total = V.total;
  for_each_item(it, n, total, [&](int i, Blk bk) {
    const Item& I = it[i];
    nnf_update_body(pd[I.pair].P, pd[I.pair].w, bk, A.a[0]);
  });
}

__device__ __forceinline__ void finalize_body(const DevParams& P, const Ws& w, Blk bk, float* flow0, float* flow1,
                                              uint8_t* occ0, uint8_t* occ1) {
  const int p = bk.x * kBlock + threadIdx.x, dir = bk.y;
  const int W = P.W;
  if (p >= W * P.H) return;
  const int x = p % W, y = p / W;
  float* flow = dir ? flow1 : flow0;
  uint8_t* occ = dir ? occ1 : occ0;
  const int j = w.win[dir][p];
  const int plane = j >= 0 ? j : -2 - j;  // j <= -2: filled
  double qx, qy;
  if (j != -1 && project(w.planes[plane].H, x, y, qx, qy)) {
    if (flow) {
      flow[2 * p] = (float)(qx - x);
      flow[2 * p + 1] = (float)(qy - y);
    }
    if (occ) occ[p] = j >= 0 ? 0 : 2;
  } else {
    const int32_t v = w.nnf[dir][p];
    if (flow) {
      flow[2 * p] = (float)off_dx(v);
      flow[2 * p + 1] = (float)off_dy(v);
    }
    if (occ) occ[p] = 1;
  }
}

__global__ __launch_bounds__(kBlock) void k_finalize(DevParams P, Ws w, float* flow0, float* flow1, uint8_t* occ0,
                                                    uint8_t* occ1) {
  finalize_body(P, w, blk_here(), flow0, flow1, occ0, occ1);
}

__global__ __launch_bounds__(kBlock) void kb_finalize(const uint8_t* __restrict__ tab, int k, BArgs A) {
  const BatchView V = batch_view(tab, k);
  const PairDesc* __restrict__ pd = V.pd;
  const Item* __restrict__ it = V.it;
  const int n = V.n, total = V.total;
  for_each_item(it, n, total, [&](int i, Blk bk) {
    const PairDesc& D = pd[it[i].pair];
    finalize_body(D.P, D.w, bk, D.flow[0], D.flow[1], D.occ[0], D.occ[1]);
  });
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static dim3 pixel_grid(const DevParams& P) { return dim3((P.W * P.H + kBlock - 1) / kBlock, 2); }

// Points of the largest window a RANSAC launch with this dynamic LDS serves.
static size_t ransac_points(size_t lds) { return (lds - kAuxDoubles * sizeof(double)) / (2 * sizeof(uint32_t)); }

size_t ransac_smem_bytes(const DevParams& P, int level) {
  const int B = P.block[level];
  const int bw = B < P.W ? B : P.W, bh = B < P.H ? B : P.H;
  const size_t n = (size_t)bw * bh;
  return kAuxDoubles * sizeof(double) + 2 * n * sizeof(uint32_t);
}

size_t ransac_smem_bytes_window(int B) { return kAuxDoubles * sizeof(double) + 2 * (size_t)B * B * sizeof(uint32_t); }

hipError_t launch_ransac(const DevParams& P, const Ws& w, int level, int stage, hipStream_t s) {
  const size_t sm = ransac_smem_bytes(P, level);
  const dim3 grid(P.nbx[level] * P.nby[level], 2);
  hipError_t e;
  if (ransac_points(sm) > kRansacWide) {
    if ((e = ransac_lds(&k_ransac<8>, sm)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_ransac<8>, grid, dim3(kBlock), sm, s, P, w, level, stage);
  } else {
    if ((e = ransac_lds(&k_ransac<4>, sm)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_ransac<4>, grid, dim3(kBlock), sm, s, P, w, level, stage);
  }
  return hipGetLastError();
}

hipError_t launch_assign(const DevParams& P, const Ws& w, int level, int stage, int tentative, hipStream_t s) {
  hipLaunchKernelGGL(k_assign, pixel_grid(P), dim3(kBlock), 0, s, P, w, level, stage, tentative);
  return hipGetLastError();
}

hipError_t launch_symmetry(const DevParams& P, const Ws& w, int level, int stage, hipStream_t s) {
  hipLaunchKernelGGL(k_symmetry, dim3(P.nbx[level] * P.nby[level], 2), dim3(kBlock), 0, s, P, w, level, stage);
  return hipGetLastError();
}

hipError_t launch_fb_unassign(const DevParams& P, const Ws& w, hipStream_t s) {
  hipLaunchKernelGGL(k_fb, pixel_grid(P), dim3(kBlock), 0, s, P, w);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_commit, pixel_grid(P), dim3(kBlock), 0, s, P, w);
  return hipGetLastError();
}

hipError_t launch_unique(const DevParams& P, const Ws& w, hipStream_t s) {
  for (int phase = 0; phase < 4; ++phase) {
    hipLaunchKernelGGL(k_unique, pixel_grid(P), dim3(kBlock), 0, s, P, w, phase);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_fill(const DevParams& P, const Ws& w, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_clear, dim3(1), dim3(kBlock), 0, s, w);
  hipError_t e = hipGetLastError();
  for (int t = 0; t < P.fill_sweeps && e == hipSuccess; ++t) {
    hipLaunchKernelGGL(k_fill, pixel_grid(P), dim3(kBlock), 0, s, P, w, t);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_nnf_update(const DevParams& P, const Ws& w, int level, hipStream_t s) {
  hipLaunchKernelGGL(k_nnf_update, pixel_grid(P), dim3(kBlock), 0, s, P, w, level);
  return hipGetLastError();
}

hipError_t launch_finalize(const DevParams& P, const Ws& w, float* flow0, float* flow1, uint8_t* occ0,
                           uint8_t* occ1, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, pixel_grid(P), dim3(kBlock), 0, s, P, w, flow0, flow1, occ0, occ1);
  return hipGetLastError();
}

hipError_t launch_batched_planes(int kind, const uint8_t* tab, int k, int ngrid, size_t lds, BArgs A,
                                 hipStream_t s) {
  const dim3 grid(ngrid, batch_grid_y(kind)), block(kBlock);
  switch (kind) {
    case BK_RANSAC: {
      hipError_t e;
      if (ransac_points(lds) > kRansacWide) {
        if ((e = ransac_lds(&kb_ransac<8>, lds)) != hipSuccess) return e;
        hipLaunchKernelGGL(kb_ransac<8>, grid, block, lds, s, tab, k, A);
      } else {
        if ((e = ransac_lds(&kb_ransac<4>, lds)) != hipSuccess) return e;
        hipLaunchKernelGGL(kb_ransac<4>, grid, block, lds, s, tab, k, A);
      }
      break;
    }
    case BK_ASSIGN:
      hipLaunchKernelGGL(kb_assign, grid, block, 0, s, tab, k, A);
      break;
    case BK_SYMMETRY:
      hipLaunchKernelGGL(kb_symmetry, grid, block, 0, s, tab, k, A);
      break;
    case BK_FB:
      hipLaunchKernelGGL(kb_fb, grid, block, 0, s, tab, k, A);
      break;
    case BK_COMMIT:
      hipLaunchKernelGGL(kb_commit, grid, block, 0, s, tab, k, A);
      break;
    case BK_NNF_UPDATE:
      hipLaunchKernelGGL(kb_nnf_update, grid, block, 0, s, tab, k, A);
      break;
    case BK_FINALIZE:
      hipLaunchKernelGGL(kb_finalize, grid, block, 0, s, tab, k, A);
      break;
    case BK_UNIQUE:
      hipLaunchKernelGGL(kb_unique, grid, block, 0, s, tab, k, A);
      break;
    case BK_FILL_CLEAR:
      hipLaunchKernelGGL(kb_fill_clear, grid, block, 0, s, tab, k, A);
      break;
    case BK_FILL:
      hipLaunchKernelGGL(kb_fill, grid, block, 0, s, tab, k, A);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int pm_batch_blocks(int kind, const DevParams& P, const int* a);

int batch_grid_y(int kind) {
  return (kind == BK_INIT_PLANES || kind == BK_ZERO_ACTIVE || kind == BK_FILL_CLEAR || kind == BK_HEQ_CLEAR) ? 1 : 2;
}

int batch_blocks(int kind, const DevParams& P, const int* a) {
  const int px = (P.W * P.H + kBlock - 1) / kBlock;
  switch (kind) {
    case BK_HEQ_CLEAR:
    case BK_HEQ_MAP:
      return 1;
    case BK_HEQ_HIST:
      return heq_hist_blocks(P);
    case BK_FEATURES:
      return (P.W * P.H + 1 + kBlock - 1) / kBlock;
    case BK_FILL_CLEAR:
      return 1;
    case BK_INIT_PLANES: {
      const int np = 2 * P.planes_per_dir;
      return ((np > kBlock ? np : kBlock) + kBlock - 1) / kBlock;
    }
    case BK_RANSAC:
    case BK_SYMMETRY:
      return P.nbx[a[0]] * P.nby[a[0]];
    case BK_EVAL_COST_IDENT:
    case BK_EVAL_COST_PLANE:
    case BK_ZERO_ACTIVE:
    case BK_ACTIVE_LIST:
    case BK_PM_INIT:
    case BK_PM_RESTRICTED:
    case BK_PM_RESTRICTED_IDENT:
      return pm_batch_blocks(kind, P, a);
    default:
      return px;
  }
}

hipError_t launch_batched(int kind, const DevParams& P0, const uint8_t* tab, int k, int grid, size_t lds, BArgs A,
                          bool persist, hipStream_t s) {
  switch (kind) {
    case BK_HEQ_CLEAR:
    case BK_HEQ_HIST:
    case BK_HEQ_MAP:
    case BK_FEATURES:
    case BK_INIT_PIXELS:
    case BK_INIT_PLANES:
      return launch_batched_init(kind, tab, k, grid, A, s);
    case BK_EVAL_COST_IDENT:
    case BK_EVAL_COST_PLANE:
    case BK_ZERO_ACTIVE:
    case BK_ACTIVE_LIST:
    case BK_PM_INIT:
    case BK_PM_RESTRICTED:
    case BK_PM_RESTRICTED_IDENT:
      return launch_batched_pm(kind, P0, tab, k, grid, A, persist, s);
    default:
      return launch_batched_planes(kind, tab, k, grid, lds, A, s);
  }
}

}  // namespace msgpm
