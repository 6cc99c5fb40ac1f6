/*
 * FP64 CPU oracle for the MSGPM hot path.  TEST INFRASTRUCTURE ONLY: see
 * msgpm_oracle.h for the scope rules and the near-tie bands.
 *
 * Section references are to Choi & Banerjee, "Multi-Scale Generalized Plane
 * Match for Optical Flow" (arXiv 1804.03787):
 *   Sec. 3.1.1 Eq. 1-2   homography plane model, colour consistency
 *   Sec. 3.1.2           RANSAC plane detection, half-overlapping windows
 *   Sec. 3.1.3 Eq. 3-4   plane-distortion compensation, truncated loss, overlap rule
 *   Sec. 3.2             residual-region second stage
 *   Sec. 3.3, Alg. 1     multi-scale loop, merge priority, NNF update, restricted PatchMatch
 *   Sec. 3.4             forward-backward plane symmetry, occlusion = no plane,
 *                        the many-to-one and RANSAC/colour-overlap cues
 *   Sec. 3.4.1           filling by homography-model propagation
 *   Sec. 4               experiment set-up (PatchMatch init, levels, FB per level)
 *   Sec. 4.2             histogram equalisation of the frames in HSV
 * PatchMatch itself (propagation + random search) is the method of Barnes et al.
 * 2009 that the paper builds on (Sec. 1, Sec. 3.1).
 *
 * Where the paper is silent the readings R1-R25 of the design notes apply; each
 * function names the ones it follows.
 */
#include "msgpm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TIE_REL 1e-9

int orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
static int imin(int a, int b) { return a < b ? a : b; }

static int32_t pack_off(int dx, int dy) {
  return (int32_t)(((uint32_t)dx & 0xffffu) | ((uint32_t)dy << 16));
}
static int unpack_dx(int32_t v) { return (int16_t)((uint32_t)v & 0xffffu); }
static int unpack_dy(int32_t v) { return (int16_t)((uint32_t)v >> 16); }

/* ------------------------------------------------------------------------ */
/* Philox4x64-10, from the published definition of the Philox family:       */
/* two 64x64->128 multiplies per round, key schedule by Weyl increments.    */
/* ------------------------------------------------------------------------ */
void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    unsigned __int128 p0 = (unsigned __int128)M0 * c0;
    unsigned __int128 p1 = (unsigned __int128)M1 * c2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

uint32_t orc_draw(uint64_t word, uint32_t n) {
  return (uint32_t)(((word >> 32) * (uint64_t)n) >> 32);
}

/* Random block for (element, draw, iteration, phase, dir, slot, stage). */
static void rng_block(const orc_pair* S, uint64_t elem, uint64_t draw, uint64_t iter,
                      int phase, int dir, int slot, int stage, uint64_t out[4]) {
  uint64_t ctr[4] = {elem, draw, iter,
                     ((uint64_t)phase << 24) | ((uint64_t)dir << 16) | ((uint64_t)slot << 8) | (uint64_t)stage};
  uint64_t key[2] = {S->seed, 0};
  orc_philox4x64(ctr, key, out);
}

/* ------------------------------------------------------------------------ */
/* Features (O1).  RGB as given; optional luma gradients (reading R20).      */
/* ------------------------------------------------------------------------ */
float orc_round_fp16(float x) {
  /* Nearest binary16 value (ties to even), widened back to binary32.  binary16
     keeps 11 significant bits for magnitudes >= 2^-14 and a fixed spacing of
     2^-24 below that; the largest finite value is 65504. */
  if (!isfinite(x) || x == 0.0f) return x;
  double a = fabs((double)x);
  int e;
  frexp(a, &e); /* a = m * 2^e with m in [0.5, 1): leading bit has weight 2^(e-1) */
  int lead = e - 1;
  if (lead < -14) lead = -14;
  double q = ldexp(1.0, lead - 10);   /* spacing of binary16 values near a */
  double r = nearbyint(a / q) * q;    /* a / q is exact; default mode rounds half to even */
  if (r > 65504.0) r = INFINITY;
  return (float)copysign(r, (double)x);
}

void orc_features(const float* rgb, int W, int H, int C, int fp16, float* feat) {
  const int n = W * H;
  float* Y = NULL;
  if (C == 5) Y = (float*)malloc(sizeof(float) * (size_t)n);
  for (int p = 0; p < n; ++p) {
    float R = rgb[3 * p], G = rgb[3 * p + 1], B = rgb[3 * p + 2];
    feat[C * p + 0] = R;
    feat[C * p + 1] = G;
    feat[C * p + 2] = B;
    if (Y) {
      float t = 0.299f * R;
      float u = 0.587f * G;
      float s = t + u;
      float v = 0.114f * B;
      Y[p] = s + v;
    }
  }
  if (Y) {
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) {
        int p = y * W + x;
        float gx = 0.5f * (Y[y * W + imin(x + 1, W - 1)] - Y[y * W + (x > 0 ? x - 1 : 0)]);
        float gy = 0.5f * (Y[imin(y + 1, H - 1) * W + x] - Y[(y > 0 ? y - 1 : 0) * W + x]);
        feat[C * p + 3] = gx;
        feat[C * p + 4] = gy;
      }
    free(Y);
  }
  if (fp16)
    for (int i = 0; i < n * C; ++i) feat[i] = orc_round_fp16(feat[i]);
}

/* ------------------------------------------------------------------------ */
/* Histogram equalisation of the value channel in HSV (Sec. 4.2; reading     */
/* R35).  V = max(R, G, B) is binned to 256 levels; level q is mapped to      */
/* (cdf(q) - cdf_min) / (n - cdf_min), cdf_min being the count of the lowest  */
/* occupied level.  Changing V alone in HSV scales R, G, B by V' / V; a pixel */
/* with V <= 0 has no hue or saturation and becomes grey V'.  A frame whose   */
/* pixels all share one level is left as it is.                              */
/* ------------------------------------------------------------------------ */
static int v_level(float V) {
  const float t = V * 255.0f + 0.5f;
  if (!(t >= 0.0f)) return 0;
  if (t >= 255.0f) return 255;
  return (int)t; /* t >= 0: truncation is the floor */
}

void orc_histeq(const float* rgb, int W, int H, float* out) {
  const int64_t n = (int64_t)W * H;
  int64_t hist[256] = {0};
  for (int64_t p = 0; p < n; ++p) {
    const float V = fmaxf(fmaxf(rgb[3 * p], rgb[3 * p + 1]), rgb[3 * p + 2]);
    ++hist[v_level(V)];
  }
  int64_t cdf[256], run = 0, cdf_min = 0;
  for (int q = 0; q < 256; ++q) {
    run += hist[q];
    cdf[q] = run;
    if (cdf_min == 0) cdf_min = run;
  }
  if (cdf_min == n) {
    memcpy(out, rgb, sizeof(float) * 3 * (size_t)n);
    return;
  }
  float lut[256];
  for (int q = 0; q < 256; ++q)
    lut[q] = cdf[q] < cdf_min ? 0.0f : (float)((double)(cdf[q] - cdf_min) / (double)(n - cdf_min));
  for (int64_t p = 0; p < n; ++p) {
    const float R = rgb[3 * p], G = rgb[3 * p + 1], B = rgb[3 * p + 2];
    const float V = fmaxf(fmaxf(R, G), B);
    const float Vn = lut[v_level(V)];
    if (V > 0.0f) {
      const float s = Vn / V;
      out[3 * p] = R * s;
      out[3 * p + 1] = G * s;
      out[3 * p + 2] = B * s;
    } else {
      out[3 * p] = out[3 * p + 1] = out[3 * p + 2] = Vn;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Homography (Eq. 1, reading R3: H maps source pixel -> target pixel).      */
/* ------------------------------------------------------------------------ */
int orc_project(const double* Hm, double x, double y, double* qx, double* qy) {
  double w = Hm[6] * x + Hm[7] * y + Hm[8];
  if (!(w > 0)) return 0;
  *qx = (Hm[0] * x + Hm[1] * y + Hm[2]) / w;
  *qy = (Hm[3] * x + Hm[4] * y + Hm[5]) / w;
  return 1;
}

static const double IDENT[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};

/* Bilinear sample of channels [0, nch) of F at integer base (bx, by) plus
   fraction (fx, fy), with the border rule of O3 (reading R17). */
static void sample(const float* F, int W, int H, int C, int nch, int bx, int by, double fx, double fy,
                   double* out) {
  if (bx < 0) { bx = 0; fx = 0; } else if (bx >= W - 1) { bx = W - 1; fx = 0; }
  if (by < 0) { by = 0; fy = 0; } else if (by >= H - 1) { by = H - 1; fy = 0; }
  int x1 = imin(bx + 1, W - 1), y1 = imin(by + 1, H - 1);
  const float* a = F + (size_t)C * (by * W + bx);
  const float* b = F + (size_t)C * (by * W + x1);
  const float* c = F + (size_t)C * (y1 * W + bx);
  const float* d = F + (size_t)C * (y1 * W + x1);
  for (int k = 0; k < nch; ++k)
    out[k] = (1 - fy) * ((1 - fx) * (double)a[k] + fx * (double)b[k]) +
             fy * ((1 - fx) * (double)c[k] + fx * (double)d[k]);
}

/* ------------------------------------------------------------------------ */
/* Warped-patch SSD (O3): the square patch of p in the source frame against  */
/* the patch of target t in the other frame, whose taps are displaced by the  */
/* local distortion of H around p (Sec. 3.1.3: compensate the plane          */
/* distortion into the patch comparison; reading R8: SSD over features).     */
/* ------------------------------------------------------------------------ */
double orc_cost(const orc_pair* S, int dir, int px, int py, int tx, int ty, const double* Hm) {
  const float* F1 = S->F[dir];
  const float* F2 = S->F[1 - dir];
  const int W = S->W, H = S->H, C = S->C, r = S->r;
  if (!Hm) Hm = IDENT;
  double cx, cy;
  if (!orc_project(Hm, px, py, &cx, &cy)) return INFINITY;
  const double lim = 4.0 * (double)(W > H ? W : H);
  double sum = 0;
  double v[5];
  for (int dy = -r; dy <= r; ++dy)
    for (int dx = -r; dx <= r; ++dx) {
      double sx, sy;
      if (!orc_project(Hm, px + dx, py + dy, &sx, &sy)) return INFINITY;
      double Dx = sx - cx, Dy = sy - cy; /* displacement of tap d under H */
      if (Dx < -lim) Dx = -lim; else if (Dx > lim) Dx = lim;
      if (Dy < -lim) Dy = -lim; else if (Dy > lim) Dy = lim;
      double flx = floor(Dx), fly = floor(Dy);
      sample(F2, W, H, C, C, tx + (int)flx, ty + (int)fly, Dx - flx, Dy - fly, v);
      const float* f1 = F1 + (size_t)C * (clampi(py + dy, 0, H - 1) * W + clampi(px + dx, 0, W - 1));
      for (int c = 0; c < C; ++c) {
        double d = (double)f1[c] - v[c];
        sum += S->wc[c] * d * d;
      }
    }
  return sum;
}

void orc_cost_all(const orc_pair* S, int dir, double* out) {
  const int n = S->W * S->H;
  for (int p = 0; p < n; ++p)
    for (int t = 0; t < n; ++t)
      out[(size_t)p * n + t] = orc_cost(S, dir, p % S->W, p / S->W, t % S->W, t / S->W, NULL);
}

/* ------------------------------------------------------------------------ */
/* Blocks (O6; Sec. 3.1.2 half-ratio overlap, reading R1) and plane table.   */
/* ------------------------------------------------------------------------ */
int orc_block_count(int n, int B) {
  if (n <= B) return 1;
  int S = B / 2;
  int m = (n - B) / S + 1;
  if ((n - B) % S) ++m;
  return m;
}

int orc_block_origin(int n, int B, int i) {
  if (n <= B) return 0;
  int o = i * (B / 2);
  return o > n - B ? n - B : o;
}

static int level_blocks(const orc_pair* S, int l) {
  return orc_block_count(S->W, S->block[l]) * orc_block_count(S->H, S->block[l]);
}

int orc_plane_capacity(const orc_pair* S) {
  int t = 0;
  for (int l = 0; l < S->n_levels; ++l) t += level_blocks(S, l);
  return 4 * t;
}

int orc_plane_index(const orc_pair* S, int dir, int level, int stage, int block) {
  int off = 0, tot = 0;
  for (int l = 0; l < S->n_levels; ++l) {
    if (l < level) off += level_blocks(S, l);
    tot += level_blocks(S, l);
  }
  return dir * 2 * tot + 2 * off + (stage - 1) * level_blocks(S, level) + block;
}

int orc_m_min(const orc_pair* S, int bw, int bh) {
  int m = (int)ceil(S->mu * (double)bw * (double)bh);
  return m > S->m_min_abs ? m : S->m_min_abs;
}

void orc_planes_init(orc_pair* S) {
  for (int dir = 0; dir < 2; ++dir)
    for (int l = 0; l < S->n_levels; ++l) {
      int B = S->block[l];
      int nbx = orc_block_count(S->W, B), nby = orc_block_count(S->H, B);
      for (int stage = 1; stage <= 2; ++stage)
        for (int by = 0; by < nby; ++by)
          for (int bx = 0; bx < nbx; ++bx) {
            int b = by * nbx + bx;
            int k = orc_plane_index(S, dir, l, stage, b);
            int32_t* I = S->pinfo + (size_t)k * ORC_PI_N;
            memset(I, 0, sizeof(int32_t) * ORC_PI_N);
            I[ORC_PI_DIR] = dir;
            I[ORC_PI_LEVEL] = l;
            I[ORC_PI_STAGE] = stage;
            I[ORC_PI_BLOCK] = b;
            I[ORC_PI_X0] = orc_block_origin(S->W, B, bx);
            I[ORC_PI_Y0] = orc_block_origin(S->H, B, by);
            I[ORC_PI_BW] = imin(B, S->W);
            I[ORC_PI_BH] = imin(B, S->H);
            I[ORC_PI_HYP] = -1;
            for (int j = 0; j < 9; ++j) S->pH[(size_t)k * 9 + j] = 0;
            if (S->bflag) S->bflag[k] = 0;
          }
    }
}

static const int32_t* pinfo_of(const orc_pair* S, int k) { return S->pinfo + (size_t)k * ORC_PI_N; }
static const double* H_of(const orc_pair* S, int k) { return S->pH + (size_t)k * 9; }

/* ------------------------------------------------------------------------ */
/* O4: random initial NNF (reading R19).                                     */
/* ------------------------------------------------------------------------ */
void orc_nnf_init(orc_pair* S, int dir) {
  const int W = S->W, H = S->H;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      uint64_t u[4];
      rng_block(S, (uint64_t)(y * W + x), 0, 0, 1, dir, 0, 0, u);
      int tx = (int)orc_draw(u[0], (uint32_t)W);
      int ty = (int)orc_draw(u[1], (uint32_t)H);
      S->nnf[dir][y * W + x] = pack_off(tx - x, ty - y);
    }
}

static const double* region_H(const orc_pair* S, int label) { return label >= 0 ? H_of(S, label) : IDENT; }

void orc_eval_cost(orc_pair* S, int dir, int mode) {
  const int W = S->W, H = S->H;
  int64_t evals = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : evals)
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      int p = y * W + x;
      const double* Hm;
      if (mode == 0) Hm = IDENT;
      else if (mode == 1) {
        if (S->win[dir][p] >= 0) continue;
        Hm = region_H(S, S->hlabel[dir][p]);
      } else {
        if (S->win[dir][p] < 0) continue;
        Hm = H_of(S, S->win[dir][p]);
      }
      int32_t v = S->nnf[dir][p];
      S->cost[dir][p] = orc_cost(S, dir, x, y, x + unpack_dx(v), y + unpack_dy(v), Hm);
      evals++;
    }
  S->evals += evals;
}

/* ------------------------------------------------------------------------ */
/* O5: PatchMatch half-sweep (propagation + random search of Barnes et al.,  */
/* red-black Jacobi schedule, reading R16; restricted pass of Sec. 3.3.2     */
/* with the region distortion and one plane candidate, readings R14/R15).    */
/* ------------------------------------------------------------------------ */
static int near_cost(const orc_pair* S, double a, double b) {
  if (!isfinite(a) || !isfinite(b)) return 0;
  double m = a > b ? a : b;
  double fl = 1e-7 * (double)((2 * S->r + 1) * (2 * S->r + 1) * S->C);
  return fabs(a - b) <= 1e-5 * m + fl;
}

static int near_half(double q) {
  double f = q - floor(q);
  return fabs(f - 0.5) <= TIE_REL;
}

/* Running state of one pixel's update: the best target and its cost, the
   second-best cost over distinct targets, near-tie flags, evaluations. */
typedef struct {
  int tx, ty;
  double c, c2;
  int flag;
  int64_t evals;
} pm_best;

static void pm_try(const orc_pair* S, int dir, int px, int py, int tx, int ty, const double* Hm, pm_best* b) {
  if (tx == b->tx && ty == b->ty) return; /* same target: same cost, never strictly better */
  double c = orc_cost(S, dir, px, py, tx, ty, Hm);
  b->evals++;
  if (near_cost(S, c, b->c)) b->flag |= ORC_F_COST;
  if (c < b->c) {
    b->c2 = b->c;
    b->tx = tx;
    b->ty = ty;
    b->c = c;
  } else if (c < b->c2) {
    b->c2 = c;
  }
}

void orc_pm_halfsweep(orc_pair* S, int dir, int colour, int iter, int slot, int restricted) {
  const int W = S->W, H = S->H;
  const int R0 = S->R0 > 0 ? S->R0 : (W > H ? W : H);
  int32_t* nnf = S->nnf[dir];
  int64_t evals = 0;
  /* a pixel of this colour reads only the other colour's offsets and writes
     only its own state, so the rows may be taken in any order */
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : evals)
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      if (((x + y) & 1) != colour) continue;
      int p = y * W + x;
      if (restricted && S->win[dir][p] >= 0) continue;
      const int label = restricted ? S->hlabel[dir][p] : -1;
      const double* Hm = region_H(S, label);
      pm_best b;
      b.tx = x + unpack_dx(nnf[p]);
      b.ty = y + unpack_dy(nnf[p]);
      b.c = S->cost[dir][p];
      b.c2 = INFINITY;
      b.flag = 0;
      b.evals = 0;
      /* propagation from the four in-image neighbours: left, right, up, down */
      const int nx[4] = {x - 1, x + 1, x, x};
      const int ny[4] = {y, y, y - 1, y + 1};
      for (int k = 0; k < 4; ++k) {
        if (nx[k] < 0 || nx[k] >= W || ny[k] < 0 || ny[k] >= H) continue;
        int32_t v = nnf[ny[k] * W + nx[k]];
        pm_try(S, dir, x, y, clampi(x + unpack_dx(v), 0, W - 1), clampi(y + unpack_dy(v), 0, H - 1), Hm, &b);
      }
      /* plane candidate: where the region plane sends p */
      if (restricted && label >= 0) {
        double qx, qy;
        if (orc_project(Hm, x, y, &qx, &qy)) {
          if (near_half(qx) || near_half(qy)) b.flag |= ORC_F_ROUND;
          double rx = floor(qx + 0.5), ry = floor(qy + 0.5);
          double lim = 4.0 * (double)(W > H ? W : H);
          if (rx < -lim) rx = -lim; else if (rx > lim) rx = lim;
          if (ry < -lim) ry = -lim; else if (ry > lim) ry = lim;
          pm_try(S, dir, x, y, clampi((int)rx, 0, W - 1), clampi((int)ry, 0, H - 1), Hm, &b);
        }
      }
      /* random search around the best offset so far, radii R0 * 2^-k */
      const int cdx = b.tx - x, cdy = b.ty - y;
      for (int k = 0; (R0 >> k) >= 1; ++k) {
        const int R = R0 >> k;
        uint64_t u[4];
        rng_block(S, (uint64_t)p, (uint64_t)k, (uint64_t)iter, 2, dir, slot, 0, u);
        int ox = (int)orc_draw(u[0], (uint32_t)(2 * R + 1)) - R;
        int oy = (int)orc_draw(u[1], (uint32_t)(2 * R + 1)) - R;
        pm_try(S, dir, x, y, clampi(x + cdx + ox, 0, W - 1), clampi(y + cdy + oy, 0, H - 1), Hm, &b);
      }
      nnf[p] = pack_off(b.tx - x, b.ty - y);
      S->cost[dir][p] = b.c;
      if (near_cost(S, b.c, b.c2)) b.flag |= ORC_F_TWOBEST;
      if (S->pflag[dir]) S->pflag[dir][p] |= (uint8_t)b.flag;
      evals += b.evals;
    }
  S->evals += evals;
}

/* ------------------------------------------------------------------------ */
/* Linear algebra for the plane fit (Sec. 3.1.1: least squares from 4        */
/* correspondences, reading R4).                                             */
/* ------------------------------------------------------------------------ */
int orc_gauss_solve(double* A, double* b, int n, double* x) {
  for (int k = 0; k < n; ++k) {
    int piv = k;
    double best = fabs(A[k * n + k]);
    for (int i = k + 1; i < n; ++i)
      if (fabs(A[i * n + k]) > best) {
        best = fabs(A[i * n + k]);
        piv = i;
      }
    if (best < 1e-10) return 0;
    if (piv != k) {
      for (int j = 0; j < n; ++j) {
        double t = A[k * n + j];
        A[k * n + j] = A[piv * n + j];
        A[piv * n + j] = t;
      }
      double t = b[k];
      b[k] = b[piv];
      b[piv] = t;
    }
    for (int i = k + 1; i < n; ++i) {
      double f = A[i * n + k] / A[k * n + k];
      for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
      b[i] -= f * b[k];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = b[i];
    for (int j = i + 1; j < n; ++j) s -= A[i * n + j] * x[j];
    x[i] = s / A[i * n + i];
  }
  return 1;
}

/* Hartley normalisation: centroid to the origin, mean distance sqrt(2). */
static int hartley(const double* x, const double* y, int n, double* s, double* cx, double* cy) {
  double sx = 0, sy = 0;
  for (int i = 0; i < n; ++i) {
    sx += x[i];
    sy += y[i];
  }
  *cx = sx / n;
  *cy = sy / n;
  double md = 0;
  for (int i = 0; i < n; ++i) {
    double ex = x[i] - *cx, ey = y[i] - *cy;
    md += sqrt(ex * ex + ey * ey);
  }
  md = md / n;
  if (!(md > 0)) return 0;
  *s = sqrt(2.0) / md;
  return 1;
}

/* H = Td^-1 * Hn * Ts, then scaled so that H[8] = 1. */
static int denormalise(const double* h8, double s1, double c1x, double c1y, double s2, double c2x, double c2y,
                       double* Hout) {
  const double Hn[9] = {h8[0], h8[1], h8[2], h8[3], h8[4], h8[5], h8[6], h8[7], 1.0};
  const double Ts[9] = {s1, 0, -s1 * c1x, 0, s1, -s1 * c1y, 0, 0, 1};
  const double Ti[9] = {1.0 / s2, 0, c2x, 0, 1.0 / s2, c2y, 0, 0, 1};
  double M[9], R[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double t = 0;
      for (int k = 0; k < 3; ++k) t += Hn[i * 3 + k] * Ts[k * 3 + j];
      M[i * 3 + j] = t;
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double t = 0;
      for (int k = 0; k < 3; ++k) t += Ti[i * 3 + k] * M[k * 3 + j];
      R[i * 3 + j] = t;
    }
  if (fabs(R[8]) < 1e-12) return 0;
  const double d = R[8];
  for (int i = 0; i < 9; ++i) Hout[i] = R[i] / d;
  return 1;
}

int orc_dlt4(const double* sx, const double* sy, const double* dx, const double* dy, double* Hout) {
  double s1, c1x, c1y, s2, c2x, c2y;
  if (!hartley(sx, sy, 4, &s1, &c1x, &c1y)) return 0;
  if (!hartley(dx, dy, 4, &s2, &c2x, &c2y)) return 0;
  double A[64], b[8], h[8];
  for (int i = 0; i < 4; ++i) {
    double x = s1 * (sx[i] - c1x), y = s1 * (sy[i] - c1y);
    double u = s2 * (dx[i] - c2x), v = s2 * (dy[i] - c2y);
    double* r0 = A + (2 * i) * 8;
    double* r1 = A + (2 * i + 1) * 8;
    r0[0] = x; r0[1] = y; r0[2] = 1; r0[3] = 0; r0[4] = 0; r0[5] = 0; r0[6] = -x * u; r0[7] = -y * u;
    r1[0] = 0; r1[1] = 0; r1[2] = 0; r1[3] = x; r1[4] = y; r1[5] = 1; r1[6] = -x * v; r1[7] = -y * v;
    b[2 * i] = u;
    b[2 * i + 1] = v;
  }
  if (!orc_gauss_solve(A, b, 8, h)) return 0;
  return denormalise(h, s1, c1x, c1y, s2, c2x, c2y, Hout);
}

int orc_refit(const double* sx, const double* sy, const double* dx, const double* dy, int n, double* Hout) {
  if (n < 4) return 0;
  double s1, c1x, c1y, s2, c2x, c2y;
  if (!hartley(sx, sy, n, &s1, &c1x, &c1y)) return 0;
  if (!hartley(dx, dy, n, &s2, &c2x, &c2y)) return 0;
  double N[64], rhs[8], h[8];
  memset(N, 0, sizeof N);
  memset(rhs, 0, sizeof rhs);
  for (int i = 0; i < n; ++i) {
    double x = s1 * (sx[i] - c1x), y = s1 * (sy[i] - c1y);
    double u = s2 * (dx[i] - c2x), v = s2 * (dy[i] - c2y);
    const double a0[8] = {x, y, 1, 0, 0, 0, -x * u, -y * u};
    const double a1[8] = {0, 0, 0, x, y, 1, -x * v, -y * v};
    for (int j = 0; j < 8; ++j) {
      for (int k = 0; k < 8; ++k) N[j * 8 + k] += a0[j] * a0[k];
      rhs[j] += a0[j] * u;
    }
    for (int j = 0; j < 8; ++j) {
      for (int k = 0; k < 8; ++k) N[j * 8 + k] += a1[j] * a1[k];
      rhs[j] += a1[j] * v;
    }
  }
  if (!orc_gauss_solve(N, rhs, 8, h)) return 0;
  return denormalise(h, s1, c1x, c1y, s2, c2x, c2y, Hout);
}

/* Reprojection inlier test (reading R7), division-free form: w > 0 and
   |(u, v) - w q|^2 < tau^2 w^2, each product-plus-sum rounded once (fma, reading
   R31); *near set when the decision is within the near-tie band. */
static int ransac_inlier(const double* Hm, double x, double y, double qx, double qy, double tau2, int* near) {
  const double w = fma(Hm[6], x, fma(Hm[7], y, Hm[8]));
  if (!(w > 0)) return 0;
  const double u = fma(Hm[0], x, fma(Hm[1], y, Hm[2]));
  const double v = fma(Hm[3], x, fma(Hm[4], y, Hm[5]));
  const double ex = fma(-w, qx, u), ey = fma(-w, qy, v);
  const double e2 = fma(ex, ex, ey * ey);
  const double t = tau2 * w * w;
  if (fabs(e2 - t) <= TIE_REL * t) *near = 1;
  return e2 < t;
}

static int64_t cross3(const int* X, const int* Y, int a, int b, int c) {
  return (int64_t)(X[b] - X[a]) * (Y[c] - Y[a]) - (int64_t)(Y[b] - Y[a]) * (X[c] - X[a]);
}

static int degenerate4(const int* X, const int* Y) {
  static const int tri[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};
  for (int t = 0; t < 4; ++t)
    if (cross3(X, Y, tri[t][0], tri[t][1], tri[t][2]) == 0) return 1;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* O7 / O11: per-block RANSAC (Sec. 3.1.2; residual stage Sec. 3.2;          */
/* readings R5, R6, R7, R9, R12).                                            */
/* ------------------------------------------------------------------------ */
void orc_ransac(orc_pair* S, int dir, int level, int stage) {
  const int W = S->W, H = S->H;
  const int B = S->block[level];
  const int nbx = orc_block_count(W, B), nby = orc_block_count(H, B);
  const int bw = imin(B, W), bh = imin(B, H);
  const double tau2 = S->tau * S->tau;
  /* every window reads the NNF and assignment and writes only its own plane
     record, so the windows may be fitted in any order */
#pragma omp parallel
  {
  int* px = (int*)malloc(sizeof(int) * (size_t)bw * bh * 4);
  int* py = px + bw * bh;
  int* qx = py + bw * bh;
  int* qy = qx + bw * bh;
  double* ax = (double*)malloc(sizeof(double) * (size_t)bw * bh * 4);
  double* ay = ax + bw * bh;
  double* aqx = ay + bw * bh;
  double* aqy = aqx + bw * bh;
  int* cnt = (int*)malloc(sizeof(int) * (size_t)S->hyps * 2);
  int* nties = cnt + S->hyps;
#pragma omp for schedule(dynamic, 1)
  for (int b = 0; b < nbx * nby; ++b) {
    {
      const int k = orc_plane_index(S, dir, level, stage, b);
      int32_t* I = S->pinfo + (size_t)k * ORC_PI_N;
      double* Hk = S->pH + (size_t)k * 9;
      const int x0 = I[ORC_PI_X0], y0 = I[ORC_PI_Y0];
      /* point list in row-major order: (p, p + v_p); stage 2 keeps unassigned pixels */
      int n = 0;
      for (int y = y0; y < y0 + bh; ++y)
        for (int x = x0; x < x0 + bw; ++x) {
          int p = y * W + x;
          if (stage == 2 && S->win[dir][p] >= 0) continue;
          px[n] = x;
          py[n] = y;
          qx[n] = x + unpack_dx(S->nnf[dir][p]);
          qy[n] = y + unpack_dy(S->nnf[dir][p]);
          ax[n] = px[n]; ay[n] = py[n]; aqx[n] = qx[n]; aqy[n] = qy[n];
          ++n;
        }
      const int mmin = orc_m_min(S, bw, bh);
      I[ORC_PI_SUPPORT] = n;
      I[ORC_PI_COUNT] = 0;
      I[ORC_PI_HYP] = -1;
      I[ORC_PI_HYPCOUNT] = 0;
      I[ORC_PI_REFIT] = 0;
      I[ORC_PI_DETECTED] = 0;
      I[ORC_PI_VALID] = 0;
      I[ORC_PI_RK] = 0;
      I[ORC_PI_PASS] = 0;
      I[ORC_PI_RIN] = 0;
      for (int j = 0; j < 9; ++j) Hk[j] = 0;
      if (n < mmin || n < 4) continue;
      int best = -1, bestc = -1;
      double Hbest[9] = {0};
      for (int h = 0; h < S->hyps; ++h) {
        uint64_t u[4];
        rng_block(S, (uint64_t)b, (uint64_t)h, 0, 3, dir, level + 1, stage, u);
        /* partial Fisher-Yates over a virtual identity permutation */
        int key[8], val[8], nm = 0, sel[4];
        for (int j = 0; j < 4; ++j) {
          int rj = j + (int)orc_draw(u[j], (uint32_t)(n - j));
          int vj = j, vr = rj;
          for (int m = 0; m < nm; ++m) {
            if (key[m] == j) vj = val[m];
            if (key[m] == rj) vr = val[m];
          }
          /* swap positions j and rj */
          int fj = -1, fr = -1;
          for (int m = 0; m < nm; ++m) {
            if (key[m] == j) fj = m;
            if (key[m] == rj) fr = m;
          }
          if (fj < 0) { key[nm] = j; fj = nm++; }
          if (fr < 0) { key[nm] = rj; fr = nm++; }
          val[fj] = vr;
          val[fr] = vj;
          sel[j] = vr;
        }
        int SX[4], SY[4], DX[4], DY[4];
        double sx[4], sy[4], dx[4], dy[4];
        for (int j = 0; j < 4; ++j) {
          SX[j] = px[sel[j]]; SY[j] = py[sel[j]]; DX[j] = qx[sel[j]]; DY[j] = qy[sel[j]];
          sx[j] = SX[j]; sy[j] = SY[j]; dx[j] = DX[j]; dy[j] = DY[j];
        }
        cnt[h] = -1;
        nties[h] = 0;
        double Hh[9];
        if (degenerate4(SX, SY) || degenerate4(DX, DY)) continue;
        if (!orc_dlt4(sx, sy, dx, dy, Hh)) continue;
        int c = 0, nt = 0;
        for (int i = 0; i < n; ++i) {
          int near = 0;
          c += ransac_inlier(Hh, ax[i], ay[i], aqx[i], aqy[i], tau2, &near);
          nt += near;
        }
        cnt[h] = c;
        nties[h] = nt;
        if (c > bestc) {
          bestc = c;
          best = h;
          memcpy(Hbest, Hh, sizeof Hbest);
        }
      }
      if (best < 0) continue;
      /* could a near-tie have changed the winning hypothesis? */
      int fragile = 0;
      for (int h = 0; h < S->hyps; ++h) {
        if (h == best || cnt[h] < 0) continue;
        int hi = cnt[h] + nties[h], lo = bestc - nties[best];
        if ((h < best && hi >= lo) || (h > best && hi > lo)) fragile = 1;
      }
      I[ORC_PI_HYP] = best;
      I[ORC_PI_HYPCOUNT] = bestc;
      int final_count = bestc;
      int final_ties = nties[best];
      memcpy(Hk, Hbest, sizeof Hbest);
      /* least-squares refit on the winner's inliers, kept unless it loses support */
      int ni = 0;
      double* rx = (double*)malloc(sizeof(double) * (size_t)n * 4);
      double *ry = rx + n, *rqx = ry + n, *rqy = rqx + n;
      for (int i = 0; i < n; ++i) {
        int near = 0;
        if (ransac_inlier(Hbest, ax[i], ay[i], aqx[i], aqy[i], tau2, &near)) {
          rx[ni] = ax[i]; ry[ni] = ay[i]; rqx[ni] = aqx[i]; rqy[ni] = aqy[i];
          ++ni;
        }
      }
      double Hr[9];
      if (orc_refit(rx, ry, rqx, rqy, ni, Hr)) {
        int cr = 0, nt = 0;
        for (int i = 0; i < n; ++i) {
          int near = 0;
          cr += ransac_inlier(Hr, ax[i], ay[i], aqx[i], aqy[i], tau2, &near);
          nt += near;
        }
        if (abs(cr - bestc) <= nt + nties[best] && nt + nties[best] > 0) fragile |= 2;
        if (cr >= bestc) {
          memcpy(Hk, Hr, sizeof Hr);
          final_count = cr;
          final_ties = nt;
          I[ORC_PI_REFIT] = 1;
        }
      }
      free(rx);
      I[ORC_PI_COUNT] = final_count;
      I[ORC_PI_DETECTED] = final_count >= mmin;
      I[ORC_PI_VALID] = I[ORC_PI_DETECTED];
      if (abs(final_count - mmin) <= final_ties && final_ties > 0) fragile |= 2;
      if (S->bflag) {
        if (fragile & 1) S->bflag[k] |= ORC_F_RANSAC;
        if ((fragile & 2) || final_ties > 0) S->bflag[k] |= 64;
      }
    }
  }
  free(px);
  free(ax);
  free(cnt);
  }
}

/* ------------------------------------------------------------------------ */
/* O8: colour-consistency error e(p, H) (Eq. 3-4 in squared RMS form,        */
/* reading R10).                                                             */
/* ------------------------------------------------------------------------ */
static int near_bound(double q, double hi) { return fabs(q) <= TIE_REL || fabs(q - hi) <= TIE_REL; }

double orc_colour_err(const orc_pair* S, int dir, int px, int py, const double* Hm, int* nb) {
  const int W = S->W, H = S->H, C = S->C;
  double qx, qy;
  if (!orc_project(Hm, px, py, &qx, &qy)) return INFINITY;
  if (nb && (near_bound(qx, W - 1) || near_bound(qy, H - 1))) *nb = 1;
  if (qx < 0 || qx > W - 1 || qy < 0 || qy > H - 1) return INFINITY;
  double fx0 = floor(qx), fy0 = floor(qy);
  double v[3];
  sample(S->F[1 - dir], W, H, C, 3, (int)fx0, (int)fy0, qx - fx0, qy - fy0, v);
  const float* f1 = S->F[dir] + (size_t)C * (py * W + px);
  double e = 0;
  for (int c = 0; c < 3; ++c) {
    double d = (double)f1[c] - v[c];
    e += d * d;
  }
  return e / 3.0;
}

static int h_equiv(const double* A, const double* B) {
  double num = 0, den = 0;
  for (int i = 0; i < 9; ++i) {
    num += (A[i] - B[i]) * (A[i] - B[i]);
    den += B[i] * B[i];
  }
  return num <= 1e-12 * den;
}

/* key (L, level, stage, block): lexicographic, smaller wins (reading R11) */
static int key_less(double L1, const int32_t* I1, double L2, const int32_t* I2) {
  if (L1 != L2) return L1 < L2;
  if (I1[ORC_PI_LEVEL] != I2[ORC_PI_LEVEL]) return I1[ORC_PI_LEVEL] < I2[ORC_PI_LEVEL];
  if (I1[ORC_PI_STAGE] != I2[ORC_PI_STAGE]) return I1[ORC_PI_STAGE] < I2[ORC_PI_STAGE];
  return I1[ORC_PI_BLOCK] < I2[ORC_PI_BLOCK];
}

/* Covering range of block indices along one axis for pixel coordinate c. */
static void cover_range(int n, int B, int c, int* lo, int* hi) {
  int m = orc_block_count(n, B);
  *lo = m;
  *hi = -1;
  for (int i = 0; i < m; ++i) {
    int o = orc_block_origin(n, B, i);
    if (o <= c && c < o + imin(B, n)) {
      if (i < *lo) *lo = i;
      *hi = i;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* O9: assignment with the overlap / multi-level merge rule (Sec. 3.1.3,     */
/* Sec. 3.3; readings R11, R12).                                             */
/* ------------------------------------------------------------------------ */
void orc_assign(orc_pair* S, int dir, int level, int stage, int tentative) {
  const int W = S->W, H = S->H;
  const int B = S->block[level];
  const int nbx = orc_block_count(W, B);
  const double eps2 = S->eps * S->eps;
  int32_t* out_win = tentative ? S->twin[dir] : S->win[dir];
  double* out_loss = tentative ? S->tloss[dir] : S->loss[dir];
  /* a pixel reads and writes only its own assignment */
#pragma omp parallel for schedule(dynamic, 1)
  for (int y = 0; y < H; ++y) {
    int ylo, yhi;
    cover_range(H, B, y, &ylo, &yhi);
    for (int x = 0; x < W; ++x) {
      const int p = y * W + x;
      int bw_ = S->win[dir][p];
      double bl = S->loss[dir][p];
      /* stage 2 takes only the residual (unassigned) pixels (Sec. 3.2); with the
         strict level priority so does every stage of every level: a pixel keeps
         the plane of the first level that assigned it (Sec. 3.3) */
      const int candidate = (stage == 1 && !S->merge_strict) || (bw_ < 0);
      int flag = 0;
      if (candidate) {
        int xlo, xhi;
        cover_range(W, B, x, &xlo, &xhi);
        /* all inlier candidates, for near-tie accounting */
        int cand[64];
        double candL[64];
        int nc = 0;
        if (bw_ >= 0) {
          cand[nc] = bw_;
          candL[nc] = bl;
          ++nc;
        }
        for (int by = ylo; by <= yhi; ++by)
          for (int bx = xlo; bx <= xhi; ++bx) {
            int k = orc_plane_index(S, dir, level, stage, by * nbx + bx);
            const int32_t* I = pinfo_of(S, k);
            if (!(tentative ? I[ORC_PI_DETECTED] : I[ORC_PI_VALID])) continue;
            int nb = 0;
            double e = orc_colour_err(S, dir, x, y, H_of(S, k), &nb);
            if (nb) flag |= ORC_F_BOUNDS;
            if (isfinite(e) && fabs(e - eps2) <= TIE_REL * eps2) flag |= ORC_F_COLOUR;
            if (!(e < eps2)) continue;
            cand[nc] = k;
            candL[nc] = e;
            ++nc;
            if (bw_ < 0 || key_less(e, I, bl, pinfo_of(S, bw_))) {
              bw_ = k;
              bl = e;
            }
          }
        /* loss near-ties between non-equivalent planes */
        for (int i = 0; i < nc; ++i)
          for (int j = i + 1; j < nc; ++j) {
            double m = candL[i] > candL[j] ? candL[i] : candL[j];
            if (fabs(candL[i] - candL[j]) <= TIE_REL * m && !h_equiv(H_of(S, cand[i]), H_of(S, cand[j])))
              flag |= ORC_F_COLOUR;
          }
      }
      out_win[p] = bw_;
      out_loss[p] = bw_ >= 0 ? bl : INFINITY;
      if (S->pflag[dir]) S->pflag[dir][p] |= (uint8_t)flag;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Forward-backward plane-projection test (Sec. 3.4 first cue, Alg. 1 plane  */
/* symmetry; readings R21, R22).                                             */
/* ------------------------------------------------------------------------ */
int orc_fb_test(const orc_pair* S, int dir, int px, int py, const double* Hm, const int32_t* other_win,
                uint8_t* flag) {
  const int W = S->W, H = S->H;
  (void)dir; /* the other direction's state is passed explicitly */
  double qx, qy;
  if (!orc_project(Hm, px, py, &qx, &qy)) return 0;
  if (flag && (near_bound(qx, W - 1) || near_bound(qy, H - 1))) *flag |= ORC_F_BOUNDS;
  if (qx < 0 || qx > W - 1 || qy < 0 || qy > H - 1) return 0;
  if (flag && (near_half(qx) || near_half(qy))) *flag |= ORC_F_ROUND;
  int rx = clampi((int)floor(qx + 0.5), 0, W - 1);
  int ry = clampi((int)floor(qy + 0.5), 0, H - 1);
  int j = other_win[ry * W + rx];
  if (j < 0) return 0;
  double bx, by;
  if (!orc_project(H_of(S, j), qx, qy, &bx, &by)) return 0;
  double d2 = (bx - px) * (bx - px) + (by - py) * (by - py);
  double t = S->tau_fb * S->tau_fb;
  if (flag && fabs(d2 - t) <= TIE_REL * t) *flag |= ORC_F_FB;
  return d2 < t;
}

/* Plane symmetry (Alg. 1): |r_k| >= m_min and pass / |r_k| > eta.  With cue 3
   (Sec. 3.4, third criterion; reading: the share of r_k that the plane's own
   RANSAC test accepts must also exceed eta), rin / |r_k| > eta as well. */
static int sym_decide(const orc_pair* S, int rk, int pass, int rin, int mmin) {
  int ok = rk >= mmin && (int64_t)pass * S->eta_den > (int64_t)S->eta_num * rk;
  if (S->cues & ORC_CUE_OVERLAP) ok = ok && (int64_t)rin * S->eta_den > (int64_t)S->eta_num * rk;
  return ok;
}

void orc_symmetry(orc_pair* S, int level, int stage) {
  const int W = S->W, H = S->H;
  const int B = S->block[level];
  const int nb = orc_block_count(W, B) * orc_block_count(H, B);
  const double eps2 = S->eps * S->eps;
  /* a window writes only its own plane record and reads the other direction's
     tentative assignment, which this step does not change */
#pragma omp parallel for schedule(dynamic, 1)
  for (int db = 0; db < 2 * nb; ++db) {
    const int dir = db / nb, b = db % nb;
    {
      const int k = orc_plane_index(S, dir, level, stage, b);
      int32_t* I = S->pinfo + (size_t)k * ORC_PI_N;
      I[ORC_PI_RK] = 0;
      I[ORC_PI_PASS] = 0;
      I[ORC_PI_RIN] = 0;
      if (!I[ORC_PI_DETECTED]) {
        I[ORC_PI_VALID] = 0;
        continue;
      }
      const double* Hk = H_of(S, k);
      const double tau2 = S->tau * S->tau;
      int rk = 0, pass = 0, rin = 0, nnear = 0;
      for (int y = I[ORC_PI_Y0]; y < I[ORC_PI_Y0] + I[ORC_PI_BH]; ++y)
        for (int x = I[ORC_PI_X0]; x < I[ORC_PI_X0] + I[ORC_PI_BW]; ++x) {
          const int p = y * W + x;
          if (stage == 2 && S->win[dir][p] >= 0) continue; /* input set = residual pixels */
          int nbnd = 0;
          double e = orc_colour_err(S, dir, x, y, Hk, &nbnd);
          uint8_t f = 0;
          if (nbnd || (isfinite(e) && fabs(e - eps2) <= TIE_REL * eps2)) f = 1;
          if (e < eps2) {
            ++rk;
            uint8_t ff = 0;
            if (orc_fb_test(S, dir, x, y, Hk, S->twin[1 - dir], &ff)) ++pass;
            if (ff) f = 1;
            /* the same reprojection test as RANSAC, on the pixel's NNF match */
            const int32_t v = S->nnf[dir][p];
            int nr = 0;
            if (ransac_inlier(Hk, x, y, x + unpack_dx(v), y + unpack_dy(v), tau2, &nr)) ++rin;
            if (nr) f = 1;
          }
          nnear += f;
        }
      const int mmin = orc_m_min(S, I[ORC_PI_BW], I[ORC_PI_BH]);
      I[ORC_PI_RK] = rk;
      I[ORC_PI_PASS] = pass;
      I[ORC_PI_RIN] = rin;
      I[ORC_PI_VALID] = sym_decide(S, rk, pass, rin, mmin);
      if (nnear && S->bflag) {
        S->bflag[k] |= 128; /* counts may differ by up to nnear */
        const int d = nnear;
        for (int a = -1; a <= 1; a += 2)
          for (int c = -1; c <= 1; c += 2)
            for (int e2 = -1; e2 <= 1; e2 += 2) {
              int rk2 = rk + a * d, ps2 = pass + c * d, ri2 = rin + e2 * d;
              if (rk2 < 0) rk2 = 0;
              if (ps2 < 0) ps2 = 0;
              if (ps2 > rk2) ps2 = rk2;
              if (ri2 < 0) ri2 = 0;
              if (ri2 > rk2) ri2 = rk2;
              if (sym_decide(S, rk2, ps2, ri2, mmin) != I[ORC_PI_VALID]) S->bflag[k] |= ORC_F_FB;
            }
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* O12: end-of-level forward-backward check, Jacobi over both directions     */
/* (Sec. 4: FB at the end of every level; reading R23).                      */
/* ------------------------------------------------------------------------ */
void orc_fb_unassign(orc_pair* S) {
  const int n = S->W * S->H;
  /* judged on the snapshot in win; the results go to twin first */
  for (int dir = 0; dir < 2; ++dir)
#pragma omp parallel for schedule(static)
    for (int p = 0; p < n; ++p) {
      int j = S->win[dir][p];
      S->twin[dir][p] = j;
      S->tloss[dir][p] = S->loss[dir][p];
      if (j < 0) continue;
      uint8_t f = 0;
      if (!orc_fb_test(S, dir, p % S->W, p / S->W, H_of(S, j), S->win[1 - dir], &f)) {
        S->twin[dir][p] = -1;
        S->tloss[dir][p] = INFINITY;
      }
      if (S->pflag[dir]) S->pflag[dir][p] |= f;
    }
  for (int dir = 0; dir < 2; ++dir) {
    memcpy(S->win[dir], S->twin[dir], sizeof(int32_t) * (size_t)n);
    memcpy(S->loss[dir], S->tloss[dir], sizeof(double) * (size_t)n);
  }
}

/* ------------------------------------------------------------------------ */
/* O13 + O14: propagate reliable plane matches into the NNF (Sec. 3.3.1,     */
/* reading R13) and choose each pixel's region distortion (reading R14).    */
/* ------------------------------------------------------------------------ */
/* ------------------------------------------------------------------------ */
/* Occlusion cue 2 (Sec. 3.4, second criterion: match uniqueness; reading:   */
/* pixel targets, smallest loss wins, ties to the smallest index, targets    */
/* rounded as in the NNF update and left out when outside the frame).        */
/* ------------------------------------------------------------------------ */
void orc_unique(orc_pair* S) {
  const int W = S->W, H = S->H, n = W * H;
  double* best_loss = (double*)malloc(sizeof(double) * (size_t)n);
  int32_t* best_p = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* target = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  for (int dir = 0; dir < 2; ++dir) {
    for (int q = 0; q < n; ++q) {
      best_loss[q] = INFINITY;
      best_p[q] = -1;
    }
    for (int p = 0; p < n; ++p) {
      target[p] = -1;
      const int j = S->win[dir][p];
      if (j < 0) continue;
      const int x = p % W, y = p / W;
      double qx, qy;
      if (!orc_project(H_of(S, j), x, y, &qx, &qy)) continue;
      if (S->pflag[dir] && (near_half(qx) || near_half(qy))) S->pflag[dir][p] |= ORC_F_ROUND;
      const double rx = floor(qx + 0.5), ry = floor(qy + 0.5);
      if (!(rx >= 0 && rx <= W - 1 && ry >= 0 && ry <= H - 1)) continue;
      const int q = (int)ry * W + (int)rx;
      target[p] = q;
      /* pixels in increasing order: a strictly smaller loss takes over, an equal one does not */
      if (S->loss[dir][p] < best_loss[q] || best_p[q] < 0) {
        best_loss[q] = S->loss[dir][p];
        best_p[q] = p;
      }
    }
    for (int p = 0; p < n; ++p) {
      const int q = target[p];
      if (q < 0) continue;
      if (S->pflag[dir] && best_p[q] != p && fabs(S->loss[dir][p] - best_loss[q]) <= TIE_REL * best_loss[q])
        S->pflag[dir][p] |= ORC_F_COLOUR;
      if (best_p[q] != p) {
        S->win[dir][p] = -1;
        S->loss[dir][p] = INFINITY;
      }
    }
  }
  free(best_loss);
  free(best_p);
  free(target);
}

/* ------------------------------------------------------------------------ */
/* Filling by homography-model propagation (Sec. 3.4.1, reading R34).        */
/* ------------------------------------------------------------------------ */
void orc_fill(orc_pair* S) {
  const int W = S->W, H = S->H;
  const double eps2 = S->eps * S->eps;
  const int nx[4] = {-1, 1, 0, 0}, ny[4] = {0, 0, -1, 1};
  for (int dir = 0; dir < 2; ++dir) {
    int32_t* win = S->win[dir];
    int quiet = 0;
    for (int t = 0; t < S->fill_sweeps && quiet < 2; ++t) {
      int filled = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : filled)
      for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
          const int p = y * W + x;
          if ((x + y) % 2 != t % 2 || win[p] != -1) continue;
          int best = -1;
          double be = INFINITY;
          for (int k = 0; k < 4; ++k) {
            const int qx = x + nx[k], qy = y + ny[k];
            if (qx < 0 || qx >= W || qy < 0 || qy >= H) continue;
            const int j = win[qy * W + qx];
            if (j == -1) continue;
            const int plane = j >= 0 ? j : -2 - j;
            const double e = orc_colour_err(S, dir, x, y, H_of(S, plane), NULL);
            if (e < be || (e == be && plane < best)) {
              be = e;
              best = plane;
            }
          }
          if (best >= 0 && be < eps2) {
            /* this pixel's colour; its neighbours, the only pixels read this
               half-sweep, have the other colour and are left alone */
            win[p] = -2 - best;
            S->loss[dir][p] = be;
            ++filled;
          }
        }
      quiet = filled ? 0 : quiet + 1;
    }
  }
}

void orc_nnf_update(orc_pair* S, int dir, int level) {
  const int W = S->W, H = S->H;
  const int B = S->block[level];
  const int nbx = orc_block_count(W, B);
  /* a pixel writes only its own offset and label */
#pragma omp parallel for schedule(dynamic, 1)
  for (int y = 0; y < H; ++y) {
    int ylo, yhi;
    cover_range(H, B, y, &ylo, &yhi);
    for (int x = 0; x < W; ++x) {
      const int p = y * W + x;
      const int j = S->win[dir][p];
      if (j >= 0) {
        double qx, qy;
        if (orc_project(H_of(S, j), x, y, &qx, &qy)) {
          if (S->pflag[dir] && (near_half(qx) || near_half(qy))) S->pflag[dir][p] |= ORC_F_ROUND;
          /* round, then clamp (reading R13), the clamp taken in FP64 so that no
             projection is converted to int out of range */
          const double fx = fmin(fmax(floor(qx + 0.5), 0.0), (double)(W - 1));
          const double fy = fmin(fmax(floor(qy + 0.5), 0.0), (double)(H - 1));
          S->nnf[dir][p] = pack_off((int)fx - x, (int)fy - y);
        }
      }
      int xlo, xhi;
      cover_range(W, B, x, &xlo, &xhi);
      int best = -1, bestc = -1;
      for (int stage = 1; stage <= 2; ++stage)
        for (int by = ylo; by <= yhi; ++by)
          for (int bx = xlo; bx <= xhi; ++bx) {
            int k = orc_plane_index(S, dir, level, stage, by * nbx + bx);
            const int32_t* I = pinfo_of(S, k);
            if (!I[ORC_PI_VALID]) continue;
            if (I[ORC_PI_COUNT] > bestc) {
              bestc = I[ORC_PI_COUNT];
              best = k;
            }
          }
      if (best >= 0) S->hlabel[dir][p] = best;
    }
  }
}

void orc_finalize(orc_pair* S, int dir, float* flow, uint8_t* occ) {
  const int W = S->W, H = S->H;
  orc_eval_cost(S, dir, 2);
#pragma omp parallel for schedule(static)
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      const int p = y * W + x;
      const int j = S->win[dir][p];
      const int plane = j >= 0 ? j : -2 - j; /* j <= -2: filled */
      double qx, qy;
      if (j != -1 && orc_project(H_of(S, plane), x, y, &qx, &qy)) {
        flow[2 * p] = (float)(qx - x);
        flow[2 * p + 1] = (float)(qy - y);
        occ[p] = j >= 0 ? 0 : 2;
      } else {
        flow[2 * p] = (float)unpack_dx(S->nnf[dir][p]);
        flow[2 * p + 1] = (float)unpack_dy(S->nnf[dir][p]);
        occ[p] = 1;
      }
    }
}

/* ------------------------------------------------------------------------ */
/* O15: the whole pipeline (Alg. 1 per level, Sec. 4 set-up).                */
/* ------------------------------------------------------------------------ */
static void pm_pass(orc_pair* S, int slot, int restricted) {
  for (int it = 0; it < S->iters; ++it)
    for (int colour = 0; colour < 2; ++colour)
      for (int dir = 0; dir < 2; ++dir) orc_pm_halfsweep(S, dir, colour, it, slot, restricted);
}

void orc_solve(orc_pair* S, const int32_t* init0, const int32_t* init1, float* flow0, float* flow1, uint8_t* occ0,
               uint8_t* occ1) {
  const int W = S->W, H = S->H, n = W * H;
  orc_planes_init(S);
  const int32_t* init[2] = {init0, init1};
  for (int dir = 0; dir < 2; ++dir) {
    if (init[dir]) {
      for (int p = 0; p < n; ++p) {
        int x = p % W, y = p / W;
        int tx = clampi(x + unpack_dx(init[dir][p]), 0, W - 1);
        int ty = clampi(y + unpack_dy(init[dir][p]), 0, H - 1);
        S->nnf[dir][p] = pack_off(tx - x, ty - y);
      }
    } else {
      orc_nnf_init(S, dir);
    }
    for (int p = 0; p < n; ++p) {
      S->win[dir][p] = -1;
      S->loss[dir][p] = INFINITY;
      S->hlabel[dir][p] = -1;
    }
    orc_eval_cost(S, dir, 0);
  }
  pm_pass(S, 0, 0);
  for (int l = 0; l < S->n_levels; ++l) {
    for (int stage = 1; stage <= 2; ++stage) {
      for (int dir = 0; dir < 2; ++dir) orc_ransac(S, dir, l, stage);
      for (int dir = 0; dir < 2; ++dir) orc_assign(S, dir, l, stage, 1);
      orc_symmetry(S, l, stage);
      for (int dir = 0; dir < 2; ++dir) orc_assign(S, dir, l, stage, 0);
    }
    orc_fb_unassign(S);
    if (S->cues & ORC_CUE_UNIQUE) orc_unique(S);
    for (int dir = 0; dir < 2; ++dir) {
      orc_nnf_update(S, dir, l);
      orc_eval_cost(S, dir, 1);
    }
    pm_pass(S, l + 1, 1);
  }
  if (S->fill_sweeps > 0) orc_fill(S);
  orc_finalize(S, 0, flow0, occ0);
  orc_finalize(S, 1, flow1, occ1);
}
