/* Driver for the sanitizer build of the oracle (AddressSanitizer and
 * UndefinedBehaviorSanitizer): whole solves of a small procedurally textured
 * pair, two levels, with every option of the pipeline switched on in turn.
 * Prints OK when every output is finite and in range. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "msgpm_oracle.h"

enum { W = 40, H = 32 };

static float texture(int x, int y, int c) {
  /* smooth, aperiodic enough for matching: a few incommensurate sinusoids */
  return 0.5f + 0.25f * (float)sin(0.37 * x + 0.23 * y + c) + 0.2f * (float)cos(0.11 * x * (c + 1) - 0.41 * y);
}

static int run(int cues, int fill, int strict, int fp16) {
  static float rgb1[W * H * 3], rgb2[W * H * 3];
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x)
      for (int c = 0; c < 3; ++c) {
        rgb1[3 * (y * W + x) + c] = texture(x, y, c);
        /* frame 2: the left part moved by (+2, +1), the right part by (-1, 0) */
        rgb2[3 * (y * W + x) + c] = x < 20 ? texture(x - 2, y - 1, c) : texture(x + 1, y, c);
      }
  const int C = 5, n = W * H;
  float* F0 = malloc(sizeof(float) * C * n);
  float* F1 = malloc(sizeof(float) * C * n);
  orc_features(rgb1, W, H, C, fp16, F0);
  orc_features(rgb2, W, H, C, fp16, F1);
  orc_pair S;
  memset(&S, 0, sizeof S);
  S.W = W; S.H = H; S.C = C; S.r = 2;
  for (int c = 0; c < 5; ++c) S.wc[c] = 1.0;
  S.F[0] = F0; S.F[1] = F1;
  S.n_levels = 2; S.block[0] = 16; S.block[1] = 8;
  S.iters = 2; S.hyps = 16; S.R0 = 0; S.m_min_abs = 8; S.eta_num = 1; S.eta_den = 2;
  S.tau = 1.0; S.eps = 0.1; S.tau_fb = 1.0; S.mu = 0.25; S.seed = 3;
  S.cues = cues; S.fill_sweeps = fill; S.merge_strict = strict;
  for (int d = 0; d < 2; ++d) {
    S.nnf[d] = calloc(n, sizeof(int32_t));
    S.cost[d] = calloc(n, sizeof(double));
    S.win[d] = calloc(n, sizeof(int32_t));
    S.loss[d] = calloc(n, sizeof(double));
    S.hlabel[d] = calloc(n, sizeof(int32_t));
    S.twin[d] = calloc(n, sizeof(int32_t));
    S.tloss[d] = calloc(n, sizeof(double));
    S.pflag[d] = calloc(n, 1);
  }
  S.P = orc_plane_capacity(&S);
  S.pH = calloc((size_t)S.P * 9, sizeof(double));
  S.pinfo = calloc((size_t)S.P * ORC_PI_N, sizeof(int32_t));
  S.bflag = calloc(S.P, 1);
  float* flow[2] = {malloc(sizeof(float) * 2 * n), malloc(sizeof(float) * 2 * n)};
  uint8_t* occ[2] = {malloc(n), malloc(n)};
  orc_solve(&S, NULL, NULL, flow[0], flow[1], occ[0], occ[1]);
  int bad = 0;
  for (int d = 0; d < 2; ++d)
    for (int p = 0; p < n; ++p) {
      bad += !isfinite(flow[d][2 * p]) || !isfinite(flow[d][2 * p + 1]) || occ[d][p] > 2;
    }
  for (int d = 0; d < 2; ++d) {
    free(S.nnf[d]); free(S.cost[d]); free(S.win[d]); free(S.loss[d]); free(S.hlabel[d]);
    free(S.twin[d]); free(S.tloss[d]); free(S.pflag[d]); free(flow[d]); free(occ[d]);
  }
  free(S.pH); free(S.pinfo); free(S.bflag); free(F0); free(F1);
  return bad;
}

int main(void) {
  int bad = 0;
  bad += run(0, 0, 0, 0);
  bad += run(ORC_CUE_OVERLAP | ORC_CUE_UNIQUE, 8, 0, 0);
  bad += run(0, 0, 1, 1);
  if (bad) {
    printf("FAILED: %d bad outputs\n", bad);
    return 1;
  }
  printf("OK\n");
  return 0;
}
