// Driver for the sanitizer build of the library's host code (AddressSanitizer
// and UndefinedBehaviorSanitizer on the host side only): parameter
// validation and workspace layout over valid and invalid parameter sets, and
// the serving and batching paths that end before any device work (refusals,
// queue limits, waits that time out, cancellation, injected allocation
// failures).  Device pointers are aligned placeholders that are never
// dereferenced.  Prints OK when every call returned the expected status.
#include <stdio.h>
#include <string.h>

#include "msgpm.h"

static int failures = 0;
static void expect(bool ok, const char* what) {
  if (!ok) {
    printf("unexpected: %s (%s)\n", what, msgpm_last_error());
    ++failures;
  }
}

static msgpm_params params(int w, int h) {
  msgpm_params p;
  memset(&p, 0, sizeof p);
  p.width = w;
  p.height = h;
  p.channels = 5;
  p.patch_radius = 4;
  p.n_levels = 3;
  p.block[0] = 64;
  p.block[1] = 32;
  p.block[2] = 16;
  p.pm_iters = 8;
  p.ransac_hyps = 256;
  p.min_support_abs = 8;
  p.eta_num = 1;
  p.eta_den = 2;
  p.grad_weight = 1.0;
  p.inlier_px = 1.0;
  p.eps_color = 0.1;
  p.fb_px = 1.0;
  p.min_support_frac = 0.25;
  return p;
}

int main() {
  msgpm_layout L;
  const int sizes[][2] = {{2, 2}, {9, 7}, {77, 53}, {1024, 436}, {2048, 872}, {32767, 3}};
  for (auto& s : sizes)
    for (unsigned flags = 0; flags < 32; ++flags) {
      msgpm_params p = params(s[0], s[1]);
      p.flags = flags;
      expect(msgpm_layout_query(&p, &L) == MSGPM_OK, "valid layout");
      expect(L.total_bytes > 0 && L.total_bytes % 256 == 0, "layout size");
    }
  {
    msgpm_params p = params(1, 5);
    expect(msgpm_layout_query(&p, &L) == MSGPM_E_INVALID, "tiny frame");
    p = params(64, 48);
    p.patch_radius = 9;
    expect(msgpm_layout_query(&p, &L) == MSGPM_E_UNSUPPORTED, "radius");
    p = params(64, 48);
    p.n_levels = 9;
    expect(msgpm_layout_query(&p, &L) == MSGPM_E_INVALID, "levels");
    p = params(64, 48);
    p.flags = 1u << 9;
    expect(msgpm_layout_query(&p, &L) == MSGPM_E_INVALID, "flags");
    expect(msgpm_layout_query(nullptr, &L) == MSGPM_E_INVALID, "null params");
    expect(msgpm_layout_query(&p, nullptr) == MSGPM_E_INVALID, "null layout");
  }
  void* fake = reinterpret_cast<void*>(0x10000000);
  float* ff = static_cast<float*>(fake);
  uint8_t* fu = static_cast<uint8_t*>(fake);
  {
    msgpm_server* sv = nullptr;
    msgpm_params p = params(320, 240);
    msgpm_layout_query(&p, &L);
    expect(msgpm_server_create(L.total_bytes - 1, 2, &sv) == MSGPM_OK, "create");
    uint64_t t = 0;
    expect(msgpm_server_submit(sv, &p, ff, ff, nullptr, nullptr, fake, ff, ff, fu, fu, &t) == MSGPM_E_OOM, "oom");
    expect(msgpm_server_destroy(sv) == MSGPM_OK, "destroy");
    expect(msgpm_server_create(1ull << 40, 2, &sv) == MSGPM_OK, "create");
    expect(msgpm_server_set_queue_limit(sv, 3) == MSGPM_OK, "limit");
    uint64_t tk[4];
    for (int i = 0; i < 3; ++i)
      expect(msgpm_server_submit(sv, &p, ff, ff, nullptr, nullptr, fake, ff, ff, fu, fu, &tk[i]) == MSGPM_OK,
             "submit");
    expect(msgpm_server_submit(sv, &p, ff, ff, nullptr, nullptr, fake, ff, ff, fu, fu, &tk[3]) == MSGPM_E_BUSY,
           "busy");
    expect(msgpm_server_wait(sv, tk[0], 0) == MSGPM_E_TIMEOUT, "timeout 0");
    expect(msgpm_server_wait(sv, tk[1], 500) == MSGPM_E_TIMEOUT, "timeout");
    int retired = 0, done = 1;
    expect(msgpm_server_cancel(sv, tk[2], &retired) == MSGPM_OK && retired == 1, "cancel queued");
    expect(msgpm_server_poll(sv, tk[2], &done) == MSGPM_E_INVALID, "retired ticket");
    expect(msgpm_server_poll(sv, tk[0], &done) == MSGPM_OK && done == 0, "poll queued");
    expect(msgpm_debug_fail_allocations(1) == MSGPM_OK, "inject");
    int pending = -1;
    expect(msgpm_server_step(sv, fake, nullptr, &pending) == MSGPM_E_OOM, "injected staging failure");
    msgpm_debug_fail_allocations(0);
    expect(msgpm_server_destroy(sv) == MSGPM_OK, "destroy");
  }
  {
    msgpm_params ps[3] = {params(64, 48), params(97, 61), params(33, 20)};
    uint64_t bytes = 0;
    expect(msgpm_batch_query(3, ps, &bytes) == MSGPM_OK && bytes > 0, "batch query");
    ps[1].pm_iters = 3;
    expect(msgpm_batch_query(3, ps, &bytes) == MSGPM_E_INVALID, "mixed batch");
    expect(msgpm_batch_query(0, ps, &bytes) == MSGPM_E_INVALID, "empty batch");
  }
  if (failures) {
    printf("FAILED: %d\n", failures);
    return 1;
  }
  printf("OK\n");
  return 0;
}
