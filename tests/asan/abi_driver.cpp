// Host-side checks of the C-ABI's argument validation, built with the host
// sanitizers (no device is touched: every call here must fail before it
// reaches the HIP runtime).  Exit status 0 when every call returns the
// documented status.
#include <cstdio>
#include <cstring>

#include "olb.h"

static int failures = 0;

static void expect(const char* what, olb_status got, olb_status want) {
  if (got != want) {
    std::fprintf(stderr, "%s: got %d, want %d\n", what, (int)got, (int)want);
    ++failures;
  }
}

static olb_params base() {
  olb_params p;
  std::memset(&p, 0, sizeof p);
  p.nx = 32;
  p.ny = 32;
  p.ds = 1.0 / 32;
  p.dt = 5e-4;
  p.tau = 0.01;
  p.a = 9.0 / 49;
  p.b = 2.0 / 21;
  p.sigma = 1e-4;
  p.tw_lo = p.tw_hi = 1.0;
  p.rho_ref = 1.0;
  return p;
}

int main() {
  size_t bytes = 0;
  olb_params p = base();
  expect("workspace ok", olb_workspace_bytes(&p, &bytes), OLB_OK);
  if (bytes < 3u * 25u * 38u * 32u * 8u) {
    std::fprintf(stderr, "workspace too small: %zu\n", bytes);
    ++failures;
  }
  expect("workspace null params", olb_workspace_bytes(nullptr, &bytes), OLB_E_ARG);
  expect("workspace null out", olb_workspace_bytes(&p, nullptr), OLB_E_ARG);
  struct Case {
    const char* what;
    void (*edit)(olb_params&);
    olb_status want;
  } cases[] = {
      {"cfl", [](olb_params& q) { q.dt = 0.02; }, OLB_E_CFL},
      {"tau", [](olb_params& q) { q.tau = 0.0; }, OLB_E_DOMAIN},
      {"bc_x walls", [](olb_params& q) { q.bc_x = 1; }, OLB_E_ARG},
      {"specular narrow", [](olb_params& q) { q.bc_x = 3; q.nx = 2; }, OLB_E_ARG},
      {"walls short", [](olb_params& q) { q.bc_y = 1; q.ny = 2; }, OLB_E_ARG},
      {"bad bc_y", [](olb_params& q) { q.bc_y = 7; }, OLB_E_ARG},
      {"nx", [](olb_params& q) { q.nx = 0; }, OLB_E_ARG},
      {"huge", [](olb_params& q) { q.nx = 1 << 20; q.ny = 1 << 12; }, OLB_E_ARG},
      {"rho_ref", [](olb_params& q) { q.precision = 1; q.rho_ref = 0.0; }, OLB_E_ARG},
      {"precision", [](olb_params& q) { q.precision = 5; }, OLB_E_ARG},
      {"wall T", [](olb_params& q) { q.bc_y = 1; q.tw_lo = 0.0; }, OLB_E_DOMAIN},
      {"sigma", [](olb_params& q) { q.sigma = -1.0; }, OLB_E_ARG},
  };
  for (const Case& c : cases) {
    olb_params q = base();
    c.edit(q);
    expect(c.what, olb_workspace_bytes(&q, &bytes), c.want);
    olb_ctx* ctx = nullptr;
    alignas(256) static unsigned char fake[256];
    expect(c.what, olb_init(&q, fake, sizeof fake, nullptr, &ctx), c.want);
    if (ctx) ++failures;
  }
  // workspace checks come before any device work
  olb_ctx* ctx = nullptr;
  alignas(256) static unsigned char small[256];
  expect("init null workspace", olb_init(&p, nullptr, bytes, nullptr, &ctx), OLB_E_WORKSPACE);
  expect("init small workspace", olb_init(&p, small, sizeof small, nullptr, &ctx), OLB_E_WORKSPACE);
  expect("init misaligned", olb_init(&p, small + 8, bytes, nullptr, &ctx), OLB_E_WORKSPACE);
  expect("init null out", olb_init(&p, small, bytes, nullptr, nullptr), OLB_E_ARG);
  // every per-context call rejects a null context
  double d[4] = {0, 0, 0, 0};
  expect("set_fields", olb_set_fields(nullptr, d, d, d, d), OLB_E_ARG);
  expect("step", olb_step(nullptr, 1), OLB_E_ARG);
  expect("sync", olb_sync(nullptr), OLB_E_ARG);
  expect("moments", olb_moments(nullptr, d, d, d, d), OLB_E_ARG);
  expect("get_f", olb_get_f(nullptr, d), OLB_E_ARG);
  expect("set_tile", olb_set_tile(nullptr, 8), OLB_E_ARG);
  int32_t a = 0, b = 0;
  expect("launch_counts", olb_launch_counts(nullptr, &a, &b), OLB_E_ARG);
  if (std::strlen(olb_strerror(OLB_E_CFL)) == 0) ++failures;
  if (std::strlen(olb_last_error(nullptr)) == 0) ++failures;
  // batches: a mixed batch and a bad count
  olb_params two[2] = {base(), base()};
  two[1].bc_y = 1;
  expect("batch mixed", olb_batch_workspace_bytes(two, 2, &bytes), OLB_E_ARG);
  expect("batch count", olb_batch_workspace_bytes(two, 0, &bytes), OLB_E_ARG);
  two[1] = base();
  two[1].nx = 77;
  expect("batch ok", olb_batch_workspace_bytes(two, 2, &bytes), OLB_OK);
  olb_batch* bt = nullptr;
  expect("batch small workspace", olb_batch_init(two, 2, small, sizeof small, nullptr, &bt), OLB_E_WORKSPACE);
  expect("batch step", olb_batch_step(nullptr, 1), OLB_E_ARG);
  // closure: sizes and null arguments
  expect("closure bytes", olb_closure_workspace_bytes(0, 4, &bytes), OLB_E_ARG);
  expect("closure bytes ok", olb_closure_workspace_bytes(64, 48, &bytes), OLB_OK);
  // the workspace layout's partial-sum rows at the smallest and the largest
  // accepted lattices (nx * ny < 2^30), and just past the largest
  expect("closure bytes 1x1", olb_closure_workspace_bytes(1, 1, &bytes), OLB_OK);
  expect("closure bytes 5x3", olb_closure_workspace_bytes(5, 3, &bytes), OLB_OK);
  expect("closure bytes max", olb_closure_workspace_bytes(32768, 32767, &bytes), OLB_OK);
  expect("closure bytes 2^30", olb_closure_workspace_bytes(32768, 32768, &bytes), OLB_E_ARG);
  olb_closure* cl = nullptr;
  expect("closure small workspace", olb_closure_init(64, 48, small, sizeof small, nullptr, &cl), OLB_E_WORKSPACE);
  expect("closure forward", olb_closure_forward(nullptr, d, d), OLB_E_ARG);
  double one[4] = {1, 1, 1, 1};
  expect("noalloc null", olb_closure_forward_noalloc(8, 8, nullptr, one, one, one, 0, d, d, nullptr), OLB_E_ARG);
  float fp[1] = {0};
  expect("noalloc size", olb_closure_forward_noalloc(0, 8, fp, one, one, one, 0, d, d, nullptr), OLB_E_ARG);
  expect("noalloc mask", olb_closure_forward_noalloc(8, 8, fp, one, one, one, 16, d, d, nullptr), OLB_E_ARG);
  expect("restrict", olb_restrict(d, 10, 8, 4, d, nullptr), OLB_E_ARG);
  if (failures) {
    std::fprintf(stderr, "%d failures\n", failures);
    return 1;
  }
  std::printf("abi validation: all statuses as documented\n");
  return 0;
}
