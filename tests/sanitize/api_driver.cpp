// Sanitizer driver for the host runtime's validation and layout code
// (test infrastructure): argument checks, workspace sizing of dense and
// compacted layouts, tilings and batches, all of which run before any device
// work.  The kernel launchers are stubbed: none of these calls reaches them.
// Exits 0 when every call returns the expected status.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/lbm.h"
#include "../../paper_2111_08666_amd/csrc/lbm_device.h"

namespace lbm {
hipError_t launch_init(const InstDev *, const InstDev &, const float *, int, hipStream_t) { return hipErrorUnknown; }
hipError_t launch_init_sat(const InstDev *, const InstDev &, const float *, float, float, float, int, hipStream_t) {
  return hipErrorUnknown;
}
hipError_t launch_step(const StepLaunch &, hipStream_t) { return hipErrorUnknown; }
hipError_t launch_observables(const InstDev *, const InstDev &, int, double *, int, double *, hipStream_t) {
  return hipErrorUnknown;
}
hipError_t launch_density(const InstDev *, const InstDev &, int, float *, hipStream_t) { return hipErrorUnknown; }
hipError_t launch_fwd_rebuild(const InstDev *, const InstDev &, int, hipStream_t) { return hipErrorUnknown; }
hipError_t launch_ivsd_freeze(const InstDev *, const InstDev &, int, hipStream_t) { return hipErrorUnknown; }
hipError_t launch_poke(const InstDev *, const InstDev &, int, int, int, int, int, int, float, int32_t *, hipStream_t) {
  return hipErrorUnknown;
}
const char *step_kernel_name(int, int, int, int, int, int) { return "stub"; }
int obs_blocks(const InstDev &) { return 1; }
}  // namespace lbm

static int fails = 0;
#define EXPECT(c)                                              \
  do {                                                         \
    if (!(c)) {                                                \
      std::fprintf(stderr, "line %d: %s\n", __LINE__, #c);     \
      ++fails;                                                 \
    }                                                          \
  } while (0)

struct Case {
  std::vector<uint8_t> solid;
  std::vector<double> rho;
  lbm_geometry g{};
  lbm_params p{};
};

static Case drainage(int q, int nx, int ny, int nz, unsigned seed) {
  Case c;
  const int N = nx * ny * nz;
  c.solid.assign((size_t)N, 0);
  c.rho.assign((size_t)2 * N, 0.0);
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const int n = x + nx * (y + ny * z);
        seed = seed * 1103515245u + 12345u;
        const bool wall = y == 0 || y == ny - 1 || (q == 19 && (z == 0 || z == nz - 1));
        c.solid[(size_t)n] = wall || (x > 3 && x < nx - 4 && (seed >> 16) % 9 == 0);
        c.rho[(size_t)n] = x < 4 ? 1.0 : 0.027;
        c.rho[(size_t)(N + n)] = x < 4 ? 0.027 : 1.0;
      }
  c.g.q = q; c.g.nx = nx; c.g.ny = ny; c.g.nz = nz;
  c.g.solid = c.solid.data();
  c.g.periodic = 0; c.g.open_x = 1; c.g.porous_x0 = 4; c.g.porous_x1 = nx - 4;
  c.p.tau[0] = 1.7; c.p.tau[1] = 0.62; c.p.G = 3.5; c.p.xi = -0.3;
  c.p.rho_in1 = 1.02; c.p.rho_out2 = 1.0; c.p.collision = LBM_TRT; c.p.bc_set = 3;
  c.p.half_force_shift = 1; c.p.lambda = 3.0 / 16.0;
  return c;
}

int main() {
  // valid problems on every layout and strategy
  for (int q : {9, 19}) {
    Case c = q == 9 ? drainage(9, 70, 26, 1, 3u) : drainage(19, 40, 20, 18, 5u);
    for (int st = LBM_AUTO; st <= LBM_COMPACT_FUSED; ++st) {
      c.p.strategy = st;
      const size_t b = lbm_workspace_bytes(&c.g, &c.p);
      EXPECT((q == 19 && st == LBM_FUSED_LIST) ? b == 0 : b > 0);
    }
    c.p.strategy = LBM_AUTO;
    for (int set = 1; set <= 3; ++set)
      for (int e26 = 0; e26 < 2; ++e26) {
        c.p.bc_set = set;
        c.p.eq26_mode = e26;
        EXPECT(lbm_workspace_bytes(&c.g, &c.p) > 0);
      }
    c.p.bc_set = 3;
    c.p.eq26_mode = 0;
    // the frozen reading of Eq. 17 adds its held values to the workspace
    const size_t dyn = lbm_workspace_bytes(&c.g, &c.p);
    c.p.ivsd_frozen = 1;
    EXPECT(lbm_workspace_bytes(&c.g, &c.p) > dyn);
    c.p.ivsd_frozen = 0;
    // a batch of three copies
    lbm_geometry gs[3] = {c.g, c.g, c.g};
    lbm_params ps[3] = {c.p, c.p, c.p};
    EXPECT(lbm_batch_workspace_bytes(3, gs, ps) > 2 * lbm_workspace_bytes(&c.g, &c.p));
    // invalid arguments, each refused before any device work
    Case bad = c;
    bad.p.tau[0] = 0.5;
    EXPECT(lbm_workspace_bytes(&bad.g, &bad.p) == 0);
    bad = c;
    bad.p.xi = 1.0;
    EXPECT(lbm_workspace_bytes(&bad.g, &bad.p) == 0);
    bad = c;
    bad.p.eq26_mode = 2;
    EXPECT(lbm_workspace_bytes(&bad.g, &bad.p) == 0);
    bad = c;
    bad.p.ivsd_frozen = -1;
    EXPECT(lbm_workspace_bytes(&bad.g, &bad.p) == 0);
    bad = c;
    bad.p.strategy = 9;
    EXPECT(lbm_workspace_bytes(&bad.g, &bad.p) == 0);
    bad = c;
    bad.g.solid = bad.solid.data();
    bad.solid[5] = 0;  // a fluid node on a closed wall (y = 0)
    EXPECT(lbm_workspace_bytes(&bad.g, &bad.p) == 0);
    bad = c;
    bad.g.solid = nullptr;
    EXPECT(lbm_workspace_bytes(&bad.g, &bad.p) == 0);
    // create: rejected without a workspace, with a small one, or unaligned
    lbm_ctx *ctx = nullptr;
    EXPECT(lbm_create(&c.g, &c.p, c.rho.data(), nullptr, 0, nullptr, &ctx) == LBM_EINVAL);
    EXPECT(lbm_create(&c.g, &c.p, c.rho.data(), (void *)4096, 16, nullptr, &ctx) == LBM_ENOMEM);
    EXPECT(lbm_create(&c.g, &c.p, c.rho.data(), (void *)4104, (size_t)1 << 40, nullptr, &ctx) == LBM_ENOMEM);
    std::vector<double> neg = c.rho;
    size_t fluid = 0;
    while (c.solid[fluid]) ++fluid;
    neg[fluid] = -1.0;
    EXPECT(lbm_create(&c.g, &c.p, neg.data(), (void *)4096, (size_t)1 << 40, nullptr, &ctx) == LBM_EINVAL);
    EXPECT(ctx == nullptr);
    EXPECT(std::strlen(lbm_last_error(nullptr)) > 0);
  }
  // null handles
  EXPECT(lbm_step(nullptr, 1) == LBM_EINVAL);
  EXPECT(lbm_init_from_saturation(nullptr, nullptr, 1, 0.5, 1.0, 0.027) == LBM_EINVAL);
  EXPECT(lbm_debug_poke(nullptr, 0, 0, 0, 0, 0, 1.0f) == LBM_EINVAL);
  EXPECT(lbm_get_step(nullptr) == -1);
  EXPECT(lbm_batch_set_active(nullptr, nullptr) == LBM_EINVAL);
  EXPECT(lbm_destroy(nullptr) == LBM_OK);
  std::printf("api sanitizer driver: %d failed checks\n", fails);
  return fails != 0;
}
