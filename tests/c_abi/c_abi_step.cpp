// The library used from C++ through its C ABI alone: no Python, no torch;
// device buffers come from hipMalloc.  A square split into two triangles,
// three flat layers of 1 m, one field: a constant field under a constant
// velocity with matching exterior values must stay constant, and its mass
// must equal the volume (3 m^3).  An argument error must come back as
// SDG_E_ARG with a message.  Exit status 0 on success.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <vector>

#include "slimdg.h"

#define CHECK_SDG(call)                                                              \
  do {                                                                               \
    sdg_status st_ = (call);                                                         \
    if (st_ != SDG_OK) {                                                             \
      std::fprintf(stderr, "%s failed (%d): %s\n", #call, (int)st_, sdg_last_error()); \
      return 1;                                                                      \
    }                                                                                \
  } while (0)
#define CHECK_HIP(call)                                                           \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      std::fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));      \
      return 1;                                                                   \
    }                                                                             \
  } while (0)

int main() {
  const double vxy[] = {0, 0, 1, 0, 1, 1, 0, 1};
  const int32_t tri[] = {0, 1, 2, 0, 2, 3};
  const int32_t nbr[] = {-1, -1, 1, 0, -1, -1};   // the shared edge 2->0 / 0->2
  const int32_t nlayers[] = {3, 3};
  std::vector<double> zlev;
  for (int c = 0; c < 2; ++c)
    for (int lv = 0; lv <= 3; ++lv)
      for (int v = 0; v < 3; ++v) zlev.push_back(-(double)lv);
  sdg_mesh_desc mesh{};
  mesh.n_members = 1;
  mesh.n_tri = 2;
  mesh.n_vert = 4;
  mesh.vxy = vxy;
  mesh.tri = tri;
  mesh.nbr = nbr;
  mesh.nlayers = nlayers;
  mesh.zlev = zlev.data();
  mesh.n_fields = 1;
  mesh.precision = SDG_FP64;

  if (sdg_abi_version() != SDG_ABI_VERSION) {
    std::fprintf(stderr, "ABI %d, header %d\n", sdg_abi_version(), SDG_ABI_VERSION);
    return 1;
  }
  sdg_layout lay{};
  CHECK_SDG(sdg_query_layout(&mesh, &lay));
  std::vector<int64_t> slots(lay.n_prisms);
  CHECK_SDG(sdg_prism_slots(&mesh, slots.data()));
  const size_t S = (size_t)lay.n_slots;

  void *ws = nullptr, *state = nullptr, *vel = nullptr;
  double* kappa = nullptr;
  CHECK_HIP(hipMalloc(&ws, lay.workspace_bytes));
  CHECK_HIP(hipMalloc(&state, lay.state_bytes));
  CHECK_HIP(hipMalloc(&vel, lay.velocity_bytes));
  CHECK_HIP(hipMalloc(&kappa, sizeof(double) * lay.max_layers));

  // host images in the cell layout: [component][node][slot]
  std::vector<double> T(6 * S, 0.0), U(3 * 6 * S, 0.0), K(lay.max_layers, 1e-2);
  for (int64_t p = 0; p < lay.n_prisms; ++p)
    for (int i = 0; i < 6; ++i) {
      T[i * S + slots[p]] = 1.0;
      U[(0 * 6 + i) * S + slots[p]] = 0.1;
      U[(1 * 6 + i) * S + slots[p]] = 0.05;
    }
  CHECK_HIP(hipMemcpy(state, T.data(), lay.state_bytes, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(vel, U.data(), lay.velocity_bytes, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(kappa, K.data(), sizeof(double) * K.size(), hipMemcpyHostToDevice));

  sdg_ctx* ctx = nullptr;
  CHECK_SDG(sdg_create(&ctx, 0, nullptr));
  CHECK_SDG(sdg_mesh_upload(ctx, &mesh, ws, lay.workspace_bytes));
  const double t_ext = 1.0;
  sdg_params prm{};
  prm.dt = 0.5;
  prm.penalty_eta = 4.0;
  prm.t_ext = &t_ext;
  prm.w_is_zero = 1;
  CHECK_SDG(sdg_set_params(ctx, &prm));
  CHECK_SDG(sdg_set_velocity(ctx, vel));
  CHECK_SDG(sdg_set_diffusivity(ctx, kappa));
  CHECK_SDG(sdg_set_fields(ctx, state));
  CHECK_SDG(sdg_step(ctx, 10));
  CHECK_SDG(sdg_sync(ctx));

  CHECK_HIP(hipMemcpy(T.data(), state, lay.state_bytes, hipMemcpyDeviceToHost));
  double dev = 0.0;
  for (int64_t p = 0; p < lay.n_prisms; ++p)
    for (int i = 0; i < 6; ++i) dev = std::fmax(dev, std::fabs(T[i * S + slots[p]] - 1.0));
  double mass = 0.0;
  CHECK_SDG(sdg_mass(ctx, state, &mass));

  // an argument error: stage 3 does not exist
  const sdg_status bad = sdg_rk_stage(ctx, 3, state, state, vel);
  const bool bad_ok = bad == SDG_E_ARG && sdg_last_error()[0] != '\0';

  CHECK_SDG(sdg_destroy(ctx));
  (void)hipFree(ws);
  (void)hipFree(state);
  (void)hipFree(vel);
  (void)hipFree(kappa);
  std::printf("c_abi_step: %lld prisms, 10 steps, max |T - 1| = %.3e, mass = %.15f, bad stage -> %d\n",
              (long long)lay.n_prisms, dev, mass, (int)bad);
  return (dev <= 1e-12 && std::fabs(mass - 3.0) <= 1e-12 && bad_ok) ? 0 : 1;
}
