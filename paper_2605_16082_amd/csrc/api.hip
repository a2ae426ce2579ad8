// Host side of libslimdg: mesh validation and layout, workspace carving,
// upload, parameter state and the extern "C" entry points of slimdg.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "slimdg.h"

using namespace sdg;

namespace {

thread_local std::string g_err;

sdg_status fail(sdg_status st, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

sdg_status hip_fail(hipError_t e, const char* what) {
  return fail(SDG_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// ---------------------------------------------------------------------------
// Layout plan: cells, slots and workspace offsets.
// ---------------------------------------------------------------------------
struct Plan {
  int C = 0, n_cells = 0, CS = 0, max_layers = 0, F = 0, prec = 0, n_members = 1;
  bool fp32 = false;
  int64_t n_prisms = 0, n_slots = 0, n_lslots = 0;
  std::vector<int32_t> cell_base, cell_lbase, cell_depth, member_off;
  std::vector<int64_t> zoff;  // per column: first row of its levels in desc.zlev
  // per cell, the lateral faces whose neighbour is in another cell
  // (the horizontal diffusion stages their values in LDS): offsets, largest count
  std::vector<int32_t> halo_off;
  int halo_max = 0;
  // cells deepest first (stable): the dispatch order of the column solves
  std::vector<int32_t> cell_order;
  int n_tiles[kTileChoices] = {};
  // workspace offsets (bytes)
  size_t o_cell_base, o_cell_lbase, o_nlay, o_nbr_slot, o_nbr_meta, o_nbr_col, o_col_member, o_member_off,
      o_geo, o_geo32, o_xy, o_zl, o_zl32, o_tiles[kTileChoices], o_tiles_bucket, o_stage_a, o_stage_b, o_scratch,
      o_tfac,
      o_colmass, o_msum, o_flag, o_kpart, o_kh, o_hface, o_hoff, o_hslot, o_hdepth, o_hidx, o_corder, total;
  size_t state_bytes, velocity_bytes;
};

sdg_status plan_mesh(const sdg_mesh_desc* d, Plan& P) {
  if (!d) return fail(SDG_E_ARG, "mesh description is NULL");
  if (d->n_tri < 1) return fail(SDG_E_MESH, "n_tri must be >= 1 (got %d)", d->n_tri);
  if (d->n_vert < 3) return fail(SDG_E_MESH, "n_vert must be >= 3 (got %d)", d->n_vert);
  if (!d->vxy || !d->tri || !d->nbr || !d->nlayers || !d->zlev)
    return fail(SDG_E_ARG, "mesh arrays vxy, tri, nbr, nlayers and zlev must be non-NULL");
  if (d->n_fields < 1 || d->n_fields > SDG_MAX_FIELDS)
    return fail(SDG_E_UNSUPPORTED, "n_fields must be in 1..%d (got %d)", SDG_MAX_FIELDS, d->n_fields);
  if (d->precision < SDG_FP64 || d->precision > SDG_FP32_STATE_FP64_SOLVE)
    return fail(SDG_E_ARG, "unknown precision %d", d->precision);
  const int C = d->n_tri;
  P.C = C;
  P.F = d->n_fields;
  P.prec = d->precision;
  P.fp32 = d->precision != SDG_FP64;
  P.n_members = d->n_members < 1 ? 1 : d->n_members;
  P.member_off.assign(P.n_members + 1, 0);
  if (d->member_tri_off) {
    if (d->n_members < 1) return fail(SDG_E_MESH, "n_members must be >= 1 with member_tri_off");
    for (int m = 0; m <= P.n_members; ++m) P.member_off[m] = d->member_tri_off[m];
    if (P.member_off[0] != 0 || P.member_off[P.n_members] != C)
      return fail(SDG_E_MESH, "member_tri_off must start at 0 and end at n_tri");
    for (int m = 0; m < P.n_members; ++m)
      if (P.member_off[m + 1] <= P.member_off[m])
        return fail(SDG_E_MESH, "member %d has no columns", m);
  } else {
    if (P.n_members != 1) return fail(SDG_E_MESH, "n_members > 1 needs member_tri_off");
    P.member_off[1] = C;
  }
  std::vector<int32_t> col_member(C);
  for (int m = 0; m < P.n_members; ++m)
    for (int c = P.member_off[m]; c < P.member_off[m + 1]; ++c) col_member[c] = m;

  // layers and level offsets
  P.zoff.assign(C + 1, 0);
  P.n_prisms = 0;
  P.max_layers = 0;
  for (int c = 0; c < C; ++c) {
    const int n = d->nlayers[c];
    if (n < 1 || n > 65535) return fail(SDG_E_MESH, "column %d has %d layers (need 1..65535)", c, n);
    P.zoff[c + 1] = P.zoff[c] + (n + 1);
    P.n_prisms += n;
    P.max_layers = std::max(P.max_layers, n);
  }
  // triangles: vertex ids, orientation, level ordering
  for (int c = 0; c < C; ++c) {
    const int32_t* t = d->tri + 3 * c;
    for (int k = 0; k < 3; ++k)
      if (t[k] < 0 || t[k] >= d->n_vert) return fail(SDG_E_MESH, "triangle %d has vertex id %d out of range", c, t[k]);
    const double* a = d->vxy + 2 * t[0];
    const double* b = d->vxy + 2 * t[1];
    const double* e = d->vxy + 2 * t[2];
    const double jh = (b[0] - a[0]) * (e[1] - a[1]) - (e[0] - a[0]) * (b[1] - a[1]);
    if (!(jh > 0.0)) return fail(SDG_E_MESH, "triangle %d is not counter-clockwise (J_h = %g)", c, jh);
    const double* z = d->zlev + 3 * P.zoff[c];
    for (int l = 0; l < d->nlayers[c]; ++l)
      for (int v = 0; v < 3; ++v)
        if (!(z[3 * l + v] > z[3 * (l + 1) + v]))
          return fail(SDG_E_MESH, "column %d layer %d vertex %d has non-positive thickness", c, l, v);
  }
  // neighbours: symmetric, reversed shared edge, same member, conforming levels
  for (int c = 0; c < C; ++c) {
    for (int k = 0; k < 3; ++k) {
      const int c2 = d->nbr[3 * c + k];
      if (c2 == -1) continue;
      if (c2 < 0 || c2 >= C || c2 == c) return fail(SDG_E_MESH, "column %d edge %d has invalid neighbour %d", c, k, c2);
      if (col_member[c2] != col_member[c]) return fail(SDG_E_MESH, "column %d neighbours column %d of another member", c, c2);
      const int va = d->tri[3 * c + k], vb = d->tri[3 * c + (k + 1) % 3];
      int k2 = -1;
      for (int j = 0; j < 3; ++j)
        if (d->tri[3 * c2 + j] == vb && d->tri[3 * c2 + (j + 1) % 3] == va) k2 = j;
      if (k2 < 0) return fail(SDG_E_MESH, "columns %d and %d do not share edge %d in opposite directions", c, c2, k);
      if (d->nbr[3 * c2 + k2] != c) return fail(SDG_E_MESH, "neighbour relation %d -> %d is not symmetric", c, c2);
      const int nl = std::min(d->nlayers[c], d->nlayers[c2]);
      const double* z1 = d->zlev + 3 * P.zoff[c];
      const double* z2 = d->zlev + 3 * P.zoff[c2];
      const int a1 = k, b1 = (k + 1) % 3, a2 = (k2 + 1) % 3, b2 = k2;
      for (int lv = 0; lv <= nl; ++lv)
        if (z1[3 * lv + a1] != z2[3 * lv + a2] || z1[3 * lv + b1] != z2[3 * lv + b2])
          return fail(SDG_E_MESH, "levels of columns %d and %d differ on their shared edge (level %d)", c, c2, lv);
    }
  }
  // cells
  P.n_cells = (C + kCell - 1) / kCell;
  P.CS = P.n_cells * kCell;
  P.cell_base.assign(P.n_cells + 1, 0);
  P.cell_lbase.assign(P.n_cells + 1, 0);
  P.cell_depth.assign(P.n_cells, 0);
  int64_t sb = 0, lb = 0;
  for (int t = 0; t < kTileChoices; ++t) P.n_tiles[t] = 0;
  for (int k = 0; k < P.n_cells; ++k) {
    int depth = 0;
    for (int c = k * kCell; c < std::min(C, (k + 1) * kCell); ++c) depth = std::max(depth, (int)d->nlayers[c]);
    P.cell_depth[k] = depth;
    P.cell_base[k] = (int32_t)sb;
    P.cell_lbase[k] = (int32_t)lb;
    sb += (int64_t)depth * kCell;
    lb += (int64_t)(depth + 1) * kCell;
    for (int t = 0; t < kTileChoices; ++t)
      P.n_tiles[t] += (depth + kTileLayerOptions[t] - 1) / kTileLayerOptions[t];
    if (sb > INT32_MAX / 2 || lb > INT32_MAX / 2) return fail(SDG_E_UNSUPPORTED, "mesh too large for 32-bit slot indices");
  }
  P.cell_base[P.n_cells] = (int32_t)sb;
  P.cell_lbase[P.n_cells] = (int32_t)lb;
  P.halo_off.assign(P.n_cells + 1, 0);
  for (int c = 0; c < C; ++c)
    for (int e = 0; e < 3; ++e) {
      const int c2 = d->nbr[3 * c + e];
      if (c2 >= 0 && c2 / kCell != c / kCell) ++P.halo_off[c / kCell + 1];
    }
  P.cell_order.resize(P.n_cells);
  for (int k = 0; k < P.n_cells; ++k) P.cell_order[k] = k;
  std::stable_sort(P.cell_order.begin(), P.cell_order.end(),
                   [&](int32_t x, int32_t y) { return P.cell_depth[x] > P.cell_depth[y]; });
  P.halo_max = 0;
  for (int k = 0; k < P.n_cells; ++k) {
    P.halo_max = std::max(P.halo_max, P.halo_off[k + 1]);
    P.halo_off[k + 1] += P.halo_off[k];
  }
  P.n_slots = sb;
  P.n_lslots = lb;
  // kernels address a field's 6 node rows (and the velocity's) with 32-bit
  // byte offsets
  if ((uint64_t)6 * (uint64_t)sb * 8u >= ((uint64_t)1 << 32) || (uint64_t)3 * (uint64_t)lb * 8u >= ((uint64_t)1 << 32))
    return fail(SDG_E_UNSUPPORTED, "mesh has %lld prism slots; at most %lld are supported", (long long)sb,
                (long long)((((uint64_t)1 << 32) - 1) / 48));

  // workspace
  const size_t es = P.fp32 ? 4 : 8;
  P.state_bytes = (size_t)P.F * 6 * (size_t)P.n_slots * es;
  P.velocity_bytes = (size_t)3 * 6 * (size_t)P.n_slots * es;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
  P.o_cell_base = take(sizeof(int32_t) * (P.n_cells + 1));
  P.o_cell_lbase = take(sizeof(int32_t) * (P.n_cells + 1));
  P.o_nlay = take(sizeof(int32_t) * P.CS);
  P.o_nbr_slot = take(sizeof(int32_t) * 3 * P.CS);
  P.o_nbr_meta = take(sizeof(int32_t) * 3 * P.CS);
  P.o_nbr_col = take(sizeof(int32_t) * 3 * P.CS);
  P.o_col_member = take(sizeof(int32_t) * P.CS);
  P.o_member_off = take(sizeof(int32_t) * (P.n_members + 1));
  P.o_geo = take(sizeof(double) * kGeoRows * P.CS);
  P.o_geo32 = take(sizeof(float) * kGeoRows * P.CS);
  P.o_xy = take(sizeof(double) * 6 * P.CS);
  P.o_zl = take(sizeof(double) * 3 * (size_t)P.n_lslots);
  P.o_zl32 = take(sizeof(float) * 3 * (size_t)P.n_lslots);
  for (int t = 0; t < kTileChoices; ++t) P.o_tiles[t] = take(sizeof(WgTile) * std::max(P.n_tiles[t], 1));
  // per-bucket walks are at least 8 layers long: no more tiles than the 8-layer table
  P.o_tiles_bucket = take(sizeof(WgTile) * std::max(P.n_tiles[3], 1));
  P.o_stage_a = take(P.state_bytes);
  P.o_stage_b = take(P.state_bytes);
  P.o_scratch = take(sizeof(double) * (size_t)(18 + 6 * P.F) * (size_t)P.n_slots);
  P.o_tfac = take(sizeof(double) * 18 * (size_t)P.n_slots);   // the adjoint's transposed factors
  P.o_colmass = take(sizeof(double) * (size_t)P.F * P.CS);
  P.o_msum = take(sizeof(double) * (size_t)P.F * P.n_members);
  P.o_flag = take(sizeof(int32_t) * 64);
  P.o_kpart = take(sizeof(double) * (size_t)P.max_layers * (size_t)P.n_cells);
  P.o_kh = take(sizeof(double) * (size_t)P.CS);
  P.o_hface = take(sizeof(double) * 15 * (size_t)P.CS);
  P.o_hoff = take(sizeof(int32_t) * (P.n_cells + 1));
  P.o_hslot = take(sizeof(int32_t) * std::max<size_t>(P.halo_off[P.n_cells], 1));
  P.o_hdepth = take(sizeof(int32_t) * std::max<size_t>(P.halo_off[P.n_cells], 1));
  P.o_hidx = take(sizeof(int32_t) * 3 * (size_t)P.CS);
  P.o_corder = take(sizeof(int32_t) * (size_t)P.n_cells);
  P.total = o;
  return SDG_OK;
}

class DeviceGuard {
 public:
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
    if (prev_ != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev_ >= 0) (void)hipSetDevice(prev_);
  }

 private:
  int prev_ = -1;
};

// ---------------------------------------------------------------------------
// Static scratch of sdg_mass_noalloc: each device holds its own copy of this
// array from the first context created on it until the process ends.  Host
// code never passes the array's name to a kernel (on the host it is a
// stand-in, not a device address): it uses the address that
// hipGetSymbolAddress returned on that device, kept per device below.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocDoubles = size_t(8) << 20;   // 64 MiB
static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Looks up this device's copy of the scratch array once; the device must be
// current.  Called by sdg_create.
hipError_t bind_static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = static_cast<double*>(p);
  return hipSuccess;
}

double* static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace

struct sdg_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool have_mesh = false;
  Plan plan;
  DevMesh dm{};
  char* ws = nullptr;
  WgTile* tiles[kTileChoices] = {};
  WgTile* tiles_bucket = nullptr;     // per-depth-bucket walk table (tile_choice == kBucketChoice)
  int n_tiles_bucket = 0;
  int walk_layers[kDepthBuckets] = {};
  // launch shape of the stage kernel (chosen by sdg_set_tuning / sdg_autotune)
  int tile_choice = 1;   // index into kTileLayerOptions (2 layers)
  int xcd = 1;
  int persistent = 0;
  int n_cu = 1;          // compute units of the device
  // captured step
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  bool graph_valid = false;
  int32_t* member_off_dev = nullptr;
  double* colmass = nullptr;
  double* msum = nullptr;
  int32_t* flag = nullptr;
  double* kpart = nullptr;
  double* kh = nullptr;     // per-column horizontal diffusivity (workspace)
  double* hface = nullptr;  // per-face neighbour table of the horizontal diffusion (workspace)
  void* stage_a = nullptr;
  void* stage_b = nullptr;
  double* scratch = nullptr;
  // the solve scratch holds the block-Thomas factors of (kappa, efac_dt, eta),
  // tfac those of the transposed system for tfac_dt
  bool efac_valid = false;
  double efac_dt = 0.0;
  double* tfac = nullptr;
  bool tfac_valid = false;
  double tfac_dt = 0.0;
  // state set by the caller
  bool have_params = false;
  double dt = 0.0, eta = 4.0;
  double t_ext[kMaxFields] = {0, 0, 0, 0};
  bool w_zero = false, check_finite = false;
  int scheme = SDG_SCHEME_SSPRK3_LIE;
  double kh_scale = 0.0;   // horizontal diffusion off when 0
  const void* U = nullptr;
  const double* kappa = nullptr;
  void* state = nullptr;
};

extern "C" {

int sdg_abi_version(void) { return SDG_ABI_VERSION; }

const char* sdg_last_error(void) { return g_err.c_str(); }

sdg_status sdg_query_layout(const sdg_mesh_desc* mesh, sdg_layout* out) {
  if (!out) return fail(SDG_E_ARG, "output layout is NULL");
  Plan P;
  sdg_status st = plan_mesh(mesh, P);
  if (st != SDG_OK) return st;
  out->n_prisms = P.n_prisms;
  out->n_slots = P.n_slots;
  out->n_cells = P.n_cells;
  out->max_layers = P.max_layers;
  out->n_fields = P.F;
  out->state_elem_bytes = P.fp32 ? 4 : 8;
  out->state_bytes = P.state_bytes;
  out->velocity_bytes = P.velocity_bytes;
  out->workspace_bytes = P.total;
  g_err.clear();
  return SDG_OK;
}

sdg_status sdg_prism_slots(const sdg_mesh_desc* mesh, int64_t* host_slots) {
  if (!host_slots) return fail(SDG_E_ARG, "host_slots is NULL");
  Plan P;
  sdg_status st = plan_mesh(mesh, P);
  if (st != SDG_OK) return st;
  int64_t q = 0;
  for (int c = 0; c < P.C; ++c) {
    const int k = c / kCell, lane = c % kCell;
    for (int l = 0; l < mesh->nlayers[c]; ++l) host_slots[q++] = (int64_t)P.cell_base[k] + (int64_t)l * kCell + lane;
  }
  g_err.clear();
  return SDG_OK;
}

sdg_status sdg_create(sdg_ctx** out, int device, void* hip_stream) {
  if (!out) return fail(SDG_E_ARG, "out is NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (device < 0 || device >= n) return fail(SDG_E_ARG, "device %d out of range (%d devices)", device, n);
  sdg_ctx* c = new (std::nothrow) sdg_ctx();
  if (!c) return fail(SDG_E_ARG, "out of host memory");
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  e = hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "hipDeviceGetAttribute(multiprocessor count)");
  }
  if (c->n_cu < 1) c->n_cu = 1;
  {
    DeviceGuard g(device);
    e = bind_static_scratch(device);
  }
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "hipGetSymbolAddress(static scratch)");
  }
  *out = c;
  g_err.clear();
  return SDG_OK;
}

namespace {
void drop_graph(sdg_ctx* ctx) {
  if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  ctx->graph_exec = nullptr;
  ctx->graph = nullptr;
  ctx->graph_valid = false;
}
}  // namespace

sdg_status sdg_destroy(sdg_ctx* ctx) {
  if (!ctx) return SDG_OK;
  {
    DeviceGuard g(ctx->device);
    drop_graph(ctx);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  }
  delete ctx;
  return SDG_OK;
}

sdg_status sdg_mesh_upload(sdg_ctx* ctx, const sdg_mesh_desc* mesh, void* dev_workspace, size_t ws_bytes) {
  if (!ctx) return fail(SDG_E_ARG, "context is NULL");
  ctx->have_mesh = false;
  ctx->have_params = false;   // t_ext and the horizontal diffusivity belong to the mesh
  ctx->kh_scale = 0.0;
  ctx->graph_valid = false;
  ctx->efac_valid = false;
  ctx->tfac_valid = false;
  ctx->U = nullptr;
  ctx->kappa = nullptr;
  ctx->state = nullptr;
  Plan P;
  sdg_status st = plan_mesh(mesh, P);
  if (st != SDG_OK) return st;
  if (!dev_workspace) return fail(SDG_E_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(dev_workspace) & 255) return fail(SDG_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < P.total)
    return fail(SDG_E_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, P.total);
  DeviceGuard g(ctx->device);
  const int CS = P.CS, C = P.C;
  // host images of the device tables
  std::vector<int32_t> nlay(CS, 0), nbr_slot(3 * (size_t)CS, -1), nbr_meta(3 * (size_t)CS, 0),
      nbr_col(3 * (size_t)CS, -1), colmem(CS, -1);
  std::vector<double> xy(6 * (size_t)CS, 0.0), zl(3 * (size_t)P.n_lslots, 0.0);
  std::vector<WgTile> tiles[kTileChoices];
  for (int t = 0; t < kTileChoices; ++t) {
    const int T = kTileLayerOptions[t];
    tiles[t].reserve(P.n_tiles[t]);
    for (int k = 0; k < P.n_cells; ++k)
      for (int l0 = 0; l0 < P.cell_depth[k]; l0 += T)
        tiles[t].push_back({k, (uint16_t)l0, (uint16_t)std::min(T, P.cell_depth[k] - l0)});
    // Full tiles first, shorter ones (a cell's last segment) after them, each
    // group in cell order.  A persistent grid strides through the table with
    // a stride that is a multiple of 8; in cell order every workgroup would
    // get the same segment of each cell it visits, and those that get the
    // short last segments would idle while the others finish.  The shorter
    // tiles also make up the tail of a one-tile-per-workgroup launch.
    std::stable_sort(tiles[t].begin(), tiles[t].end(),
                     [](const WgTile& x, const WgTile& y) { return x.nlay > y.nlay; });
  }
  for (int m = 0; m < P.n_members; ++m)
    for (int c = P.member_off[m]; c < P.member_off[m + 1]; ++c) colmem[c] = m;
  // other-cell neighbours per cell, column by column, faces in order
  const size_t n_halo = (size_t)P.halo_off[P.n_cells];
  std::vector<int32_t> hslot(std::max<size_t>(n_halo, 1), 0), hdepth(std::max<size_t>(n_halo, 1), 0),
      hidx(3 * (size_t)CS, -1);
  {
    // each cell's list sorted by the neighbour's slot (then column and face),
    // so that consecutive entries read nearby addresses
    std::vector<std::array<int32_t, 3>> ent;   // (neighbour slot, column, face)
    for (int k = 0; k < P.n_cells; ++k) {
      ent.clear();
      for (int c = k * kCell; c < std::min(C, (k + 1) * kCell); ++c)
        for (int e = 0; e < 3; ++e) {
          const int c2 = mesh->nbr[3 * c + e];
          if (c2 < 0 || c2 / kCell == k) continue;
          ent.push_back({P.cell_base[c2 / kCell] + c2 % kCell, c, e});
        }
      std::sort(ent.begin(), ent.end());
      for (size_t i = 0; i < ent.size(); ++i) {
        const int j = P.halo_off[k] + (int)i;
        const int c = ent[i][1], e = ent[i][2], c2 = mesh->nbr[3 * c + e];
        hslot[j] = ent[i][0];
        hdepth[j] = mesh->nlayers[c2];
        hidx[e * (size_t)CS + c] = (int32_t)i;
      }
    }
  }
  for (int c = 0; c < C; ++c) {
    const int k = c / kCell, lane = c % kCell;
    const int n = mesh->nlayers[c];
    nlay[c] = n;
    for (int v = 0; v < 3; ++v) {
      const int vid = mesh->tri[3 * c + v];
      xy[(2 * v) * (size_t)CS + c] = mesh->vxy[2 * vid];
      xy[(2 * v + 1) * (size_t)CS + c] = mesh->vxy[2 * vid + 1];
    }
    for (int e = 0; e < 3; ++e) {
      const int c2 = mesh->nbr[3 * c + e];
      if (c2 < 0) continue;
      const int va = mesh->tri[3 * c + e], vb = mesh->tri[3 * c + (e + 1) % 3];
      int k2 = 0;
      for (int j = 0; j < 3; ++j)
        if (mesh->tri[3 * c2 + j] == vb && mesh->tri[3 * c2 + (j + 1) % 3] == va) k2 = j;
      nbr_slot[e * (size_t)CS + c] = P.cell_base[c2 / kCell] + c2 % kCell;
      nbr_meta[e * (size_t)CS + c] = (mesh->nlayers[c2] << 2) | k2;
      nbr_col[e * (size_t)CS + c] = c2;
    }
    const double* z = mesh->zlev + 3 * P.zoff[c];
    for (int lv = 0; lv <= n; ++lv)
      for (int v = 0; v < 3; ++v)
        zl[v * (size_t)P.n_lslots + P.cell_lbase[k] + (size_t)lv * kCell + lane] = z[3 * lv + v];
  }
  char* ws = static_cast<char*>(dev_workspace);
  hipStream_t s = ctx->stream;
  struct Cp { size_t off; const void* src; size_t bytes; };
  const Cp cps[] = {
      {P.o_cell_base, P.cell_base.data(), sizeof(int32_t) * P.cell_base.size()},
      {P.o_cell_lbase, P.cell_lbase.data(), sizeof(int32_t) * P.cell_lbase.size()},
      {P.o_nlay, nlay.data(), sizeof(int32_t) * nlay.size()},
      {P.o_nbr_slot, nbr_slot.data(), sizeof(int32_t) * nbr_slot.size()},
      {P.o_nbr_meta, nbr_meta.data(), sizeof(int32_t) * nbr_meta.size()},
      {P.o_nbr_col, nbr_col.data(), sizeof(int32_t) * nbr_col.size()},
      {P.o_col_member, colmem.data(), sizeof(int32_t) * colmem.size()},
      {P.o_member_off, P.member_off.data(), sizeof(int32_t) * P.member_off.size()},
      {P.o_xy, xy.data(), sizeof(double) * xy.size()},
      {P.o_zl, zl.data(), sizeof(double) * zl.size()},
      {P.o_tiles[0], tiles[0].data(), sizeof(WgTile) * tiles[0].size()},
      {P.o_tiles[1], tiles[1].data(), sizeof(WgTile) * tiles[1].size()},
      {P.o_tiles[2], tiles[2].data(), sizeof(WgTile) * tiles[2].size()},
      {P.o_tiles[3], tiles[3].data(), sizeof(WgTile) * tiles[3].size()},
      {P.o_tiles[4], tiles[4].data(), sizeof(WgTile) * tiles[4].size()},
      {P.o_tiles[5], tiles[5].data(), sizeof(WgTile) * tiles[5].size()},
      {P.o_tiles[6], tiles[6].data(), sizeof(WgTile) * tiles[6].size()},
      {P.o_hoff, P.halo_off.data(), sizeof(int32_t) * P.halo_off.size()},
      {P.o_hslot, hslot.data(), sizeof(int32_t) * hslot.size()},
      {P.o_hdepth, hdepth.data(), sizeof(int32_t) * hdepth.size()},
      {P.o_hidx, hidx.data(), sizeof(int32_t) * hidx.size()},
      {P.o_corder, P.cell_order.data(), sizeof(int32_t) * P.cell_order.size()},
  };
  static_assert(kTileChoices == 7, "one copy per tile table");
  for (const Cp& cp : cps) {
    if (cp.bytes == 0) continue;
    hipError_t e = hipMemcpyAsync(ws + cp.off, cp.src, cp.bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync (mesh upload)");
  }
  DevMesh& dm = ctx->dm;
  dm.n_cols = C;
  dm.n_cells = P.n_cells;
  dm.n_col_slots = CS;
  dm.max_layers = P.max_layers;
  dm.n_slots = P.n_slots;
  dm.n_lslots = P.n_lslots;
  dm.cell_base = reinterpret_cast<const int32_t*>(ws + P.o_cell_base);
  dm.cell_lbase = reinterpret_cast<const int32_t*>(ws + P.o_cell_lbase);
  dm.nlay = reinterpret_cast<const int32_t*>(ws + P.o_nlay);
  dm.nbr_slot = reinterpret_cast<const int32_t*>(ws + P.o_nbr_slot);
  dm.nbr_meta = reinterpret_cast<const int32_t*>(ws + P.o_nbr_meta);
  dm.nbr_col = reinterpret_cast<const int32_t*>(ws + P.o_nbr_col);
  dm.halo_max = P.halo_max;
  dm.halo_off = reinterpret_cast<const int32_t*>(ws + P.o_hoff);
  dm.halo_slot = reinterpret_cast<const int32_t*>(ws + P.o_hslot);
  dm.halo_depth = reinterpret_cast<const int32_t*>(ws + P.o_hdepth);
  dm.halo_idx = reinterpret_cast<const int32_t*>(ws + P.o_hidx);
  dm.cell_order = reinterpret_cast<const int32_t*>(ws + P.o_corder);
  dm.geo = reinterpret_cast<const double*>(ws + P.o_geo);
  dm.geo32 = reinterpret_cast<const float*>(ws + P.o_geo32);
  dm.zl = reinterpret_cast<const double*>(ws + P.o_zl);
  dm.zl32 = reinterpret_cast<const float*>(ws + P.o_zl32);
  dm.xy = reinterpret_cast<const double*>(ws + P.o_xy);
  dm.col_member = reinterpret_cast<const int32_t*>(ws + P.o_col_member);
  hipError_t e = launch_geometry(dm, reinterpret_cast<double*>(ws + P.o_geo), reinterpret_cast<float*>(ws + P.o_geo32), s);
  if (e != hipSuccess) return hip_fail(e, "geometry kernel launch");
  e = launch_z32(dm, reinterpret_cast<float*>(ws + P.o_zl32), s);
  if (e != hipSuccess) return hip_fail(e, "level conversion launch");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "mesh upload");
  ctx->plan = std::move(P);
  const Plan& Q = ctx->plan;
  ctx->ws = ws;
  for (int t = 0; t < kTileChoices; ++t) ctx->tiles[t] = reinterpret_cast<WgTile*>(ws + Q.o_tiles[t]);
  ctx->tiles_bucket = reinterpret_cast<WgTile*>(ws + Q.o_tiles_bucket);
  ctx->n_tiles_bucket = 0;
  if (ctx->tile_choice == kBucketChoice) ctx->tile_choice = 1;   // the table belongs to the old mesh
  ctx->member_off_dev = reinterpret_cast<int32_t*>(ws + Q.o_member_off);
  ctx->colmass = reinterpret_cast<double*>(ws + Q.o_colmass);
  ctx->msum = reinterpret_cast<double*>(ws + Q.o_msum);
  ctx->flag = reinterpret_cast<int32_t*>(ws + Q.o_flag);
  ctx->kpart = reinterpret_cast<double*>(ws + Q.o_kpart);
  ctx->kh = reinterpret_cast<double*>(ws + Q.o_kh);
  ctx->hface = reinterpret_cast<double*>(ws + Q.o_hface);
  ctx->stage_a = ws + Q.o_stage_a;
  ctx->stage_b = ws + Q.o_stage_b;
  ctx->scratch = reinterpret_cast<double*>(ws + Q.o_scratch);
  ctx->tfac = reinterpret_cast<double*>(ws + Q.o_tfac);
  ctx->have_mesh = true;
  g_err.clear();
  return SDG_OK;
}

sdg_status sdg_set_params(sdg_ctx* ctx, const sdg_params* p) {
  if (!ctx || !p) return fail(SDG_E_ARG, "context or params is NULL");
  if (!ctx->have_mesh) return fail(SDG_E_STATE, "sdg_set_params needs an uploaded mesh");
  if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return fail(SDG_E_ARG, "dt must be finite and > 0 (got %g)", p->dt);
  const double eta = p->penalty_eta > 0.0 ? p->penalty_eta : 4.0;
  if (!std::isfinite(eta)) return fail(SDG_E_ARG, "penalty_eta must be finite");
  double text[kMaxFields] = {};
  for (int f = 0; f < ctx->plan.F; ++f) {
    const double v = p->t_ext ? p->t_ext[f] : 0.0;
    if (!std::isfinite(v)) return fail(SDG_E_ARG, "t_ext[%d] is not finite", f);
    text[f] = v;
  }
  if (p->time_scheme != SDG_SCHEME_SSPRK3_LIE && p->time_scheme != SDG_SCHEME_SPLIT_IMEX)
    return fail(SDG_E_ARG, "unknown time_scheme %d", p->time_scheme);
  if (!(p->okubo_scale >= 0.0) || !std::isfinite(p->okubo_scale))
    return fail(SDG_E_ARG, "okubo_scale must be finite and >= 0 (got %g)", p->okubo_scale);
  if (p->okubo_scale > 0.0) {
    // Okubo: K = 0.0103 l^1.15 cm^2/s with l in cm = 0.0103 100^1.15 1e-4 l^1.15 m^2/s, l in m
    DeviceGuard g(ctx->device);
    const double coef = p->okubo_scale * 0.0103 * std::pow(100.0, 1.15) * 1.0e-4;
    hipError_t e = launch_hdiff_setup(ctx->dm, coef, eta, ctx->kh, ctx->hface, ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "horizontal diffusivity launch");
  }
  for (int f = 0; f < ctx->plan.F; ++f) ctx->t_ext[f] = text[f];
  ctx->scheme = p->time_scheme;
  ctx->kh_scale = p->okubo_scale;
  ctx->dt = p->dt;
  ctx->eta = eta;
  ctx->w_zero = p->w_is_zero != 0;
  ctx->check_finite = p->check_finite != 0;
  ctx->graph_valid = false;
  ctx->efac_valid = false;
  ctx->tfac_valid = false;
  ctx->have_params = true;
  g_err.clear();
  return SDG_OK;
}

sdg_status sdg_set_velocity(sdg_ctx* ctx, const void* dev_uvw) {
  if (!ctx || !dev_uvw) return fail(SDG_E_ARG, "context or velocity is NULL");
  if (!ctx->have_mesh) return fail(SDG_E_STATE, "sdg_set_velocity needs an uploaded mesh");
  ctx->U = dev_uvw;
  ctx->graph_valid = false;
  g_err.clear();
  return SDG_OK;
}

sdg_status sdg_set_diffusivity(sdg_ctx* ctx, const double* dev_kappa) {
  if (!ctx || !dev_kappa) return fail(SDG_E_ARG, "context or diffusivity is NULL");
  if (!ctx->have_mesh) return fail(SDG_E_STATE, "sdg_set_diffusivity needs an uploaded mesh");
  ctx->kappa = dev_kappa;
  ctx->graph_valid = false;
  ctx->efac_valid = false;
  ctx->tfac_valid = false;
  g_err.clear();
  return SDG_OK;
}

sdg_status sdg_set_fields(sdg_ctx* ctx, void* dev_state) {
  if (!ctx || !dev_state) return fail(SDG_E_ARG, "context or state is NULL");
  if (!ctx->have_mesh) return fail(SDG_E_STATE, "sdg_set_fields needs an uploaded mesh");
  ctx->state = dev_state;
  ctx->graph_valid = false;
  g_err.clear();
  return SDG_OK;
}

namespace {

sdg_status check_explicit(sdg_ctx* ctx, const char* who) {
  if (!ctx) return fail(SDG_E_ARG, "%s: context is NULL", who);
  if (!ctx->have_mesh) return fail(SDG_E_STATE, "%s needs an uploaded mesh", who);
  if (!ctx->have_params) return fail(SDG_E_STATE, "%s needs sdg_set_params", who);
  if (!ctx->U) return fail(SDG_E_STATE, "%s needs sdg_set_velocity", who);
  return SDG_OK;
}

StageArgs stage_args(sdg_ctx* ctx, const void* Tn, const void* Ts, void* Tout, double a, double b, double dt) {
  StageArgs s{};
  s.m = ctx->dm;
  if (ctx->tile_choice == kBucketChoice) {
    s.tiles = ctx->tiles_bucket;
    s.n_tiles = ctx->n_tiles_bucket;
    s.tile_layers = kBucketWalkMax;
  } else {
    s.tiles = ctx->tiles[ctx->tile_choice];
    s.n_tiles = ctx->plan.n_tiles[ctx->tile_choice];
    s.tile_layers = kTileLayerOptions[ctx->tile_choice];
  }
  s.xcd = ctx->xcd;
  s.persistent = ctx->persistent;
  s.n_cu = ctx->n_cu;
  s.n_fields = ctx->plan.F;
  s.Tn = Tn;
  s.Ts = Ts;
  s.Tout = Tout;
  s.U = ctx->U;
  for (int f = 0; f < kMaxFields; ++f) s.t_ext[f] = ctx->t_ext[f];
  s.dt = dt;
  s.a = a;
  s.b = b;
  return s;
}

// The horizontal diffusion part of an explicit stage (forward or adjoint)
// whose other terms were just written: Tout += c1 M^-1 D(Ts) (and
// Tout2 += c2 M^-1 D(Ts)).  No launch when horizontal diffusion is off.
hipError_t enqueue_hdiff(sdg_ctx* ctx, const void* Ts, void* Tout, void* Tout2, double c1, double c2,
                         hipStream_t strm) {
  if (!(ctx->kh_scale > 0.0)) return hipSuccess;
  HdiffArgs h{};
  h.m = ctx->dm;
  h.tiles = ctx->tiles[1];
  h.n_tiles = ctx->plan.n_tiles[1];
  h.tile_layers = kTileLayerOptions[1];
  h.n_fields = ctx->plan.F;
  h.Ts = Ts;
  h.Tout = Tout;
  h.Tout2 = Tout2;
  h.c1 = c1;
  h.c2 = c2;
  h.kh = ctx->kh;
  h.hface = ctx->hface;
  return launch_hdiff(h, ctx->plan.fp32, strm);
}

hipError_t hdiff_after_stage(sdg_ctx* ctx, const StageArgs& s, double c1, double c2, hipStream_t strm) {
  return enqueue_hdiff(ctx, s.Ts, s.Tout, s.Tout2, c1, c2, strm);
}

constexpr double kRk[3][2] = {{0.0, 1.0}, {0.75, 0.25}, {1.0 / 3.0, 2.0 / 3.0}};

sdg_status enqueue_stage(sdg_ctx* ctx, int stage, const void* Tn, const void* Ts, void* Tout,
                         hipStream_t strm) {
  StageArgs s = stage_args(ctx, Tn, Ts, Tout, kRk[stage][0], kRk[stage][1], ctx->dt);
  hipError_t e = launch_stage(s, ctx->plan.fp32, ctx->w_zero, false, stage > 0, strm);
  if (e == hipSuccess) e = hdiff_after_stage(ctx, s, kRk[stage][1] * ctx->dt, 0.0, strm);
  if (e != hipSuccess) return hip_fail(e, "rk_stage launch");
  return SDG_OK;
}

SolveArgs solve_args(sdg_ctx* ctx, const void* Tstar, void* Tout, double dt) {
  SolveArgs a{};
  a.m = ctx->dm;
  a.n_fields = ctx->plan.F;
  a.Tstar = Tstar;
  a.Tout = Tout;
  a.kappa = ctx->kappa;
  a.scratch = ctx->scratch;
  a.dt = dt;
  a.eta = ctx->eta;
  return a;
}

// The block-Thomas factors for a solve over dt: kept in the solve scratch
// until kappa, the parameters or the mesh change, or the adjoint's
// transposed solve reuses the scratch.
sdg_status ensure_factors(sdg_ctx* ctx, double dt, hipStream_t strm) {
  if (ctx->efac_valid && ctx->efac_dt == dt) return SDG_OK;
  hipError_t e = launch_vsolve(solve_args(ctx, nullptr, nullptr, dt), ctx->plan.fp32, ctx->plan.prec == SDG_FP32,
                               true, strm);
  if (e != hipSuccess) return hip_fail(e, "column factor launch");
  ctx->efac_valid = true;
  ctx->efac_dt = dt;
  return SDG_OK;
}

// The transposed system's factors for the adjoint's solve over dt, kept in
// their own array (the forward factors stay valid).
sdg_status ensure_tfactors(sdg_ctx* ctx, double dt, hipStream_t strm) {
  if (ctx->tfac_valid && ctx->tfac_dt == dt) return SDG_OK;
  hipError_t e = launch_tsolve(ctx->dm, ctx->plan.F, nullptr, nullptr, ctx->kappa, ctx->tfac, dt, ctx->eta, true, strm);
  if (e != hipSuccess) return hip_fail(e, "transposed column factor launch");
  ctx->tfac_valid = true;
  ctx->tfac_dt = dt;
  return SDG_OK;
}

// the solve's dt in a step of the context's scheme
double step_solve_dt(const sdg_ctx* ctx) { return ctx->scheme == SDG_SCHEME_SPLIT_IMEX ? 0.5 * ctx->dt : ctx->dt; }

sdg_status enqueue_solve(sdg_ctx* ctx, const void* Tstar, void* Tout, double dt, hipStream_t strm) {
  sdg_status st = ensure_factors(ctx, dt, strm);
  if (st != SDG_OK) return st;
  hipError_t e = launch_vsolve(solve_args(ctx, Tstar, Tout, dt), ctx->plan.fp32, ctx->plan.prec == SDG_FP32,
                               false, strm);
  if (e != hipSuccess) return hip_fail(e, "vertical solve launch");
  return SDG_OK;
}

// One split-IMEX step (x_0 = X), three launches:
//   A <- y   = x_0 + dt/2 M^-1 R(x_0),  B <- x_0 - 2 y     explicit half step
//   A <- x_h = (M - dt/2 A)^-1 M y  (in place)            vertically implicit half step
//   X <- B + 2 (x_h + dt/2 M^-1 R(x_h))                    explicit full step
// The last line is x_0 + 2 (x_h - y) + dt M^-1 R(x_h), and 2 (x_h - y) is
// dt M^-1 A x_h by the half step's own system.
// With xh, the half step's solve writes x_h there (the caller's buffer)
// instead of back into the stage buffer, and the second stage reads it there.
sdg_status enqueue_imex_step(sdg_ctx* ctx, hipStream_t strm, void* xh = nullptr) {
  void* X = ctx->state;
  void* A = ctx->stage_a;
  void* B = ctx->stage_b;
  void* H = xh ? xh : A;
  const double h = 0.5 * ctx->dt;
  StageArgs s1 = stage_args(ctx, nullptr, X, A, 0.0, 1.0, h);
  s1.Tout2 = B;
  hipError_t e = launch_stage(s1, ctx->plan.fp32, ctx->w_zero, false, false, strm);
  if (e == hipSuccess) e = hdiff_after_stage(ctx, s1, h, -2.0 * h, strm);
  if (e != hipSuccess) return hip_fail(e, "split-IMEX half step launch");
  sdg_status st = enqueue_solve(ctx, A, H, h, strm);
  if (st != SDG_OK) return st;
  StageArgs s2 = stage_args(ctx, B, H, X, 1.0, 2.0, h);
  e = launch_stage(s2, ctx->plan.fp32, ctx->w_zero, false, true, strm);
  if (e == hipSuccess) e = hdiff_after_stage(ctx, s2, 2.0 * h, 0.0, strm);
  if (e != hipSuccess) return hip_fail(e, "split-IMEX full step launch");
  return SDG_OK;
}

// One step on the set fields in the context's scheme.  SSP-RK3 + Lie: three
// stages through the two workspace stage buffers, then the column solve back
// into the state.
sdg_status enqueue_step(sdg_ctx* ctx, hipStream_t strm) {
  if (ctx->scheme == SDG_SCHEME_SPLIT_IMEX) return enqueue_imex_step(ctx, strm);
  void* X = ctx->state;
  void* A = ctx->stage_a;
  void* B = ctx->stage_b;
  sdg_status st;
  if ((st = enqueue_stage(ctx, 0, nullptr, X, A, strm)) != SDG_OK) return st;
  if ((st = enqueue_stage(ctx, 1, X, A, B, strm)) != SDG_OK) return st;
  if ((st = enqueue_stage(ctx, 2, X, B, A, strm)) != SDG_OK) return st;
  return enqueue_solve(ctx, A, X, ctx->dt, strm);
}

}  // namespace

sdg_status sdg_rhs_3d(sdg_ctx* ctx, const void* dev_T, void* dev_L) {
  sdg_status st = check_explicit(ctx, "sdg_rhs_3d");
  if (st != SDG_OK) return st;
  if (!dev_T || !dev_L) return fail(SDG_E_ARG, "sdg_rhs_3d: NULL buffer");
  if (dev_T == dev_L) return fail(SDG_E_ARG, "sdg_rhs_3d: output must not alias input");
  DeviceGuard g(ctx->device);
  StageArgs s = stage_args(ctx, nullptr, dev_T, dev_L, 0.0, 1.0, ctx->dt);
  hipError_t e = launch_stage(s, ctx->plan.fp32, ctx->w_zero, true, false, ctx->stream);
  if (e == hipSuccess) e = hdiff_after_stage(ctx, s, 1.0, 0.0, ctx->stream);
  if (e != hipSuccess) return hip_fail(e, "rhs_3d launch");
  g_err.clear();
  return SDG_OK;
}

sdg_status sdg_rk_stage(sdg_ctx* ctx, int stage, const void* dev_Tn, const void* dev_Ts, void* dev_Tout) {
  sdg_status st = check_explicit(ctx, "sdg_rk_stage");
  if (st != SDG_OK) return st;
  if (stage < 0 || stage > 2) return fail(SDG_E_ARG, "sdg_rk_stage: stage must be 0, 1 or 2 (got %d)", stage);
  if (!dev_Ts || !dev_Tout || (stage > 0 && !dev_Tn)) return fail(SDG_E_ARG, "sdg_rk_stage: NULL buffer");
  if (dev_Tout == dev_Ts || (stage > 0 && dev_Tout == dev_Tn))
    return fail(SDG_E_ARG, "sdg_rk_stage: output must not alias an input");
  DeviceGuard g(ctx->device);
  st = enqueue_stage(ctx, stage, dev_Tn, dev_Ts, dev_Tout, ctx->stream);
  if (st == SDG_OK) g_err.clear();
  return st;
}

sdg_status sdg_vertical_implicit_solve(sdg_ctx* ctx, const void* dev_Tstar, void* dev_Tout) {
  if (!ctx) return fail(SDG_E_ARG, "context is NULL");
  if (!ctx->have_mesh) return fail(SDG_E_STATE, "sdg_vertical_implicit_solve needs an uploaded mesh");
  if (!ctx->have_params) return fail(SDG_E_STATE, "sdg_vertical_implicit_solve needs sdg_set_params");
  if (!ctx->kappa) return fail(SDG_E_STATE, "sdg_vertical_implicit_solve needs sdg_set_diffusivity");
  if (!dev_Tstar || !dev_Tout) return fail(SDG_E_ARG, "sdg_vertical_implicit_solve: NULL buffer");
  DeviceGuard g(ctx->device);
  sdg_status st = enqueue_solve(ctx, dev_Tstar, dev_Tout, ctx->dt, ctx->stream);
  if (st == SDG_OK) g_err.clear();
  return st;
}

sdg_status sdg_step(sdg_ctx* ctx, int n_steps) {
  sdg_status st = check_explicit(ctx, "sdg_step");
  if (st != SDG_OK) return st;
  if (!ctx->kappa) return fail(SDG_E_STATE, "sdg_step needs sdg_set_diffusivity");
  if (!ctx->state) return fail(SDG_E_STATE, "sdg_step needs sdg_set_fields");
  if (n_steps < 0) return fail(SDG_E_ARG, "n_steps must be >= 0");
  DeviceGuard g(ctx->device);
  void* X = ctx->state;
  for (int n = 0; n < n_steps; ++n)
    if ((st = enqueue_step(ctx, ctx->stream)) != SDG_OK) return st;
  if (ctx->check_finite && n_steps > 0) {
    hipError_t e = launch_finite_check(ctx->dm, X, ctx->plan.F, ctx->plan.fp32, ctx->flag, ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "finite check launch");
    int32_t h = 0;
    e = hipMemcpyAsync(&h, ctx->flag, sizeof h, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "finite check");
    if (h) return fail(SDG_E_NUMERIC, "non-finite values in the state after %d steps", n_steps);
  }
  g_err.clear();
  return SDG_OK;
}

sdg_status sdg_step_keep_half(sdg_ctx* ctx, void* dev_x_half) {
  sdg_status st = check_explicit(ctx, "sdg_step_keep_half");
  if (st != SDG_OK) return st;
  if (ctx->scheme != SDG_SCHEME_SPLIT_IMEX)
    return fail(SDG_E_UNSUPPORTED, "sdg_step_keep_half: the context's time scheme is not split-IMEX");
  if (!ctx->kappa) return fail(SDG_E_STATE, "sdg_step_keep_half needs sdg_set_diffusivity");
  if (!ctx->state) return fail(SDG_E_STATE, "sdg_step_keep_half needs sdg_set_fields");
  if (!dev_x_half) return fail(SDG_E_ARG, "sdg_step_keep_half: NULL buffer");
  if (dev_x_half == ctx->state || dev_x_half == ctx->stage_a || dev_x_half == ctx->stage_b)
    return fail(SDG_E_ARG, "sdg_step_keep_half: x_half must not be the state or a workspace stage buffer");
  DeviceGuard g(ctx->device);
  if ((st = enqueue_imex_step(ctx, ctx->stream, dev_x_half)) != SDG_OK) return st;
  g_err.clear();
  return SDG_OK;
}

sdg_status sdg_mass(sdg_ctx* ctx, const void* dev_T, double* host_mass) {
  if (!ctx || !dev_T || !host_mass) return fail(SDG_E_ARG, "sdg_mass: NULL argument");
  if (!ctx->have_mesh) return fail(SDG_E_STATE, "sdg_mass needs an uploaded mesh");
  DeviceGuard g(ctx->device);
  const Plan& P = ctx->plan;
  hipError_t e = launch_column_mass(ctx->dm, dev_T, P.F, P.fp32, ctx->colmass, ctx->stream);
  if (e != hipSuccess) return hip_fail(e, "column mass launch");
  e = launch_member_sum(ctx->colmass, P.CS, P.F, ctx->member_off_dev, P.n_members, ctx->msum, ctx->stream);
  if (e != hipSuccess) return hip_fail(e, "member sum launch");
  e = hipMemcpyAsync(host_mass, ctx->msum, sizeof(double) * P.F * P.n_members, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(e, "sdg_mass");
  g_err.clear();
  return SDG_OK;
}

sdg_status sdg_mass_noalloc(sdg_ctx* ctx, const void* dev_T, double* host_mass) {
  if (!ctx || !dev_T || !host_mass) return fail(SDG_E_ARG, "sdg_mass_noalloc: NULL argument");
  if (!ctx->have_mesh) return fail(SDG_E_STATE, "sdg_mass_noalloc needs an uploaded mesh");
  const Plan& P = ctx->plan;
  // per-column partials [F][n_col_slots], then the member sums [n_members][F];
  // every entry is written before it is read, so nothing needs clearing
  const size_t n_part = (size_t)P.F * (size_t)P.CS;
  const size_t need = n_part + (size_t)P.F * (size_t)P.n_members;
  if (need > kNoAllocDoubles)
    return fail(SDG_E_WORKSPACE,
                "sdg_mass_noalloc: this mesh needs %zu doubles of static scratch (n_fields x (column slots + "
                "members)), more than its %zu; use sdg_mass",
                need, kNoAllocDoubles);
  double* base = static_scratch(ctx->device);
  if (!base) return fail(SDG_E_STATE, "sdg_mass_noalloc: no static scratch bound on device %d", ctx->device);
  DeviceGuard g(ctx->device);
  hipError_t e = launch_column_mass(ctx->dm, dev_T, P.F, P.fp32, base, ctx->stream);
  if (e != hipSuccess) return hip_fail(e, "column mass launch");
  e = launch_member_sum(base, P.CS, P.F, ctx->member_off_dev, P.n_members, base + n_part, ctx->stream);
  if (e != hipSuccess) return hip_fail(e, "member sum launch");
  e = hipMemcpyAsync(host_mass, base + n_part, sizeof(double) * P.F * P.n_members, hipMemcpyDeviceToHost,
                     ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(e, "sdg_mass_noalloc");
  g_err.clear();
  return SDG_OK;
}

namespace {
// Walk segments of a cell of D layers for the bucket setting L: L > 0 fixed
// segments of L layers (the last one shorter), L < 0 the same number of
// segments, ceil(D / |L|), of balanced lengths (the longer ones first).
void bucket_segments(int D, int L, std::vector<std::pair<int, int>>& seg) {
  seg.clear();
  const int A = L < 0 ? -L : L;
  const int n = (D + A - 1) / A;
  if (L > 0) {
    for (int l0 = 0; l0 < D; l0 += A) seg.push_back({l0, std::min(A, D - l0)});
  } else {
    const int q = D / n, r = D % n;
    for (int i = 0, l0 = 0; i < n; ++i) {
      const int len = q + (i < r ? 1 : 0);
      seg.push_back({l0, len});
      l0 += len;
    }
  }
}

bool valid_walk_setting(int L) {
  const int A = L < 0 ? -L : L;
  return A >= kWalkMinLayers && A <= kBucketWalkMax;
}

// Build the per-bucket walk table for walk_layers (only the cells of bucket
// `only`, if only >= 0) and upload it; the table lists longer tiles first,
// each length in cell order.  Synchronises the stream.
sdg_status upload_bucket_table(sdg_ctx* ctx, const int* walk_layers, int only) {
  const Plan& P = ctx->plan;
  std::vector<WgTile> t;
  t.reserve(P.n_tiles[3]);
  std::vector<std::pair<int, int>> seg;
  for (int k = 0; k < P.n_cells; ++k) {
    const int D = P.cell_depth[k];
    if (D == 0) continue;
    const int b = depth_bucket(D);
    if (only >= 0 && b != only) continue;
    bucket_segments(D, walk_layers[b], seg);
    for (auto& sg : seg) t.push_back({k, (uint16_t)sg.first, (uint16_t)sg.second});
  }
  if ((int)t.size() > std::max(P.n_tiles[3], 1)) return fail(SDG_E_ARG, "per-bucket walk table too large");
  std::stable_sort(t.begin(), t.end(), [](const WgTile& x, const WgTile& y) { return x.nlay > y.nlay; });
  if (!t.empty()) {
    hipError_t e = hipMemcpyAsync(ctx->tiles_bucket, t.data(), sizeof(WgTile) * t.size(), hipMemcpyHostToDevice,
                                  ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "per-bucket walk table upload");
  }
  ctx->n_tiles_bucket = (int)t.size();
  return SDG_OK;
}
}  // namespace

sdg_status sdg_get_tuning(sdg_ctx* ctx, sdg_tuning* out) {
  if (!ctx || !out) return fail(SDG_E_ARG, "sdg_get_tuning: NULL argument");
  const bool bucket = ctx->tile_choice == kBucketChoice;
  out->tile_layers = bucket ? 0 : kTileLayerOptions[ctx->tile_choice];
  out->xcd_remap = ctx->xcd;
  out->persistent = ctx->persistent;
  for (int b = 0; b < kDepthBuckets; ++b) out->walk_layers[b] = bucket ? ctx->walk_layers[b] : 0;
  g_err.clear();
  return SDG_OK;
}

sdg_status sdg_set_tuning(sdg_ctx* ctx, const sdg_tuning* t) {
  if (!ctx || !t) return fail(SDG_E_ARG, "sdg_set_tuning: NULL argument");
  int choice = -1;
  for (int i = 0; i < kTileChoices; ++i)
    if (kTileLayerOptions[i] == t->tile_layers) choice = i;
  if (t->tile_layers == 0) choice = kBucketChoice;
  if (choice < 0)
    return fail(SDG_E_ARG, "tile_layers must be 0 (per depth bucket), 1, 2, 4, 8, 12, 16 or 32 (got %d)",
                t->tile_layers);
  if (t->xcd_remap != 0 && t->xcd_remap != 1) return fail(SDG_E_ARG, "xcd_remap must be 0 or 1");
  if (t->persistent != 0 && t->persistent != 1) return fail(SDG_E_ARG, "persistent must be 0 or 1");
  if (choice == kBucketChoice) {
    if (!ctx->have_mesh) return fail(SDG_E_STATE, "per-bucket walks need an uploaded mesh");
    for (int b = 0; b < kDepthBuckets; ++b)
      if (!valid_walk_setting(t->walk_layers[b]))
        return fail(SDG_E_ARG, "walk_layers[%d] = %d: need 8..64 (fixed) or -64..-8 (balanced)", b,
                    t->walk_layers[b]);
    DeviceGuard g(ctx->device);
    sdg_status st = upload_bucket_table(ctx, t->walk_layers, -1);
    if (st != SDG_OK) return st;
    for (int b = 0; b < kDepthBuckets; ++b) ctx->walk_layers[b] = t->walk_layers[b];
  }
  ctx->tile_choice = choice;
  ctx->xcd = t->xcd_remap;
  ctx->persistent = t->persistent;
  ctx->graph_valid = false;
  g_err.clear();
  return SDG_OK;
}

namespace {
sdg_status timed_stages(sdg_ctx* ctx) {
  sdg_status st = enqueue_stage(ctx, 0, nullptr, ctx->state, ctx->stage_a, ctx->stream);
  if (st == SDG_OK) st = enqueue_stage(ctx, 1, ctx->state, ctx->stage_a, ctx->stage_b, ctx->stream);
  if (st == SDG_OK) st = enqueue_stage(ctx, 2, ctx->state, ctx->stage_b, ctx->stage_a, ctx->stream);
  return st;
}
}  // namespace

sdg_status sdg_autotune(sdg_ctx* ctx, int reps, sdg_tuning* chosen) {
  sdg_status st = check_explicit(ctx, "sdg_autotune");
  if (st != SDG_OK) return st;
  if (!ctx->state) return fail(SDG_E_STATE, "sdg_autotune needs sdg_set_fields");
  if (reps < 1) reps = 1;
  DeviceGuard g(ctx->device);
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) return hip_fail(e, "sdg_autotune: hipEventCreate");
  // mean time of the three stages of a step in the current shape, with
  // sdg_step's buffer pattern (Tn = the fields, stage inputs and outputs in
  // the two workspace buffers), so the set fields are only read
  auto time_shape = [&](float* ms) -> sdg_status {
    sdg_status s2 = timed_stages(ctx);
    if (s2 != SDG_OK) return s2;
    hipError_t e2 = hipEventRecord(e0, ctx->stream);
    for (int r = 0; r < reps && s2 == SDG_OK; ++r) s2 = timed_stages(ctx);
    if (s2 != SDG_OK) return s2;
    if (e2 == hipSuccess) e2 = hipEventRecord(e1, ctx->stream);
    if (e2 == hipSuccess) e2 = hipEventSynchronize(e1);
    if (e2 == hipSuccess) e2 = hipEventElapsedTime(ms, e0, e1);
    return e2 == hipSuccess ? SDG_OK : hip_fail(e2, "sdg_autotune: timing");
  };
  float best = 1e30f;
  int best_choice = ctx->tile_choice == kBucketChoice ? 1 : ctx->tile_choice;
  int best_xcd = ctx->xcd, best_pers = ctx->persistent;
  for (int shape = 0; shape < kTileChoices * 4 && st == SDG_OK; ++shape) {
    const int c = shape >> 2, x = shape & 1, pers = (shape >> 1) & 1;
    ctx->tile_choice = c;
    ctx->xcd = x;
    ctx->persistent = pers;
    float ms = 0.f;
    st = time_shape(&ms);
    if (st == SDG_OK && ms < best) {
      best = ms;
      best_choice = c;
      best_xcd = x;
      best_pers = pers;
    }
  }
  // With a column walk fastest, choose each depth bucket's segmentation
  // (fixed or balanced lengths) by timing that bucket's tiles alone, one
  // bucket at a time, then keep the per-bucket table if the whole of it
  // beats the uniform walk.
  int wl[kDepthBuckets];
  bool use_buckets = false;
  if (st == SDG_OK && best_choice >= kThreadTileChoices) {
    static constexpr int kOpts[] = {8, 12, 16, 32, 64, -8, -12, -16, -24, -32};
    const Plan& P = ctx->plan;
    int present[kDepthBuckets] = {};
    for (int k = 0; k < P.n_cells; ++k)
      if (P.cell_depth[k] > 0) present[depth_bucket(P.cell_depth[k])] = 1;
    for (int b = 0; b < kDepthBuckets; ++b) wl[b] = kTileLayerOptions[best_choice];
    ctx->tile_choice = kBucketChoice;
    ctx->xcd = best_xcd;
    ctx->persistent = best_pers;
    for (int b = 0; b < kDepthBuckets && st == SDG_OK; ++b) {
      if (!present[b]) continue;
      float bb = 1e30f;
      int bo = wl[b];
      for (int o : kOpts) {
        wl[b] = o;
        st = upload_bucket_table(ctx, wl, b);
        float ms = 0.f;
        if (st == SDG_OK) st = time_shape(&ms);
        if (st != SDG_OK) break;
        if (ms < bb) {
          bb = ms;
          bo = o;
        }
      }
      wl[b] = bo;
    }
    float ms = 1e30f;
    if (st == SDG_OK) st = upload_bucket_table(ctx, wl, -1);
    if (st == SDG_OK) st = time_shape(&ms);
    use_buckets = st == SDG_OK && ms < best;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ctx->tile_choice = use_buckets ? kBucketChoice : best_choice;
  ctx->xcd = best_xcd;
  ctx->persistent = best_pers;
  if (use_buckets)
    for (int b = 0; b < kDepthBuckets; ++b) ctx->walk_layers[b] = wl[b];
  ctx->graph_valid = false;
  if (st != SDG_OK) return st;
  if (chosen) {
    sdg_status s2 = sdg_get_tuning(ctx, chosen);
    if (s2 != SDG_OK) return s2;
  }
  g_err.clear();
  return SDG_OK;
}

sdg_status sdg_graph_capture_step(sdg_ctx* ctx) {
  sdg_status st = check_explicit(ctx, "sdg_graph_capture_step");
  if (st != SDG_OK) return st;
  if (!ctx->kappa) return fail(SDG_E_STATE, "sdg_graph_capture_step needs sdg_set_diffusivity");
  if (!ctx->state) return fail(SDG_E_STATE, "sdg_graph_capture_step needs sdg_set_fields");
  DeviceGuard g(ctx->device);
  drop_graph(ctx);
  hipError_t e = hipSuccess;
  if (!ctx->cap_stream) e = hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "sdg_graph_capture_step: stream");
  // the factors are computed outside the graph (sdg_graph_launch keeps
  // them current); the captured kernels must not overtake work already
  // queued on the context stream: capture starts after it has drained
  st = ensure_factors(ctx, step_solve_dt(ctx), ctx->stream);
  if (st != SDG_OK) return st;
  e = hipStreamSynchronize(ctx->stream);
  if (e == hipSuccess) e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "sdg_graph_capture_step: begin capture");
  st = enqueue_step(ctx, ctx->cap_stream);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(ctx->cap_stream, &graph);
  if (st != SDG_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "sdg_graph_capture_step: end capture");
  ctx->graph = graph;
  e = hipGraphInstantiate(&ctx->graph_exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    drop_graph(ctx);
    return hip_fail(e, "sdg_graph_capture_step: instantiate");
  }
  ctx->graph_valid = true;
  g_err.clear();
  return SDG_OK;
}

sdg_status sdg_graph_launch(sdg_ctx* ctx, int n_steps) {
  if (!ctx) return fail(SDG_E_ARG, "context is NULL");
  if (!ctx->graph_valid) return fail(SDG_E_STATE, "no valid captured step (capture again after any set_* call)");
  if (n_steps < 0) return fail(SDG_E_ARG, "n_steps must be >= 0");
  DeviceGuard g(ctx->device);
  if (n_steps > 0) {
    sdg_status st = ensure_factors(ctx, step_solve_dt(ctx), ctx->stream);
    if (st != SDG_OK) return st;
  }
  for (int n = 0; n < n_steps; ++n) {
    hipError_t e = hipGraphLaunch(ctx->graph_exec, ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  }
  g_err.clear();
  return SDG_OK;
}

sdg_status sdg_apply_mass(sdg_ctx* ctx, const void* dev_X, void* dev_Y, int inverse) {
  if (!ctx || !dev_X || !dev_Y) return fail(SDG_E_ARG, "sdg_apply_mass: NULL argument");
  if (!ctx->have_mesh) return fail(SDG_E_STATE, "sdg_apply_mass needs an uploaded mesh");
  DeviceGuard g(ctx->device);
  hipError_t e = launch_mass_apply(ctx->dm, dev_X, dev_Y, ctx->plan.F, ctx->plan.fp32, inverse != 0, ctx->stream);
  if (e != hipSuccess) return hip_fail(e, "mass apply launch");
  g_err.clear();
  return SDG_OK;
}

sdg_status sdg_m_dot(sdg_ctx* ctx, const void* dev_X, const void* dev_Y, double* host_out) {
  if (!ctx || !dev_X || !dev_Y || !host_out) return fail(SDG_E_ARG, "sdg_m_dot: NULL argument");
  if (!ctx->have_mesh) return fail(SDG_E_STATE, "sdg_m_dot needs an uploaded mesh");
  DeviceGuard g(ctx->device);
  const Plan& P = ctx->plan;
  hipError_t e = launch_mdot_columns(ctx->dm, dev_X, dev_Y, P.F, P.fp32, ctx->colmass, ctx->stream);
  if (e != hipSuccess) return hip_fail(e, "m_dot launch");
  e = launch_member_sum(ctx->colmass, P.CS, P.F, ctx->member_off_dev, P.n_members, ctx->msum, ctx->stream);
  if (e != hipSuccess) return hip_fail(e, "m_dot reduction launch");
  e = hipMemcpyAsync(host_out, ctx->msum, sizeof(double) * P.F * P.n_members, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(e, "sdg_m_dot");
  g_err.clear();
  return SDG_OK;
}

sdg_status sdg_step_adjoint(sdg_ctx* ctx, const void* dev_z_next, void* dev_z_out, const void* dev_x_next,
                            double* dev_dkappa) {
  sdg_status st = check_explicit(ctx, "sdg_step_adjoint");
  if (st != SDG_OK) return st;
  if (ctx->plan.fp32) return fail(SDG_E_UNSUPPORTED, "sdg_step_adjoint needs an FP64 context");
  if (ctx->scheme != SDG_SCHEME_SSPRK3_LIE)
    return fail(SDG_E_UNSUPPORTED, "sdg_step_adjoint reverses the SSP-RK3 + Lie step only");
  if (!ctx->kappa) return fail(SDG_E_STATE, "sdg_step_adjoint needs sdg_set_diffusivity");
  if (!dev_z_next || !dev_z_out) return fail(SDG_E_ARG, "sdg_step_adjoint: NULL buffer");
  if (dev_dkappa && !dev_x_next) return fail(SDG_E_ARG, "sdg_step_adjoint: dkappa needs x_next");
  if (dev_dkappa && dev_x_next == dev_z_out)
    return fail(SDG_E_ARG, "sdg_step_adjoint: x_next must not be z_out (the solve overwrites z_out before x_next is read)");
  if (dev_z_out == ctx->stage_a || dev_z_out == ctx->stage_b || dev_z_next == ctx->stage_a || dev_z_next == ctx->stage_b)
    return fail(SDG_E_ARG, "sdg_step_adjoint: buffers must not be the workspace stage buffers");
  DeviceGuard g(ctx->device);
  const Plan& P = ctx->plan;
  double* mu = static_cast<double*>(dev_z_out);
  double* zb2 = static_cast<double*>(ctx->stage_a);
  double* zb1 = static_cast<double*>(ctx->stage_b);
  const double* U = static_cast<const double*>(ctx->U);
  // the adjoint stages run one thread per prism: a walk shape maps to 2-layer
  // tiles with the XCD remap (at the 998,560-prism adjoint workload 0.52 ms
  // per reverse step against 0.65 ms without the remap)
  const bool walk = ctx->tile_choice >= kThreadTileChoices;
  const int choice = walk ? 1 : ctx->tile_choice;
  const int xcd = walk ? 1 : ctx->xcd;
  const int tl = kTileLayerOptions[choice];
  const WgTile* tiles = ctx->tiles[choice];
  const int nt = P.n_tiles[choice];
  hipStream_t s = ctx->stream;
  sdg_status fst = ensure_tfactors(ctx, ctx->dt, s);
  if (fst != SDG_OK) return fst;
  hipError_t e = launch_tsolve(ctx->dm, P.F, static_cast<const double*>(dev_z_next), mu, ctx->kappa,
                               ctx->tfac, ctx->dt, ctx->eta, false, s);
  if (e != hipSuccess) return hip_fail(e, "transposed solve launch");
  if (dev_dkappa) {
    e = launch_kappa_gradient(ctx->dm, ctx->tiles[1], P.n_tiles[1], P.F, mu, static_cast<const double*>(dev_x_next),
                              ctx->kpart, ctx->eta,
                              ctx->dt, dev_dkappa, s);
    if (e != hipSuccess) return hip_fail(e, "kappa gradient launch");
  }
  const bool wz = ctx->w_zero;
  // the horizontal diffusion D is symmetric, so its part of M^-1 (R_lin + D)^T
  // is M^-1 D, added to each stage as in the forward step
  const double dt = ctx->dt;
  e = launch_adjoint_stage(ctx->dm, tiles, nt, tl, xcd, P.F, wz, mu, nullptr, nullptr, zb2, U, dt,
                           2.0 / 3.0, 0.0, 0.0, s);
  if (e == hipSuccess) e = enqueue_hdiff(ctx, mu, zb2, nullptr, 2.0 / 3.0 * dt, 0.0, s);
  if (e == hipSuccess)
    e = launch_adjoint_stage(ctx->dm, tiles, nt, tl, xcd, P.F, wz, zb2, nullptr, nullptr, zb1, U, dt,
                             0.25, 0.0, 0.0, s);
  if (e == hipSuccess) e = enqueue_hdiff(ctx, zb2, zb1, nullptr, 0.25 * dt, 0.0, s);
  if (e == hipSuccess)
    e = launch_adjoint_stage(ctx->dm, tiles, nt, tl, xcd, P.F, wz, zb1, mu, zb2, mu, U, dt, 1.0,
                             1.0 / 3.0, 0.75, s);
  if (e == hipSuccess) e = enqueue_hdiff(ctx, zb1, mu, nullptr, dt, 0.0, s);
  if (e != hipSuccess) return hip_fail(e, "adjoint stage launch");
  g_err.clear();
  return SDG_OK;
}

namespace {
// The reverse split-IMEX step; x is the state before the forward step
// (half = false: x_h is rebuilt from it when dkappa is asked for) or that
// step's x_h (half = true).
sdg_status adjoint_imex(sdg_ctx* ctx, const char* who, const void* dev_z_next, void* dev_z_out, const void* dev_x,
                        bool half, double* dev_dkappa) {
  sdg_status st = check_explicit(ctx, who);
  if (st != SDG_OK) return st;
  if (ctx->plan.fp32) return fail(SDG_E_UNSUPPORTED, "%s needs an FP64 context", who);
  if (ctx->scheme != SDG_SCHEME_SPLIT_IMEX) return fail(SDG_E_UNSUPPORTED, "%s reverses the split-IMEX step only", who);
  if (!ctx->kappa) return fail(SDG_E_STATE, "%s needs sdg_set_diffusivity", who);
  if (!dev_z_next || !dev_z_out) return fail(SDG_E_ARG, "%s: NULL buffer", who);
  if (dev_z_out == dev_z_next || dev_z_out == dev_x)
    return fail(SDG_E_ARG, "%s: z_out must not alias z_next or the forward state", who);
  if (dev_dkappa && !dev_x) return fail(SDG_E_ARG, "%s: dkappa needs the forward state", who);
  void* A = ctx->stage_a;
  void* B = ctx->stage_b;
  if (dev_z_out == A || dev_z_out == B || dev_z_next == A || dev_z_next == B || dev_x == A || dev_x == B)
    return fail(SDG_E_ARG, "%s: buffers must not be the workspace stage buffers", who);
  DeviceGuard g(ctx->device);
  const Plan& P = ctx->plan;
  hipStream_t s = ctx->stream;
  const double h = 0.5 * ctx->dt;
  const bool walk = ctx->tile_choice >= kThreadTileChoices;   // as in sdg_step_adjoint
  const int choice = walk ? 1 : ctx->tile_choice;
  const int xcd = walk ? 1 : ctx->xcd;
  const int tl = kTileLayerOptions[choice];
  const WgTile* tiles = ctx->tiles[choice];
  const int nt = P.n_tiles[choice];
  const bool wz = ctx->w_zero;
  const double* U = static_cast<const double*>(ctx->U);
  const double* Z1 = static_cast<const double*>(dev_z_next);
  double* out = static_cast<double*>(dev_z_out);
  double* mu = static_cast<double*>(A);
  double* w = static_cast<double*>(B);
  hipError_t e = hipSuccess;
  const double* xh = half ? static_cast<const double*>(dev_x) : out;
  if (dev_dkappa && !half) {
    // x_h of the step being reversed, kept in z_out until the last stage:
    // the half step from x_prev, then its column solve in place
    StageArgs s1 = stage_args(ctx, nullptr, dev_x, dev_z_out, 0.0, 1.0, h);
    e = launch_stage(s1, false, wz, false, false, s);
    if (e == hipSuccess) e = hdiff_after_stage(ctx, s1, h, 0.0, s);
    if (e != hipSuccess) return hip_fail(e, "split-IMEX adjoint half step launch");
    if ((st = enqueue_solve(ctx, dev_z_out, dev_z_out, h, s)) != SDG_OK) return st;
  }
  // w = 2 (Z1 + h L~ Z1)
  e = launch_adjoint_stage(ctx->dm, tiles, nt, tl, xcd, P.F, wz, Z1, nullptr, nullptr, w, U, h, 2.0, 0.0,
                           0.0, s);
  if (e == hipSuccess) e = enqueue_hdiff(ctx, Z1, w, nullptr, 2.0 * h, 0.0, s);
  // mu' = (M - h A^T)^-1 M w;  dJ/dkappa_l += h mu'^T A_l x_h
  if (e == hipSuccess) {
    sdg_status fst = ensure_tfactors(ctx, h, s);
    if (fst != SDG_OK) return fst;
    e = launch_tsolve(ctx->dm, P.F, w, mu, ctx->kappa, ctx->tfac, h, ctx->eta, false, s);
  }
  if (e == hipSuccess && dev_dkappa)
    e = launch_kappa_gradient(ctx->dm, ctx->tiles[1], P.n_tiles[1], P.F, mu, xh, ctx->kpart, ctx->eta, h,
                              dev_dkappa, s);
  // Z0 = mu' + h L~ mu' + Z1 - w
  if (e == hipSuccess)
    e = launch_adjoint_stage(ctx->dm, tiles, nt, tl, xcd, P.F, wz, mu, Z1, w, out, U, h, 1.0, 1.0, -1.0, s);
  if (e == hipSuccess) e = enqueue_hdiff(ctx, mu, out, nullptr, h, 0.0, s);
  if (e != hipSuccess) return hip_fail(e, "split-IMEX adjoint launch");
  g_err.clear();
  return SDG_OK;
}
}  // namespace

sdg_status sdg_step_adjoint_imex(sdg_ctx* ctx, const void* dev_z_next, void* dev_z_out, const void* dev_x_prev,
                                 double* dev_dkappa) {
  return adjoint_imex(ctx, "sdg_step_adjoint_imex", dev_z_next, dev_z_out, dev_x_prev, false, dev_dkappa);
}

sdg_status sdg_step_adjoint_imex_half(sdg_ctx* ctx, const void* dev_z_next, void* dev_z_out, const void* dev_x_half,
                                      double* dev_dkappa) {
  return adjoint_imex(ctx, "sdg_step_adjoint_imex_half", dev_z_next, dev_z_out, dev_x_half, true, dev_dkappa);
}

sdg_status sdg_column_dv_solve(sdg_ctx* ctx, int kind, int n_comp, const void* dev_F, void* dev_x) {
  if (!ctx || !dev_F || !dev_x) return fail(SDG_E_ARG, "sdg_column_dv_solve: NULL argument");
  if (!ctx->have_mesh) return fail(SDG_E_STATE, "sdg_column_dv_solve needs an uploaded mesh");
  if (kind != SDG_DV_VU && kind != SDG_DV_VD)
    return fail(SDG_E_ARG, "sdg_column_dv_solve: unknown kind %d", kind);
  if (n_comp < 1 || n_comp > SDG_DV_MAX_COMP)
    return fail(SDG_E_ARG, "sdg_column_dv_solve: n_comp must be in 1..%d (got %d)", SDG_DV_MAX_COMP, n_comp);
  DeviceGuard g(ctx->device);
  const Plan& P = ctx->plan;
  hipError_t e = launch_column_dv(ctx->dm, kind == SDG_DV_VU, n_comp, dev_F, dev_x, P.fp32,
                                  P.prec == SDG_FP32, ctx->stream);
  if (e != hipSuccess) return hip_fail(e, "column D_v solve launch");
  g_err.clear();
  return SDG_OK;
}

sdg_status sdg_sync(sdg_ctx* ctx) {
  if (!ctx) return fail(SDG_E_ARG, "context is NULL");
  DeviceGuard g(ctx->device);
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "sdg_sync");
  g_err.clear();
  return SDG_OK;
}

}  // extern "C"
