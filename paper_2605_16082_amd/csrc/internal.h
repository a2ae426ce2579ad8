// Internal definitions shared by the host code and the kernels of libslimdg.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace sdg {

constexpr int kCell = 64;           // columns per cell = wavefront width
constexpr int kMaxFields = 4;

// Per-column geometry rows in DevMesh::geo ([kGeoRows][n_col_slots]).
enum GeoRow : int {
  G_XXI = 0,  // x1 - x0
  G_XET = 1,  // x2 - x0
  G_YXI = 2,  // y1 - y0
  G_YET = 3,  // y2 - y0
  G_JH = 4,   // (x1-x0)(y2-y0) - (x2-x0)(y1-y0) = 2 * area
  G_NX = 5,   // 5,6,7: outward unit normal x of edge k
  G_NY = 8,   // 8,9,10
  G_LE = 11,  // 11,12,13: edge length
  kGeoRows = 14
};

// Device view of an uploaded mesh.  Column slot = cell * 64 + lane; prism
// slot = cell_base[cell] + layer * 64 + lane; level slot = cell_lbase[cell]
// + level * 64 + lane.
struct DevMesh {
  int32_t n_cols;          // live columns
  int32_t n_cells;
  int32_t n_col_slots;     // n_cells * 64
  int32_t max_layers;
  int64_t n_slots;         // prism slots
  int64_t n_lslots;        // level slots
  const int32_t* cell_base;    // [n_cells + 1]
  const int32_t* cell_lbase;   // [n_cells + 1]
  const int32_t* nlay;         // [n_col_slots], 0 on padding columns
  const int32_t* nbr_slot;     // [3][n_col_slots]: prism slot of the neighbour's layer 0, or -1
  const int32_t* nbr_meta;     // [3][n_col_slots]: (neighbour nlayers << 2) | neighbour edge
  const int32_t* nbr_col;      // [3][n_col_slots]: neighbour column slot, or -1
  const double* geo;           // [kGeoRows][n_col_slots]
  const float* geo32;          // same, float
  const double* zl;            // [3][n_lslots] level heights
  const float* zl32;           // same, float
  const double* xy;            // [6][n_col_slots] x0,y0,x1,y1,x2,y2 (input of the geometry kernel)
  const int32_t* col_member;   // [n_col_slots] member id (-1 on padding)
  // lateral faces whose neighbour is in another cell, listed per cell
  // (column by column, faces in order): the list of cell k is
  // halo_off[k] .. halo_off[k + 1] - 1, with the neighbour's layer-0 slot and
  // depth; halo_idx[e][c] is face e of column c's place in its cell's list,
  // or -1.  halo_max: the longest list.
  int32_t halo_max;
  const int32_t* halo_off;     // [n_cells + 1]
  const int32_t* halo_slot;
  const int32_t* halo_depth;
  const int32_t* halo_idx;     // [3][n_col_slots]
  // the cells deepest first: the column solves take their cells in this
  // order, so the longest columns do not end the launch alone
  const int32_t* cell_order;   // [n_cells]
};

// A workgroup of the per-prism kernels covers tile_layers consecutive layers
// of one cell: (cell, first layer).  Tile heights from kWalkMinLayers up are
// walked by one wavefront (the column-walk form of the stage kernel); the
// smaller ones run one thread per prism.
// nlay: layers of the tile (the walk covers layer0 .. layer0 + nlay - 1);
// tile tables of one height list min(height, depth - layer0).
struct WgTile {
  int32_t cell;
  uint16_t layer0;
  uint16_t nlay;
};
constexpr int kTileChoices = 7;
constexpr int kTileLayerOptions[kTileChoices] = {1, 2, 4, 8, 12, 16, 32};
constexpr int kWalkMinLayers = 8;
constexpr int kThreadTileChoices = 3;           // choices 0..2 run one thread per prism
// The per-depth-bucket walk table (tile_layers 0 in sdg_tuning): every tile
// is a walk of its own length, at most kBucketWalkMax layers.
constexpr int kBucketChoice = kTileChoices;     // tile_choice of that table
constexpr int kBucketWalkMax = 64;
constexpr int kDepthBuckets = 6;
// depth bucket of a cell of D layers: 1-8, 9-16, 17-24, 25-32, 33-48, > 48
inline int depth_bucket(int D) {
  return D <= 8 ? 0 : D <= 16 ? 1 : D <= 24 ? 2 : D <= 32 ? 3 : D <= 48 ? 4 : 5;
}

struct StageArgs {
  DevMesh m;
  const WgTile* tiles;   // one entry per workgroup: (cell, first layer)
  int32_t n_tiles;
  int32_t tile_layers;   // layers per tile: 1, 2, 4 (blockDim 64 * tile_layers), or >= 8: walks of
                         // each tile's own length (kBucketWalkMax for the per-bucket table)
  int32_t xcd;           // 1: XCD-contiguous tile order
  int32_t persistent;    // 1: grid of resident workgroups walking the tiles
  int32_t n_cu;          // compute units of the device (persistent grid size)
  int32_t n_fields;
  const void* Tn;      // [F][6][n_slots]
  const void* Ts;
  void* Tout;
  void* Tout2;         // optional second output Ts - 2 Tout (stage without Tn only)
  const void* U;       // [3][6][n_slots]
  double t_ext[kMaxFields];
  double dt;
  double a, b;         // Tout = a Tn + b (Ts + dt L)
};

struct SolveArgs {
  DevMesh m;
  int32_t n_fields;
  const void* Tstar;
  void* Tout;
  const double* kappa;   // [max_layers]
  double* scratch;       // [18 + 6F][n_slots] values of the solve's arithmetic type:
                         // the kept E_l (18), then y_l (6F)
  double dt;
  double eta;
};

// Horizontal diffusion: Tout += c1 M^-1 D(Ts) (and Tout2 += c2 M^-1 D(Ts)).
struct HdiffArgs {
  DevMesh m;
  const WgTile* tiles;   // the 2-layer tile table
  int32_t n_tiles;
  int32_t tile_layers;   // 2
  int32_t n_fields;
  const void* Ts;
  void* Tout;
  void* Tout2;           // optional
  double c1, c2;
  const double* kh;      // [n_col_slots] horizontal diffusivity per column
  const double* hface;   // [3 faces][5][n_col_slots]: neighbour kh, penalty, n . grad of its basis
};

// Kernel launchers (defined next to their kernels).
hipError_t launch_hdiff(const HdiffArgs& a, bool fp32, hipStream_t s);
// kh[c] = coef * sqrt(J_h)^1.15 for every live column.
// kh per column (coef sqrt(J_h)^1.15) and the per-face neighbour table of the
// horizontal diffusion (penalty factor eta)
hipError_t launch_hdiff_setup(const DevMesh& m, double coef, double eta, double* kh, double* hface,
                              hipStream_t s);
hipError_t launch_geometry(const DevMesh& m, double* geo, float* geo32, hipStream_t s);
hipError_t launch_z32(const DevMesh& m, float* zl32, hipStream_t s);
hipError_t launch_stage(const StageArgs& a, bool fp32, bool w_zero, bool rhs_only,
                        bool read_tn, hipStream_t s);
// factor = true: compute and keep the block-Thomas factors E_l for (kappa, dt,
// eta) in a.scratch (the fields are not read); false: solve with kept factors.
hipError_t launch_vsolve(const SolveArgs& a, bool fp32_state, bool fp32_solve, bool factor, hipStream_t s);
// Matrix-free D_vu (down = true) / D_vd column solves; fp32_arith only with fp32_state.
hipError_t launch_column_dv(const DevMesh& m, bool down, int n_comp, const void* F, void* X, bool fp32_state,
                            bool fp32_arith, hipStream_t s);
hipError_t launch_column_mass(const DevMesh& m, const void* T, int n_fields, bool fp32,
                              double* col_mass, hipStream_t s);
hipError_t launch_member_sum(const double* col_mass, int n_col_slots, int n_fields,
                             const int32_t* member_off, int n_members, double* out,
                             hipStream_t s);
hipError_t launch_finite_check(const DevMesh& m, const void* T, int n_fields, bool fp32,
                               int32_t* flag, hipStream_t s);

// Adjoint (FP64 only).
hipError_t launch_adjoint_stage(const DevMesh& m, const WgTile* tiles, int n_tiles, int tile_layers, int xcd,
                                int n_fields, bool w_zero, const double* Y, const double* X1, const double* X2,
                                double* out, const double* U, double dt, double b, double a1, double a2,
                                hipStream_t s);
// factor = true: compute and keep the transposed block-Thomas factors G_l for
// (kappa, dt, eta) in gfac ([18][n_slots]); false: mu from Z with the kept
// factors (mu may be Z).
hipError_t launch_tsolve(const DevMesh& m, int n_fields, const double* Z, double* mu, const double* kappa,
                         double* gfac, double dt, double eta, bool factor, hipStream_t s);
// dkappa[l] += dt sum mu^T (dA/dkappa_l) x, one thread per prism over the
// 2-layer tile table (tiles2, n_tiles2), per-cell sums in partial.
hipError_t launch_kappa_gradient(const DevMesh& m, const WgTile* tiles2, int n_tiles2, int n_fields,
                                 const double* mu, const double* x, double* partial, double eta, double dt,
                                 double* dkappa, hipStream_t s);
hipError_t launch_mass_apply(const DevMesh& m, const void* X, void* Y, int n_fields, bool fp32, bool inverse,
                             hipStream_t s);
hipError_t launch_mdot_columns(const DevMesh& m, const void* X, const void* Y, int n_fields, bool fp32,
                               double* col_out, hipStream_t s);

// Workgroup index -> tile index so that each of the 8 XCDs (which receive
// workgroups round-robin) processes one contiguous range of tiles, keeping
// lateral neighbours in the same L2.
__device__ __forceinline__ int xcd_tile(int b, int n) {
  const int q = n >> 3, r = n & 7;
  const int x = b & 7, j = b >> 3;
  return (x < r) ? x * (q + 1) + j : r * (q + 1) + (x - r) * q + j;
}

}  // namespace sdg
