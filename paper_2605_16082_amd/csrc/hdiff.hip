// Horizontal tracer diffusion (the paper's section 1.1 split of the
// diffusivity into horizontal and vertical parts, Okubo's model for the
// horizontal diffusivity; section 2: horizontal terms are explicit), taken
// along the layers with a symmetric interior penalty on the lateral faces:
//
//   D_i = - int_K kh grad_z T . grad_z phi_i dV
//         + sum_faces int ( {kh grad_z T}.n phi_i + 1/2 kh (grad_z phi_i . n) [T] - sigma [T] phi_i ) dS
//
// grad_z = derivatives at constant zeta, [T] = T_K - T_neighbour, {.} the
// mean of both sides, sigma = eta (kh + kh')/2 / min(J_h/|e|, J_h'/|e|), zero
// flux at open boundaries and walls, kh = coef * sqrt(J_h)^1.15 per column
// (Okubo's relation in metres, coef from the host).
//
// For linear prisms every integral has a closed form: grad_z T is constant on
// each layer surface and linear in zeta, (1+zeta)/2 g_top + (1-zeta)/2 g_bot
// with g = sum_a grad(lambda_a) T_a of the face's three nodes; the face
// measure is |e| z_zeta(s) ds dzeta with z_zeta linear along the edge.  The
// kernel adds c1 M^-1 D to Tout (and c2 M^-1 D to Tout2), after the stage
// kernel has written them, one thread per prism over tiles of two layers of a
// cell (128 threads): the per-column factors are cheap to rebuild, and the
// many independent prisms keep enough loads in flight.  The tile's stage
// input is staged in LDS first, so neighbours in the same cell (most lateral
// faces of a locality-ordered mesh) are read from there.  A field's current
// output values are loaded before its arithmetic rather than at the update, so
// that their latency overlaps it.  When the parameters are set, kh is computed
// once per column (okubo_kernel) and, per column and lateral face, what the
// face terms need of the neighbour (hface_kernel), so that the kernel's loads
// of per-column data do not wait on the neighbour's index.
#include "internal.h"

namespace sdg {
namespace {

template <typename R> __device__ __forceinline__ const R* geo_rows(const DevMesh& m);
template <> __device__ __forceinline__ const double* geo_rows<double>(const DevMesh& m) { return m.geo; }
template <> __device__ __forceinline__ const float* geo_rows<float>(const DevMesh& m) { return m.geo32; }
template <typename R> __device__ __forceinline__ const R* level_rows(const DevMesh& m);
template <> __device__ __forceinline__ const double* level_rows<double>(const DevMesh& m) { return m.zl; }
template <> __device__ __forceinline__ const float* level_rows<float>(const DevMesh& m) { return m.zl32; }

// Gradients of the three barycentric functions of column c: gl[a] = (d/dx, d/dy).
template <typename R>
__device__ __forceinline__ void lambda_grads(const R* geo, int CS, int c, R gl[3][2], R& Jh) {
  const R xxi = geo[G_XXI * CS + c], xet = geo[G_XET * CS + c];
  const R yxi = geo[G_YXI * CS + c], yet = geo[G_YET * CS + c];
  Jh = geo[G_JH * CS + c];
  const R inv = R(1) / Jh;
  gl[1][0] = yet * inv;
  gl[1][1] = -xet * inv;
  gl[2][0] = -yxi * inv;
  gl[2][1] = xxi * inv;
  gl[0][0] = -(gl[1][0] + gl[2][0]);
  gl[0][1] = -(gl[1][1] + gl[2][1]);
}

// kh[c] = coef sqrt(J_h)^1.15, coef = okubo_scale * (Okubo's constant in metres)
__global__ __launch_bounds__(256) void okubo_kernel(DevMesh m, double coef, double* kh) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m.n_col_slots) return;
  kh[c] = m.nlay[c] > 0 ? coef * pow(m.geo[G_JH * m.n_col_slots + c], 0.575) : 0.0;
}

// Rows of the per-face table, [face][row][column slot]: the neighbour's kh,
// the penalty sigma, and n . grad(lambda') of the neighbour's three vertices
// (n the face's outward normal); zero on faces without a neighbour.
constexpr int kHfRows = 5;

__global__ __launch_bounds__(256) void hface_kernel(DevMesh m, const double* kh, double eta, double* hf) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int CS = m.n_col_slots;
  if (c >= CS) return;
  const double* geo = m.geo;
  double gl[3][2], Jh;
  lambda_grads<double>(geo, CS, c, gl, Jh);
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const int ncol = m.nlay[c] > 0 ? m.nbr_col[e * CS + c] : -1;
    double v[kHfRows] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (ncol >= 0) {
      const double nx = geo[(G_NX + e) * CS + c], ny = geo[(G_NY + e) * CS + c];
      const double Le = geo[(G_LE + e) * CS + c];
      double gn[3][2], Jn;
      lambda_grads<double>(geo, CS, ncol, gn, Jn);
      v[0] = kh[ncol];
      const double h = (Jh < Jn ? Jh : Jn) / Le;
      v[1] = eta * 0.5 * (kh[c] + v[0]) / h;
#pragma unroll
      for (int j = 0; j < 3; ++j) v[2 + j] = nx * gn[j][0] + ny * gn[j][1];
    }
#pragma unroll
    for (int r = 0; r < kHfRows; ++r) hf[(size_t)(e * kHfRows + r) * CS + c] = v[r];
  }
}

// Field-independent data of one lateral face of a column.
template <typename R>
struct HFace {
  bool interior;
  int nslot, depth, nA, nB;  // neighbour layer-0 slot, depth, its nodes at the edge ends A and B
  int nlane;                 // neighbour lane when it is in the same cell, else -1
  int hidx;                  // else its place in the cell's list of other-cell faces
  R Le, sig, khn;            // edge length, penalty, neighbour kh
  R dn[3], dnn[3];           // n . grad(lambda) of the own and the neighbour's basis
};

constexpr int kHdiffLayers = 2;   // layers per workgroup (the 2-layer tile table)

// With HALO, the values of the neighbours in other cells are staged in LDS
// by the whole workgroup, one field ahead of its use: each thread loads a
// few of the tile's (face, layer, node) items of the next field while the
// current field computes, stores them after it, and one barrier per field
// publishes them, instead of each thread gathering its own other-cell
// neighbours in a memory round per field (5% faster in FP64; the gathers'
// scattered 8-byte reads themselves remain).  Cells with more than kHaloCap
// such faces (none on a locality-ordered mesh of 64-column cells) take the
// kernel without HALO, which gathers them per thread.
constexpr int kHaloCap = 64;
constexpr int kHaloItems = (kHaloCap * kHdiffLayers * 6 + kCell * kHdiffLayers - 1) / (kCell * kHdiffLayers);

template <typename R, int NF, bool OUT2, bool HALO>
__global__ __launch_bounds__(kCell * kHdiffLayers) void hdiff_kernel(HdiffArgs a) {
  const DevMesh& m = a.m;
  const WgTile tile = a.tiles[blockIdx.x];
  const int lane = threadIdx.x % kCell;
  const int l = tile.layer0 + threadIdx.x / kCell;
  const int cell = tile.cell;
  const int c = cell * kCell + lane;
  const size_t S = (size_t)m.n_slots, LS = (size_t)m.n_lslots;
  const R* Ts = static_cast<const R*>(a.Ts);
  // the tile's stage input, [row][layer][lane]: neighbours in the same cell
  // are read from here
  __shared__ R sh[6 * NF][kHdiffLayers][kCell];
  // other-cell neighbours of one field, double-buffered: [buffer][face][layer][node]
  __shared__ R hb[HALO ? 2 : 1][HALO ? kHaloCap : 1][kHdiffLayers][6];
  const int li = threadIdx.x / kCell;
  const bool live = l < m.nlay[c];
  const int64_t p = (int64_t)m.cell_base[cell] + lane + (int64_t)l * kCell;
  const int CS = m.n_col_slots;
  const R* geo = geo_rows<R>(m);
  const R* zl = level_rows<R>(m);
  const uint32_t cbase = (uint32_t)m.cell_base[cell];
  R* Out = static_cast<R*>(a.Tout);
  R* Out2 = static_cast<R*>(a.Tout2);
  const R c1 = R(a.c1), c2 = R(a.c2);

  // per-column data first (every column slot is in bounds), so that its
  // loads are in flight together with the staging loads below
  R gl[3][2], Jh;
  lambda_grads<R>(geo, CS, c, gl, Jh);
  const R kh = R(a.kh[c]);

  HFace<R> fc[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    HFace<R>& F = fc[e];
    const R nx = geo[(G_NX + e) * CS + c], ny = geo[(G_NY + e) * CS + c];
    F.Le = geo[(G_LE + e) * CS + c];
    F.nslot = m.nbr_slot[e * CS + c];
    F.interior = F.nslot >= 0;
    const uint32_t nl_ = (uint32_t)F.nslot - cbase;
    F.nlane = (F.interior && nl_ < (uint32_t)kCell) ? (int)nl_ : -1;
    F.hidx = HALO ? m.halo_idx[e * CS + c] : -1;
    const int meta = m.nbr_meta[e * CS + c];
    F.depth = F.interior ? (meta >> 2) : 0;
    const int kp = meta & 3;
    F.nA = (kp + 1) % 3;
    F.nB = kp;
#pragma unroll
    for (int j = 0; j < 3; ++j) F.dn[j] = nx * gl[j][0] + ny * gl[j][1];
    const double* hfe = a.hface + (size_t)(e * kHfRows) * CS + c;
    F.khn = R(hfe[0]);
    F.sig = R(hfe[(size_t)CS]);
#pragma unroll
    for (int j = 0; j < 3; ++j) F.dnn[j] = R(hfe[(size_t)(2 + j) * CS]);
  }

  // this thread's halo items: item it = (face j, layer lj, node i), read
  // from the neighbour's slot at the tile's layer when the neighbour has it
  uint32_t hsrc[HALO ? kHaloItems : 1];
  int hdst[HALO ? kHaloItems : 1];
  R hv[HALO ? kHaloItems : 1];
  if constexpr (HALO) {
    const int hbase = m.halo_off[cell];
    const int hn = m.halo_off[cell + 1] - hbase;
#pragma unroll
    for (int k = 0; k < kHaloItems; ++k) {
      // consecutive threads take consecutive faces of the list (sorted by the
      // neighbour's slot) for one (node, layer), so neighbouring lanes read
      // nearby addresses of one row
      const int it = (int)threadIdx.x + k * kCell * kHdiffLayers;
      const int j = it % kHaloCap, lj = (it / kHaloCap) % kHdiffLayers, i = it / (kHaloCap * kHdiffLayers);
      const int ll = tile.layer0 + lj;
      // list index in bounds for every thread (entry 0 exists), used only when valid
      const int e = j < hn ? hbase + j : 0;
      const int nslot = m.halo_slot[e], ndepth = m.halo_depth[e];
      const bool ok = j < hn && lj < (int)tile.nlay && ll < ndepth;
      hdst[k] = ok ? (j * kHdiffLayers + lj) * 6 + i : -1;
      // an invalid item reads offset 0 (in bounds) and is never stored
      hsrc[k] = ok ? ((uint32_t)i * (uint32_t)S + (uint32_t)nslot + (uint32_t)ll * kCell) * (uint32_t)sizeof(R) : 0u;
      hv[k] = *reinterpret_cast<const R*>(reinterpret_cast<const char*>(Ts) + hsrc[k]);
    }
  }

  const int64_t lt = (int64_t)m.cell_lbase[cell] + lane + (int64_t)l * kCell;
  R dz[3] = {R(0), R(0), R(0)};
  if (live) {
#pragma unroll
    for (int v = 0; v < 3; ++v) dz[v] = zl[v * LS + (size_t)lt] - zl[v * LS + (size_t)(lt + kCell)];
#pragma unroll
    for (int r = 0; r < 6 * NF; ++r) sh[r][li][lane] = Ts[(size_t)r * S + (size_t)p];
  }
  if constexpr (HALO) {
#pragma unroll
    for (int k = 0; k < kHaloItems; ++k)
      if (hdst[k] >= 0) (&hb[0][0][0][0])[hdst[k]] = hv[k];
  }
  __syncthreads();
  if (!HALO && !live) return;
  {
    // volume factor kh int_K z_zeta J_h dxi deta = kh J_h (dz_0 + dz_1 + dz_2) / 12
    const R vf = kh * Jh * (dz[0] + dz[1] + dz[2]) * R(1.0 / 12.0);
    // Mz^-1 = sc * cofactors of m (Mz = J_h/120 m), M^-1 = [2 -1; -1 2] (x) Mz^-1
    const R m00 = R(3) * dz[0] + dz[1] + dz[2], m11 = dz[0] + R(3) * dz[1] + dz[2];
    const R m22 = dz[0] + dz[1] + R(3) * dz[2];
    const R m01 = dz[0] + dz[1] + R(0.5) * dz[2], m02 = dz[0] + dz[2] + R(0.5) * dz[1];
    const R m12 = dz[1] + dz[2] + R(0.5) * dz[0];
    const R k00 = m11 * m22 - m12 * m12, k01 = m02 * m12 - m01 * m22, k02 = m01 * m12 - m02 * m11;
    const R k11 = m00 * m22 - m02 * m02, k12 = m01 * m02 - m00 * m12, k22 = m00 * m11 - m01 * m01;
    const R sc = R(120) / (Jh * (m00 * k00 + m01 * k01 + m02 * k02));
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const R* Tf = Ts + (size_t)(f * 6) * S;
      // the next field's halo items, stored after this field's arithmetic
      if constexpr (HALO) {
        if (f + 1 < NF) {
          const char* nb = reinterpret_cast<const char*>(Ts + (size_t)((f + 1) * 6) * S);
#pragma unroll
          for (int k = 0; k < kHaloItems; ++k) hv[k] = *reinterpret_cast<const R*>(nb + hsrc[k]);
        }
      }
      if (HALO && !live) goto next_field;
      {
      // the field's current output values, loaded before its arithmetic
      R o[6], o2[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        const size_t oi = (size_t)(f * 6 + i) * S + (size_t)p;
        o[i] = Out[oi];
        o2[i] = OUT2 ? Out2[oi] : R(0);
      }
      R T[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) T[i] = sh[f * 6 + i][li][lane];
      R gt[2], gb[2];
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        gt[d] = gl[0][d] * T[0] + gl[1][d] * T[1] + gl[2][d] * T[2];
        gb[d] = gl[0][d] * T[3] + gl[1][d] * T[4] + gl[2][d] * T[5];
      }
      R res[6];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const R dt_ = gl[j][0] * gt[0] + gl[j][1] * gt[1];
        const R db_ = gl[j][0] * gb[0] + gl[j][1] * gb[1];
        res[j] = -vf * (R(2.0 / 3.0) * dt_ + R(1.0 / 3.0) * db_);
        res[j + 3] = -vf * (R(1.0 / 3.0) * dt_ + R(2.0 / 3.0) * db_);
      }
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        const HFace<R>& F = fc[e];
        if (!(F.interior && l < F.depth)) continue;
        const int A = e, B = (e + 1) % 3;
        const size_t q = (size_t)F.nslot + (size_t)l * kCell;
        R Tn[6];
        if (F.nlane >= 0) {
#pragma unroll
          for (int i = 0; i < 6; ++i) Tn[i] = sh[f * 6 + i][li][F.nlane];
        } else if constexpr (HALO) {
#pragma unroll
          for (int i = 0; i < 6; ++i) Tn[i] = hb[f & 1][F.hidx][li][i];
        } else {
#pragma unroll
          for (int i = 0; i < 6; ++i) Tn[i] = Tf[(size_t)i * S + q];
        }
        // normal derivatives of both sides on the top and bottom traces
        const R gnt = F.dn[0] * T[0] + F.dn[1] * T[1] + F.dn[2] * T[2];
        const R gnb = F.dn[0] * T[3] + F.dn[1] * T[4] + F.dn[2] * T[5];
        const R gmt = F.dnn[0] * Tn[0] + F.dnn[1] * Tn[1] + F.dnn[2] * Tn[2];
        const R gmb = F.dnn[0] * Tn[3] + F.dnn[1] * Tn[4] + F.dnn[2] * Tn[5];
        const R Ft = R(0.5) * (kh * gnt + F.khn * gmt);
        const R Fb = R(0.5) * (kh * gnb + F.khn * gmb);
        // jumps at the edge ends, top and bottom
        const R jAt = T[A] - Tn[F.nA], jBt = T[B] - Tn[F.nB];
        const R jAb = T[A + 3] - Tn[F.nA + 3], jBb = T[B + 3] - Tn[F.nB + 3];
        const R dA = dz[A], dB = dz[B];
        const R wA = (R(2) * dA + dB) * R(1.0 / 12.0), wB = (dA + R(2) * dB) * R(1.0 / 12.0);
        const R Le = F.Le;
        // consistency term {kh grad T . n} phi_i on the face nodes
        const R ct = R(2.0 / 3.0) * Ft + R(1.0 / 3.0) * Fb, cb = R(1.0 / 3.0) * Ft + R(2.0 / 3.0) * Fb;
        res[A] += Le * wA * ct;
        res[B] += Le * wB * ct;
        res[A + 3] += Le * wA * cb;
        res[B + 3] += Le * wB * cb;
        // symmetry term 1/2 kh (grad phi_i . n) [T] on all six nodes
        const R Qt = jAt * wA + jBt * wB, Qb = jAb * wA + jBb * wB;
        const R st = R(0.5) * kh * Le * (R(2.0 / 3.0) * Qt + R(1.0 / 3.0) * Qb);
        const R sb = R(0.5) * kh * Le * (R(1.0 / 3.0) * Qt + R(2.0 / 3.0) * Qb);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          res[j] += F.dn[j] * st;
          res[j + 3] += F.dn[j] * sb;
        }
        // penalty -sigma [T] phi_i on the face nodes
        const R eAA = (R(3) * dA + dB) * R(1.0 / 24.0), eAB = (dA + dB) * R(1.0 / 24.0);
        const R eBB = (dA + R(3) * dB) * R(1.0 / 24.0);
        const R pAt = jAt * eAA + jBt * eAB, pBt = jAt * eAB + jBt * eBB;
        const R pAb = jAb * eAA + jBb * eAB, pBb = jAb * eAB + jBb * eBB;
        const R sl = F.sig * Le;
        res[A] -= sl * (R(2.0 / 3.0) * pAt + R(1.0 / 3.0) * pAb);
        res[B] -= sl * (R(2.0 / 3.0) * pBt + R(1.0 / 3.0) * pBb);
        res[A + 3] -= sl * (R(1.0 / 3.0) * pAt + R(2.0 / 3.0) * pAb);
        res[B + 3] -= sl * (R(1.0 / 3.0) * pBt + R(2.0 / 3.0) * pBb);
      }
      // L = M^-1 res, then Tout += c1 L (and Tout2 += c2 L)
      const R ht[3] = {R(2) * res[0] - res[3], R(2) * res[1] - res[4], R(2) * res[2] - res[5]};
      const R hb[3] = {R(2) * res[3] - res[0], R(2) * res[4] - res[1], R(2) * res[5] - res[2]};
      R L[6];
      L[0] = sc * (k00 * ht[0] + k01 * ht[1] + k02 * ht[2]);
      L[1] = sc * (k01 * ht[0] + k11 * ht[1] + k12 * ht[2]);
      L[2] = sc * (k02 * ht[0] + k12 * ht[1] + k22 * ht[2]);
      L[3] = sc * (k00 * hb[0] + k01 * hb[1] + k02 * hb[2]);
      L[4] = sc * (k01 * hb[0] + k11 * hb[1] + k12 * hb[2]);
      L[5] = sc * (k02 * hb[0] + k12 * hb[1] + k22 * hb[2]);
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        const size_t oi = (size_t)(f * 6 + i) * S + (size_t)p;
        Out[oi] = o[i] + c1 * L[i];
        if (OUT2) Out2[oi] = o2[i] + c2 * L[i];
      }
      }
    next_field:
      if constexpr (HALO) {
        if (f + 1 < NF) {
#pragma unroll
          for (int k = 0; k < kHaloItems; ++k)
            if (hdst[k] >= 0) (&hb[(f + 1) & 1][0][0][0])[hdst[k]] = hv[k];
          __syncthreads();
        }
      }
    }
  }
}

template <typename R, bool OUT2, bool HALO>
hipError_t launch_halo(const HdiffArgs& a, hipStream_t s) {
  const dim3 grid(a.n_tiles), block(kCell * kHdiffLayers);
  switch (a.n_fields) {
    case 1: hipLaunchKernelGGL((hdiff_kernel<R, 1, OUT2, HALO>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((hdiff_kernel<R, 2, OUT2, HALO>), grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL((hdiff_kernel<R, 3, OUT2, HALO>), grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL((hdiff_kernel<R, 4, OUT2, HALO>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename R, bool OUT2>
hipError_t launch_nf(const HdiffArgs& a, hipStream_t s) {
  return a.m.halo_max <= kHaloCap ? launch_halo<R, OUT2, true>(a, s) : launch_halo<R, OUT2, false>(a, s);
}

}  // namespace

hipError_t launch_hdiff_setup(const DevMesh& m, double coef, double eta, double* kh, double* hface,
                              hipStream_t s) {
  const int n = m.n_col_slots;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(okubo_kernel, dim3((n + 255) / 256), dim3(256), 0, s, m, coef, kh);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(hface_kernel, dim3((n + 255) / 256), dim3(256), 0, s, m, kh, eta, hface);
  return hipGetLastError();
}

hipError_t launch_hdiff(const HdiffArgs& a, bool fp32, hipStream_t s) {
  if (a.n_tiles == 0) return hipSuccess;
  if (a.tile_layers != kHdiffLayers) return hipErrorInvalidValue;
  const bool out2 = a.Tout2 != nullptr;
  if (fp32) return out2 ? launch_nf<float, true>(a, s) : launch_nf<float, false>(a, s);
  return out2 ? launch_nf<double, true>(a, s) : launch_nf<double, false>(a, s);
}

}  // namespace sdg
