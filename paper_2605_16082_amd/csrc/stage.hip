// Explicit DG operator and SSP-RK3 stage on extruded linear prisms.
//
// One thread per prism.  A workgroup covers 1, 2 or 4 consecutive layers of
// one cell of 64 columns (one wavefront per layer), so each wavefront reads 64
// consecutive slots of every nodal array (cell layout, section 2.1.1 of the
// paper, with wavefront-sized cells).  No load depends on control flow: lanes
// past their column's depth compute on in-bounds padding slots and skip the
// store, and faces without a neighbour address the prism's own nodes and
// select the exterior value, so each wavefront needs only two dependent
// memory round trips (own data and neighbour slots, then neighbour data).  Per prism and field it computes
//
//   R_i = int_K T U.grad(phi_i) dV - sum_faces int_f phi_i Fhat dS
//   L   = M^-1 R                          (block-diagonal mass matrix)
//   out = a Tn + b (Ts + dt L)            (SSP-RK3, Shu-Osher form)
//
// with the quadrature that defines the operator: 6-point degree-4 triangle
// rule x 2-point Gauss in zeta for the volume and horizontal faces, 3-point
// Gauss along edges x 2-point in zeta for lateral faces; upwind flux per
// quadrature point, Fhat dS = max(u_n dS, 0) T_in + min(u_n dS, 0) T_out
// with u_n the average of the two velocity traces.
//
// The volume term uses contravariant fluxes: with alpha = y_eta u - x_eta v
// and beta = x_xi v - y_xi u, the integrand T U.(|J| grad phi_i) equals
// T (dphi_i/dxi z_zeta alpha + dphi_i/deta z_zeta beta
//    + dphi_i/dzeta (J_h w - z_xi alpha - z_eta beta)),
// so the geometric work is shared by all fields.  The mass matrix of a prism
// is H (x) Mz with H = [2 1; 1 2]/3 and Mz_ab = J_h int lambda_a lambda_b
// z_zeta, so M^-1 = [2 -1; -1 2] (x) Mz^-1 and only a symmetric 3x3 inverse
// is needed.
#include <atomic>

#include "internal.h"

namespace sdg {
namespace {

// 6-point triangle rule: barycentric points (lambda0, lambda1, lambda2);
// weights include the reference-triangle area 1/2.
constexpr double kA1 = 0.44594849091596488631832925388305199;
constexpr double kB1 = 0.10810301816807022736334149223390401;
constexpr double kW1 = 0.5 * 0.22338158967801146569500700843312280;
constexpr double kA2 = 0.091576213509770743459571463402201508;
constexpr double kB2 = 0.81684757298045851308085707319559698;
constexpr double kW2 = 0.5 * 0.10995174365532186763832632490021053;
constexpr double kL0[6] = {kB1, kA1, kA1, kB2, kA2, kA2};
constexpr double kL1[6] = {kA1, kA1, kB1, kA2, kA2, kB2};
constexpr double kL2[6] = {kA1, kB1, kA1, kA2, kB2, kA2};
constexpr double kTw[6] = {kW1, kW1, kW1, kW2, kW2, kW2};
// zeta = -1/sqrt(3), +1/sqrt(3): t = (1+zeta)/2, b = (1-zeta)/2; weights 1.
constexpr double kZt[2] = {0.21132486540518711774542560974902127, 0.78867513459481288225457439025097873};
constexpr double kZb[2] = {0.78867513459481288225457439025097873, 0.21132486540518711774542560974902127};
// 3-point Gauss on [0, 1].
constexpr double kS[3] = {0.11270166537925831148207346002176005, 0.5, 0.88729833462074168851792653997823995};
constexpr double kSw[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};

template <typename R> __device__ __forceinline__ const R* geo_of(const DevMesh& m);
template <> __device__ __forceinline__ const double* geo_of<double>(const DevMesh& m) { return m.geo; }
template <> __device__ __forceinline__ const float* geo_of<float>(const DevMesh& m) { return m.geo32; }
template <typename R> __device__ __forceinline__ const R* zl_of(const DevMesh& m);
template <> __device__ __forceinline__ const double* zl_of<double>(const DevMesh& m) { return m.zl; }
template <> __device__ __forceinline__ const float* zl_of<float>(const DevMesh& m) { return m.zl32; }

// Load from a row whose base pointer is wavefront-uniform, at a 32-bit byte
// offset: lets the compiler use the scalar-base + vector-offset load form
// instead of per-lane 64-bit address arithmetic.
template <typename T>
__device__ __forceinline__ T ldb(const T* __restrict__ row, uint32_t byte_off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(row) + byte_off);
}
template <typename T>
__device__ __forceinline__ void stb(T* __restrict__ row, uint32_t byte_off, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(row) + byte_off) = v;
}


template <typename R>
__device__ __forceinline__ R upos(R x) { return x > R(0) ? x : R(0); }
template <typename R>
__device__ __forceinline__ R uneg(R x) { return x < R(0) ? x : R(0); }

template <typename R, int NF, bool WZ, bool RHS, bool READ_TN>
__device__ __forceinline__ void stage_tile(const StageArgs& a, const WgTile tile) {
  const DevMesh& m = a.m;
  const int lane = threadIdx.x & (kCell - 1);
  const int l = tile.layer0 + (threadIdx.x >> 6);
  const int c = tile.cell * kCell + lane;
  // Threads past their column's depth still run (on in-bounds padding slots
  // of their cell) so that no load waits on nlay; only the store is masked.
  const int N = m.nlay[c];
  const int depth = (m.cell_base[tile.cell + 1] - m.cell_base[tile.cell]) / kCell;
  if (l >= depth) return;  // uniform per wavefront
  const bool active = l < N;

  const size_t S = (size_t)m.n_slots;
  const size_t LS = (size_t)m.n_lslots;
  const int CS = m.n_col_slots;
  const uint32_t p = (uint32_t)m.cell_base[tile.cell] + (uint32_t)l * kCell + lane;
  const uint32_t lt = (uint32_t)m.cell_lbase[tile.cell] + (uint32_t)l * kCell + lane;
  const uint32_t rs = (uint32_t)(S * sizeof(R));     // bytes per node row
  const uint32_t po = p * (uint32_t)sizeof(R);       // this prism's byte offset in a row
  const uint32_t co = (uint32_t)c * (uint32_t)sizeof(R);
  const R* __restrict__ Ts = static_cast<const R*>(a.Ts);
  const R* __restrict__ U = static_cast<const R*>(a.U);
  const R* __restrict__ geo = geo_of<R>(m);
  const R* __restrict__ zl = zl_of<R>(m);
  const uint32_t co4 = (uint32_t)c * 4u;

  const R xxi = ldb(geo + G_XXI * CS, co), xet = ldb(geo + G_XET * CS, co);
  const R yxi = ldb(geo + G_YXI * CS, co), yet = ldb(geo + G_YET * CS, co);
  const R Jh = ldb(geo + G_JH * CS, co);

  R zt[3], zb[3], dz[3];
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    zt[v] = ldb(zl + v * LS, lt * (uint32_t)sizeof(R));
    zb[v] = ldb(zl + v * LS, (lt + kCell) * (uint32_t)sizeof(R));
    dz[v] = zt[v] - zb[v];
  }

  R T[NF][6];
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int i = 0; i < 6; ++i) T[f][i] = ldb(Ts + (size_t)(f * 6 + i) * S, po);
  R u[6], v[6], w[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    u[i] = ldb(U + (size_t)(0 * 6 + i) * S, po);
    v[i] = ldb(U + (size_t)(1 * 6 + i) * S, po);
    w[i] = WZ ? R(0) : ldb(U + (size_t)(2 * 6 + i) * S, po);
  }

  R res[NF][6];
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int i = 0; i < 6; ++i) res[f][i] = R(0);

  // ---------------- volume term ----------------
  {
    R sx[NF][2], se[NF][2], sz[NF][3];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      sx[f][0] = sx[f][1] = se[f][0] = se[f][1] = R(0);
      sz[f][0] = sz[f][1] = sz[f][2] = R(0);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const R tk = R(kZt[k]), bk = R(kZb[k]);
      R ua[3], va[3], wa[3], ta[NF][3];
#pragma unroll
      for (int n = 0; n < 3; ++n) {
        ua[n] = tk * u[n] + bk * u[n + 3];
        va[n] = tk * v[n] + bk * v[n + 3];
        wa[n] = WZ ? R(0) : tk * w[n] + bk * w[n + 3];
#pragma unroll
        for (int f = 0; f < NF; ++f) ta[f][n] = tk * T[f][n] + bk * T[f][n + 3];
      }
      const R z_xi = tk * (zt[1] - zt[0]) + bk * (zb[1] - zb[0]);
      const R z_et = tk * (zt[2] - zt[0]) + bk * (zb[2] - zb[0]);
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const R l0 = R(kL0[q]), l1 = R(kL1[q]), l2 = R(kL2[q]), wq = R(kTw[q]);
        const R uq = l0 * ua[0] + l1 * ua[1] + l2 * ua[2];
        const R vq = l0 * va[0] + l1 * va[1] + l2 * va[2];
        const R zz = R(0.5) * (l0 * dz[0] + l1 * dz[1] + l2 * dz[2]);
        const R al = yet * uq - xet * vq;
        const R be = xxi * vq - yxi * uq;
        const R Vx = wq * zz * al;
        const R Ve = wq * zz * be;
        R Vz = -(z_xi * al + z_et * be);
        if (!WZ) Vz += Jh * (l0 * wa[0] + l1 * wa[1] + l2 * wa[2]);
        Vz *= wq;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          const R tq = l0 * ta[f][0] + l1 * ta[f][1] + l2 * ta[f][2];
          sx[f][k] += tq * Vx;
          se[f][k] += tq * Ve;
          const R wz = tq * Vz;
          sz[f][0] += l0 * wz;
          sz[f][1] += l1 * wz;
          sz[f][2] += l2 * wz;
        }
      }
    }
    // dphi/dxi = dlambda/dxi * (t or b), dphi/dzeta = +-lambda/2
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const R sxt = R(kZt[0]) * sx[f][0] + R(kZt[1]) * sx[f][1];
      const R sxb = R(kZb[0]) * sx[f][0] + R(kZb[1]) * sx[f][1];
      const R set = R(kZt[0]) * se[f][0] + R(kZt[1]) * se[f][1];
      const R seb = R(kZb[0]) * se[f][0] + R(kZb[1]) * se[f][1];
      res[f][0] = -sxt - set + R(0.5) * sz[f][0];
      res[f][1] = sxt + R(0.5) * sz[f][1];
      res[f][2] = set + R(0.5) * sz[f][2];
      res[f][3] = -sxb - seb - R(0.5) * sz[f][0];
      res[f][4] = sxb - R(0.5) * sz[f][1];
      res[f][5] = seb - R(0.5) * sz[f][2];
    }
  }

  // ---------------- lateral faces ----------------
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const int A = e, B = (e + 1) % 3;
    const int nslot = ldb(m.nbr_slot + e * CS, co4);
    const int meta = ldb(m.nbr_meta + e * CS, co4);
    const bool interior = nslot >= 0;
    const bool wall = interior && l >= (meta >> 2);   // shallower neighbour: no flux
    const bool live = interior && !wall;
    const R nx = ldb(geo + (G_NX + e) * CS, co), ny = ldb(geo + (G_NY + e) * CS, co);
    const R Le = ldb(geo + (G_LE + e) * CS, co);
    // normal velocity at the 4 face nodes (A top, B top, A bottom, B bottom)
    R un[4] = {nx * u[A] + ny * v[A], nx * u[B] + ny * v[B], nx * u[A + 3] + ny * v[A + 3],
               nx * u[B + 3] + ny * v[B + 3]};
    // byte offsets (within a field block) of the neighbour's 4 face nodes;
    // without a live neighbour they point at this prism's own nodes (never
    // used, but always in bounds) so the loads need no branch
    uint32_t no[4];
    {
      const int kp = meta & 3;
      const uint32_t nA = live ? (uint32_t)((kp + 1) % 3) : (uint32_t)A;
      const uint32_t nB = live ? (uint32_t)kp : (uint32_t)B;
      const uint32_t pno = live ? ((uint32_t)nslot + (uint32_t)l * kCell) * (uint32_t)sizeof(R) : po;
      no[0] = nA * rs + pno;
      no[1] = nB * rs + pno;
      no[2] = no[0] + 3u * rs;
      no[3] = no[1] + 3u * rs;
    }
    {
      const int nodes_in[4] = {A, B, A + 3, B + 3};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const R uo = ldb(U, no[j]);
        const R vo = ldb(U + 6 * S, no[j]);
        const R avg = R(0.5) * (un[j] + nx * uo + ny * vo);
        un[j] = live ? avg : un[j];
        (void)nodes_in;
      }
    }
    const R fscale = wall ? R(0) : R(1);
    R up[3][2], um[3][2];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const R s = R(kS[j]), s1 = R(1) - R(kS[j]);
      const R dS = fscale * R(kSw[j]) * Le * R(0.5) * (s1 * dz[A] + s * dz[B]);
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const R tk = R(kZt[k]), bk = R(kZb[k]);
        const R q = (s1 * (tk * un[0] + bk * un[2]) + s * (tk * un[1] + bk * un[3])) * dS;
        up[j][k] = upos(q);
        um[j][k] = uneg(q);
      }
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      R to[4];
      {
        const R* fb = Ts + (size_t)(f * 6) * S;
        const R te = R(a.t_ext[f]);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const R x = ldb(fb, no[j]);
          to[j] = interior ? x : te;
        }
      }
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const R s = R(kS[j]), s1 = R(1) - R(kS[j]);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const R tk = R(kZt[k]), bk = R(kZb[k]);
          const R ti = s1 * (tk * T[f][A] + bk * T[f][A + 3]) + s * (tk * T[f][B] + bk * T[f][B + 3]);
          const R tq = s1 * (tk * to[0] + bk * to[2]) + s * (tk * to[1] + bk * to[3]);
          const R fl = up[j][k] * ti + um[j][k] * tq;
          res[f][A] -= s1 * tk * fl;
          res[f][B] -= s * tk * fl;
          res[f][A + 3] -= s1 * bk * fl;
          res[f][B + 3] -= s * bk * fl;
        }
      }
    }
  }

  // ---------------- top and bottom faces ----------------
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    // side 0: top face (nodes 0..2, neighbour above, its bottom nodes);
    // side 1: bottom face (nodes 3..5, neighbour below, its top nodes).
    const int o = side == 0 ? 0 : 3;
    const int oo = side == 0 ? 3 : 0;
    const bool has_nb = side == 0 ? (l > 0) : (l < N - 1);
    // the address only needs the (wavefront-uniform) cell depth; the value
    // select uses the column's own depth
    const bool nb_slot = side == 0 ? (l > 0) : (l + 1 < depth);
    const uint32_t pno = nb_slot ? (side == 0 ? p - kCell : p + kCell) * (uint32_t)sizeof(R) : po;
    const R* zf = side == 0 ? zt : zb;
    // J_h * grad_h z of the (planar) face
    const R zxi = zf[1] - zf[0], zet = zf[2] - zf[0];
    const R jzx = zxi * yet - zet * yxi;
    const R jzy = zet * xxi - zxi * xet;
    const R sg = side == 0 ? R(1) : R(-1);
    R un[3];
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      R val = -(u[o + n] * jzx + v[o + n] * jzy);
      if (!WZ) val += Jh * w[o + n];
      un[n] = val;
    }
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const R uo = ldb(U + (size_t)(0 * 6 + oo + n) * S, pno);
      const R vo = ldb(U + (size_t)(1 * 6 + oo + n) * S, pno);
      R val = -(uo * jzx + vo * jzy);
      if (!WZ) val += Jh * ldb(U + (size_t)(2 * 6 + oo + n) * S, pno);
      un[n] = has_nb ? R(0.5) * (un[n] + val) : un[n];
    }
    R up[6], um[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const R fq = sg * R(kTw[q]) * (R(kL0[q]) * un[0] + R(kL1[q]) * un[1] + R(kL2[q]) * un[2]);
      up[q] = upos(fq);
      um[q] = uneg(fq);
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      R to[3];
      {
        const R te = R(a.t_ext[f]);
#pragma unroll
        for (int n = 0; n < 3; ++n) {
          const R x = ldb(Ts + (size_t)(f * 6 + oo + n) * S, pno);
          to[n] = has_nb ? x : te;
        }
      }
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const R l0 = R(kL0[q]), l1 = R(kL1[q]), l2 = R(kL2[q]);
        const R ti = l0 * T[f][o] + l1 * T[f][o + 1] + l2 * T[f][o + 2];
        const R tq = l0 * to[0] + l1 * to[1] + l2 * to[2];
        const R fl = up[q] * ti + um[q] * tq;
        res[f][o] -= l0 * fl;
        res[f][o + 1] -= l1 * fl;
        res[f][o + 2] -= l2 * fl;
      }
    }
  }

  // ---------------- M^-1 and the stage combination ----------------
  // Mz = J_h/120 * m, m_aa = 3 dz_a + dz_b + dz_c, m_ab = dz_a + dz_b + dz_c / 2.
  const R m00 = R(3) * dz[0] + dz[1] + dz[2];
  const R m11 = dz[0] + R(3) * dz[1] + dz[2];
  const R m22 = dz[0] + dz[1] + R(3) * dz[2];
  const R m01 = dz[0] + dz[1] + R(0.5) * dz[2];
  const R m02 = dz[0] + dz[2] + R(0.5) * dz[1];
  const R m12 = dz[1] + dz[2] + R(0.5) * dz[0];
  const R c00 = m11 * m22 - m12 * m12;
  const R c01 = m02 * m12 - m01 * m22;
  const R c02 = m01 * m12 - m02 * m11;
  const R c11 = m00 * m22 - m02 * m02;
  const R c12 = m01 * m02 - m00 * m12;
  const R c22 = m00 * m11 - m01 * m01;
  const R det = m00 * c00 + m01 * c01 + m02 * c02;
  const R sc = R(120) / (Jh * det);  // Mz^-1 = sc * cofactor matrix

  const R* __restrict__ Tn = static_cast<const R*>(a.Tn);
  R* __restrict__ Out = static_cast<R*>(a.Tout);
  const R dt = R(a.dt), ca = R(a.a), cb = R(a.b);
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const R ht[3] = {R(2) * res[f][0] - res[f][3], R(2) * res[f][1] - res[f][4],
                     R(2) * res[f][2] - res[f][5]};
    const R hb[3] = {R(2) * res[f][3] - res[f][0], R(2) * res[f][4] - res[f][1],
                     R(2) * res[f][5] - res[f][2]};
    R L[6];
    L[0] = sc * (c00 * ht[0] + c01 * ht[1] + c02 * ht[2]);
    L[1] = sc * (c01 * ht[0] + c11 * ht[1] + c12 * ht[2]);
    L[2] = sc * (c02 * ht[0] + c12 * ht[1] + c22 * ht[2]);
    L[3] = sc * (c00 * hb[0] + c01 * hb[1] + c02 * hb[2]);
    L[4] = sc * (c01 * hb[0] + c11 * hb[1] + c12 * hb[2]);
    L[5] = sc * (c02 * hb[0] + c12 * hb[1] + c22 * hb[2]);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      const size_t row = (size_t)(f * 6 + i) * S;
      R out;
      if (RHS) {
        out = L[i];
      } else {
        out = cb * (T[f][i] + dt * L[i]);
        if (READ_TN) out += ca * ldb(Tn + row, po);
      }
      if (active) stb(Out + row, po, out);
    }
  }
}

// One workgroup per tile, or (a.persistent) a grid sized to what the chip
// holds at once, each workgroup walking tiles with a stride.  With the XCD
// remap, tile ranges are split into 8 contiguous parts and workgroup b, which
// the dispatcher places on XCD b mod 8, walks part b mod 8, so the tiles that
// share faces are processed on one XCD and its L2 (the grid is a multiple of 8).
template <typename R, int NF, bool WZ, bool RHS, bool READ_TN>
__global__ __launch_bounds__(256) void stage_kernel(StageArgs a) {
  const int b = (int)blockIdx.x;
  int t, end, step;
  if (!a.persistent) {
    t = a.xcd ? xcd_tile(b, a.n_tiles) : b;
    end = t + 1;
    step = 1;
  } else if (a.xcd) {
    const int q = a.n_tiles >> 3, r = a.n_tiles & 7, x = b & 7;
    const int lo = x * q + (x < r ? x : r);
    t = lo + (b >> 3);
    end = lo + q + (x < r ? 1 : 0);
    step = (int)gridDim.x >> 3;
  } else {
    t = b;
    end = a.n_tiles;
    step = (int)gridDim.x;
  }
  for (; t < end; t += step) stage_tile<R, NF, WZ, RHS, READ_TN>(a, a.tiles[t]);
}

// Workgroups of `threads` threads that fit on one CU at once, per kernel
// instance and tile height, queried once.
template <typename R, int NF, bool WZ, bool RHS, bool READ_TN>
hipError_t resident_per_cu(int threads, int* out) {
  static std::atomic<int> cache[5];
  const int k = threads / kCell;
  int v = cache[k].load(std::memory_order_relaxed);
  if (v == 0) {
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &v, reinterpret_cast<const void*>(&stage_kernel<R, NF, WZ, RHS, READ_TN>), threads, 0);
    if (e != hipSuccess) return e;
    if (v < 1) v = 1;
    cache[k].store(v, std::memory_order_relaxed);
  }
  *out = v;
  return hipSuccess;
}

template <typename R, int NF, bool WZ, bool RHS, bool READ_TN>
hipError_t launch_mode(const StageArgs& a, hipStream_t s) {
  const int threads = kCell * a.tile_layers;
  int grid = a.n_tiles;
  if (a.persistent) {
    int per_cu = 1;
    hipError_t e = resident_per_cu<R, NF, WZ, RHS, READ_TN>(threads, &per_cu);
    if (e != hipSuccess) return e;
    grid = (per_cu * a.n_cu) & ~7;
    if (grid < 8) grid = 8;
    const int need = (a.n_tiles + 7) & ~7;
    if (grid > need) grid = need;
  }
  hipLaunchKernelGGL((stage_kernel<R, NF, WZ, RHS, READ_TN>), dim3(grid), dim3(threads), 0, s, a);
  return hipGetLastError();
}

template <typename R, int NF>
hipError_t launch_nf(const StageArgs& a, bool w_zero, bool rhs_only, bool read_tn, hipStream_t s) {
  if (rhs_only) return w_zero ? launch_mode<R, NF, true, true, false>(a, s) : launch_mode<R, NF, false, true, false>(a, s);
  if (read_tn) return w_zero ? launch_mode<R, NF, true, false, true>(a, s) : launch_mode<R, NF, false, false, true>(a, s);
  return w_zero ? launch_mode<R, NF, true, false, false>(a, s) : launch_mode<R, NF, false, false, false>(a, s);
}

template <typename R>
hipError_t launch_r(const StageArgs& a, bool w_zero, bool rhs_only, bool read_tn, hipStream_t s) {
  switch (a.n_fields) {
    case 1: return launch_nf<R, 1>(a, w_zero, rhs_only, read_tn, s);
    case 2: return launch_nf<R, 2>(a, w_zero, rhs_only, read_tn, s);
    case 3: return launch_nf<R, 3>(a, w_zero, rhs_only, read_tn, s);
    case 4: return launch_nf<R, 4>(a, w_zero, rhs_only, read_tn, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_stage(const StageArgs& a, bool fp32, bool w_zero, bool rhs_only, bool read_tn,
                        hipStream_t s) {
  if (a.n_tiles == 0) return hipSuccess;
  return fp32 ? launch_r<float>(a, w_zero, rhs_only, read_tn, s)
              : launch_r<double>(a, w_zero, rhs_only, read_tn, s);
}

}  // namespace sdg
