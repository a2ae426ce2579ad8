// Discrete adjoint of the tracer step (FP64), in the variable Z = M^-1 lambda.
//
// Forward step: x^{n+1} = S P(x^n) + c with P the SSP-RK3 stages of
// L = M^-1 R and S = (M - dt A)^-1 M.  With lambda = M Z the reverse sweep is
//
//   mu       = (M - dt A^T)^-1 M Z^{n+1}                    (transposed solve)
//   dJ/dkappa_l += dt mu^T (dA/dkappa_l) x^{n+1}             (A is linear in kappa)
//   Zb2 = 2/3 (mu + dt Lt mu),  Zb1 = 1/4 (Zb2 + dt Lt Zb2)
//   Z^n = (Zb1 + dt Lt Zb1) + 1/3 mu + 3/4 Zb2                (reverse RK3 stages)
//
// where Lt = M^-1 R_lin^T is the adjoint of L in the M inner product and
// R_lin the advective residual without the exterior inflow values.  Per prism
// q, with the upwind-positive face matrices K+ of the forward kernel,
//
//   (R_lin^T y)_j = int phi_j U.grad(y_h) dV - sum_faces K+ (y_q - y_nbr),
//
// (y_nbr = 0 on open boundaries, no term on walls): the volume part reuses
// the forward kernel's contravariant contractions, the face part is the
// downwind counterpart of the forward upwind flux.
#include "internal.h"

namespace sdg {
namespace {

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
constexpr double kZt[2] = {0.21132486540518711774542560974902127, 0.78867513459481288225457439025097873};
constexpr double kZb[2] = {0.78867513459481288225457439025097873, 0.21132486540518711774542560974902127};
constexpr double kS[3] = {0.11270166537925831148207346002176005, 0.5, 0.88729833462074168851792653997823995};
constexpr double kSw[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};

__device__ __forceinline__ double ld(const double* __restrict__ row, uint32_t byte_off) {
  return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(row) + byte_off);
}
__device__ __forceinline__ void st(double* __restrict__ row, uint32_t byte_off, double v) {
  *reinterpret_cast<double*>(reinterpret_cast<char*>(row) + byte_off) = v;
}
__device__ __forceinline__ double upos(double x) { return x > 0.0 ? x : 0.0; }

// symmetric 3x3 storage: 0:00 1:11 2:22 3:01 4:02 5:12
__device__ __forceinline__ int sidx(int a, int b) {
  return a == b ? a : (a + b == 1 ? 3 : (a + b == 2 ? 4 : 5));
}

// ---------------------------------------------------------------------------
// Adjoint stage: out = b (Y + dt M^-1 R_lin^T Y) + a1 X1 + a2 X2
// ---------------------------------------------------------------------------
struct AdjStageArgs {
  DevMesh m;
  const WgTile* tiles;
  int32_t n_tiles;
  int32_t xcd;
  const double* Y;
  const double* X1;   // may be null (then a1 is ignored)
  const double* X2;
  double* out;        // may alias X1 or X2 (element-local reads), never Y
  const double* U;
  double dt, b, a1, a2;
};

template <int NF, bool WZ>
__global__ __launch_bounds__(256) void adj_stage_kernel(AdjStageArgs a) {
  const DevMesh& m = a.m;
  const WgTile tile = a.tiles[a.xcd ? xcd_tile(blockIdx.x, a.n_tiles) : (int)blockIdx.x];
  const int lane = threadIdx.x & (kCell - 1);
  const int l = tile.layer0 + (threadIdx.x >> 6);
  const int c = tile.cell * kCell + lane;
  const int N = m.nlay[c];
  if (l >= N) return;
  const size_t S = (size_t)m.n_slots;
  const size_t LS = (size_t)m.n_lslots;
  const int CS = m.n_col_slots;
  const uint32_t p = (uint32_t)m.cell_base[tile.cell] + (uint32_t)l * kCell + lane;
  const uint32_t lt = (uint32_t)m.cell_lbase[tile.cell] + (uint32_t)l * kCell + lane;
  const uint32_t rs = (uint32_t)(S * 8);
  const uint32_t po = p * 8u;
  const uint32_t co = (uint32_t)c * 8u;
  const uint32_t co4 = (uint32_t)c * 4u;
  const double* __restrict__ Y = a.Y;
  const double* __restrict__ U = a.U;
  const double* __restrict__ geo = m.geo;

  const double xxi = ld(geo + G_XXI * CS, co), xet = ld(geo + G_XET * CS, co);
  const double yxi = ld(geo + G_YXI * CS, co), yet = ld(geo + G_YET * CS, co);
  const double Jh = ld(geo + G_JH * CS, co);
  double zt[3], zb[3], dz[3];
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    zt[v] = ld(m.zl + v * LS, lt * 8u);
    zb[v] = ld(m.zl + v * LS, (lt + kCell) * 8u);
    dz[v] = zt[v] - zb[v];
  }
  double res[NF][6];
  // the prism's own velocity and Y, loaded once and reused by every term
  double u[6], v[6], w[6], yv[NF][6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    u[i] = ld(U + (size_t)(0 * 6 + i) * S, po);
    v[i] = ld(U + (size_t)(1 * 6 + i) * S, po);
    w[i] = WZ ? 0.0 : ld(U + (size_t)(2 * 6 + i) * S, po);
  }
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int i = 0; i < 6; ++i) yv[f][i] = ld(Y + (size_t)(f * 6 + i) * S, po);

  // ---- volume: int phi_j U.grad(y_h) ----
  {
    double hx[2][3], he[2][3], G[2][6];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const double tk = kZt[k], bk = kZb[k];
      double ua[3], va[3], wa[3];
#pragma unroll
      for (int n = 0; n < 3; ++n) {
        ua[n] = tk * u[n] + bk * u[n + 3];
        va[n] = tk * v[n] + bk * v[n + 3];
        wa[n] = WZ ? 0.0 : tk * w[n] + bk * w[n + 3];
        hx[k][n] = he[k][n] = 0.0;
      }
#pragma unroll
      for (int i = 0; i < 6; ++i) G[k][i] = 0.0;
      const double z_xi = tk * (zt[1] - zt[0]) + bk * (zb[1] - zb[0]);
      const double z_et = tk * (zt[2] - zt[0]) + bk * (zb[2] - zb[0]);
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const double l0 = kL0[q], l1 = kL1[q], l2 = kL2[q], wq = kTw[q];
        const double uq = l0 * ua[0] + l1 * ua[1] + l2 * ua[2];
        const double vq = l0 * va[0] + l1 * va[1] + l2 * va[2];
        const double wz = wq * 0.5 * (l0 * dz[0] + l1 * dz[1] + l2 * dz[2]);
        const double al = yet * uq - xet * vq;
        const double be = xxi * vq - yxi * uq;
        const double Vx = wz * al, Ve = wz * be;
        double Vz = -(z_xi * al + z_et * be);
        if (!WZ) Vz += Jh * (l0 * wa[0] + l1 * wa[1] + l2 * wa[2]);
        Vz *= wq;
        hx[k][0] += l0 * Vx;
        hx[k][1] += l1 * Vx;
        hx[k][2] += l2 * Vx;
        he[k][0] += l0 * Ve;
        he[k][1] += l1 * Ve;
        he[k][2] += l2 * Ve;
        G[k][0] += kL0[q] * kL0[q] * Vz;
        G[k][1] += kL1[q] * kL1[q] * Vz;
        G[k][2] += kL2[q] * kL2[q] * Vz;
        G[k][3] += kL0[q] * kL1[q] * Vz;
        G[k][4] += kL0[q] * kL2[q] * Vz;
        G[k][5] += kL1[q] * kL2[q] * Vz;
      }
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const double* y = yv[f];
      const double d0 = y[0] - y[3], d1 = y[1] - y[4], d2 = y[2] - y[5];
#pragma unroll
      for (int i = 0; i < 6; ++i) res[f][i] = 0.0;
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const double tk = kZt[k], bk = kZb[k];
        const double yx = tk * (y[1] - y[0]) + bk * (y[4] - y[3]);
        const double ye = tk * (y[2] - y[0]) + bk * (y[5] - y[3]);
#pragma unroll
        for (int n = 0; n < 3; ++n) {
          const double gz = 0.5 * (G[k][sidx(n, 0)] * d0 + G[k][sidx(n, 1)] * d1 + G[k][sidx(n, 2)] * d2);
          const double s = hx[k][n] * yx + he[k][n] * ye + gz;
          res[f][n] += tk * s;
          res[f][n + 3] += bk * s;
        }
      }
    }
  }

  // ---- lateral faces: -K+ (y_q - y_nbr) ----
  // the three faces' neighbour slots and metadata first, so that each face's
  // loads below do not wait on its own metadata
  int nslots[3], metas[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    nslots[e] = *reinterpret_cast<const int*>(reinterpret_cast<const char*>(m.nbr_slot + e * CS) + co4);
    metas[e] = *reinterpret_cast<const int*>(reinterpret_cast<const char*>(m.nbr_meta + e * CS) + co4);
  }
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const int A = e, B = (e + 1) % 3;
    const int nslot = nslots[e];
    const int meta = metas[e];
    const bool interior = nslot >= 0;
    if (interior && l >= (meta >> 2)) continue;  // wall
    const double nx = ld(geo + (G_NX + e) * CS, co), ny = ld(geo + (G_NY + e) * CS, co);
    const double Le = ld(geo + (G_LE + e) * CS, co);
    const int oi[4] = {A, B, A + 3, B + 3};      // the face's own nodes
    double un[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) un[n] = nx * u[oi[n]] + ny * v[oi[n]];
    uint32_t no[4] = {0, 0, 0, 0};
    if (interior) {
      const int kp = meta & 3;
      const uint32_t nA = (uint32_t)((kp + 1) % 3), nB = (uint32_t)kp;
      const uint32_t pno = ((uint32_t)nslot + (uint32_t)l * kCell) * 8u;
      no[0] = nA * rs + pno;
      no[1] = nB * rs + pno;
      no[2] = no[0] + 3u * rs;
      no[3] = no[1] + 3u * rs;
#pragma unroll
      for (int n = 0; n < 4; ++n) un[n] = 0.5 * (un[n] + nx * ld(U, no[n]) + ny * ld(U + 6 * S, no[n]));
    }
    double gp[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double s = kS[j], s1 = 1.0 - kS[j];
      const double dS = kSw[j] * Le * 0.5 * (s1 * dz[A] + s * dz[B]);
      double qp[2];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const double q = (s1 * (kZt[k] * un[0] + kZb[k] * un[2]) + s * (kZt[k] * un[1] + kZb[k] * un[3])) * dS;
        qp[k] = upos(q);
      }
      gp[j][0] = kZt[0] * kZt[0] * qp[0] + kZt[1] * kZt[1] * qp[1];
      gp[j][1] = kZt[0] * kZb[0] * qp[0] + kZt[1] * kZb[1] * qp[1];
      gp[j][2] = kZb[0] * kZb[0] * qp[0] + kZb[1] * kZb[1] * qp[1];
    }
    double Kp[3][3];
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
      for (int y = 0; y < 3; ++y) {
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const double sj = kS[j], s1j = 1.0 - kS[j];
          acc += (x == 0 ? s1j * s1j : (x == 1 ? s1j * sj : sj * sj)) * gp[j][y];
        }
        Kp[x][y] = acc;
      }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const double* fb = Y + (size_t)(f * 6) * S;
      double d[4];
#pragma unroll
      for (int n = 0; n < 4; ++n) d[n] = yv[f][oi[n]] - (interior ? ld(fb, no[n]) : 0.0);
      res[f][A] -= Kp[0][0] * d[0] + Kp[1][0] * d[1] + Kp[0][1] * d[2] + Kp[1][1] * d[3];
      res[f][B] -= Kp[1][0] * d[0] + Kp[2][0] * d[1] + Kp[1][1] * d[2] + Kp[2][1] * d[3];
      res[f][A + 3] -= Kp[0][1] * d[0] + Kp[1][1] * d[1] + Kp[0][2] * d[2] + Kp[1][2] * d[3];
      res[f][B + 3] -= Kp[1][1] * d[0] + Kp[2][1] * d[1] + Kp[1][2] * d[2] + Kp[2][2] * d[3];
    }
  }

  // ---- top and bottom faces ----
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int o = side == 0 ? 0 : 3;
    const int oo = side == 0 ? 3 : 0;
    const bool has_nb = side == 0 ? (l > 0) : (l < N - 1);
    const uint32_t pno = has_nb ? (side == 0 ? p - kCell : p + kCell) * 8u : po;
    const double* zf = side == 0 ? zt : zb;
    const double zxi = zf[1] - zf[0], zet = zf[2] - zf[0];
    const double jzx = zxi * yet - zet * yxi;
    const double jzy = zet * xxi - zxi * xet;
    const double sg = side == 0 ? 1.0 : -1.0;
    double un[3];
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      double val = -(u[o + n] * jzx + v[o + n] * jzy);
      if (!WZ) val += Jh * w[o + n];
      un[n] = val;
    }
    if (has_nb) {
#pragma unroll
      for (int n = 0; n < 3; ++n) {
        const size_t ro = (size_t)(oo + n) * S;
        double val = -(ld(U + ro, pno) * jzx + ld(U + 6 * S + ro, pno) * jzy);
        if (!WZ) val += Jh * ld(U + 12 * S + ro, pno);
        un[n] = 0.5 * (un[n] + val);
      }
    }
    double Kp[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const double fq = sg * kTw[q] * (kL0[q] * un[0] + kL1[q] * un[1] + kL2[q] * un[2]);
      const double qp = upos(fq);
      Kp[0] += kL0[q] * kL0[q] * qp;
      Kp[1] += kL1[q] * kL1[q] * qp;
      Kp[2] += kL2[q] * kL2[q] * qp;
      Kp[3] += kL0[q] * kL1[q] * qp;
      Kp[4] += kL0[q] * kL2[q] * qp;
      Kp[5] += kL1[q] * kL2[q] * qp;
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      double d[3];
#pragma unroll
      for (int n = 0; n < 3; ++n)
        d[n] = yv[f][o + n] - (has_nb ? ld(Y + (size_t)(f * 6 + oo + n) * S, pno) : 0.0);
      res[f][o] -= Kp[0] * d[0] + Kp[3] * d[1] + Kp[4] * d[2];
      res[f][o + 1] -= Kp[3] * d[0] + Kp[1] * d[1] + Kp[5] * d[2];
      res[f][o + 2] -= Kp[4] * d[0] + Kp[5] * d[1] + Kp[2] * d[2];
    }
  }

  // ---- M^-1 and the combination ----
  const double m00 = 3.0 * dz[0] + dz[1] + dz[2];
  const double m11 = dz[0] + 3.0 * dz[1] + dz[2];
  const double m22 = dz[0] + dz[1] + 3.0 * dz[2];
  const double m01 = dz[0] + dz[1] + 0.5 * dz[2];
  const double m02 = dz[0] + dz[2] + 0.5 * dz[1];
  const double m12 = dz[1] + dz[2] + 0.5 * dz[0];
  const double c00 = m11 * m22 - m12 * m12, c01 = m02 * m12 - m01 * m22, c02 = m01 * m12 - m02 * m11;
  const double c11 = m00 * m22 - m02 * m02, c12 = m01 * m02 - m00 * m12, c22 = m00 * m11 - m01 * m01;
  const double sc = 120.0 / (Jh * (m00 * c00 + m01 * c01 + m02 * c02));
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const double ht[3] = {2.0 * res[f][0] - res[f][3], 2.0 * res[f][1] - res[f][4], 2.0 * res[f][2] - res[f][5]};
    const double hb[3] = {2.0 * res[f][3] - res[f][0], 2.0 * res[f][4] - res[f][1], 2.0 * res[f][5] - res[f][2]};
    double L[6];
    L[0] = sc * (c00 * ht[0] + c01 * ht[1] + c02 * ht[2]);
    L[1] = sc * (c01 * ht[0] + c11 * ht[1] + c12 * ht[2]);
    L[2] = sc * (c02 * ht[0] + c12 * ht[1] + c22 * ht[2]);
    L[3] = sc * (c00 * hb[0] + c01 * hb[1] + c02 * hb[2]);
    L[4] = sc * (c01 * hb[0] + c11 * hb[1] + c12 * hb[2]);
    L[5] = sc * (c02 * hb[0] + c12 * hb[1] + c22 * hb[2]);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      const size_t row = (size_t)(f * 6 + i) * S;
      double o = a.b * (yv[f][i] + a.dt * L[i]);
      if (a.X1) o += a.a1 * ld(a.X1 + row, po);
      if (a.X2) o += a.a2 * ld(a.X2 + row, po);
      st(a.out + row, po, o);
    }
  }
}

// ---------------------------------------------------------------------------
// Per-prism geometry shared by the transposed solve and the kappa gradient
// ---------------------------------------------------------------------------
struct LayerGeo {
  double dz[3];
  double hbar;
};

__device__ __forceinline__ void load_layer(const DevMesh& m, size_t lt, LayerGeo& g) {
  const size_t LS = (size_t)m.n_lslots;
#pragma unroll
  for (int v = 0; v < 3; ++v) g.dz[v] = m.zl[v * LS + lt] - m.zl[v * LS + lt + kCell];
  g.hbar = (g.dz[0] + g.dz[1] + g.dz[2]) * (1.0 / 3.0);
}

__device__ __forceinline__ void vertical_stiffness(const LayerGeo& g, double Jh, double kv[6]) {
#pragma unroll
  for (int i = 0; i < 6; ++i) kv[i] = 0.0;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const double l0 = kL0[q], l1 = kL1[q], l2 = kL2[q];
    const double inv = kTw[q] / (l0 * g.dz[0] + l1 * g.dz[1] + l2 * g.dz[2]);
    kv[0] += l0 * l0 * inv;
    kv[1] += l1 * l1 * inv;
    kv[2] += l2 * l2 * inv;
    kv[3] += l0 * l1 * inv;
    kv[4] += l0 * l2 * inv;
    kv[5] += l1 * l2 * inv;
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) kv[i] *= Jh;
}

__device__ __forceinline__ void mass_z(const LayerGeo& g, double Jh, double mz[6]) {
  const double s = Jh * (1.0 / 120.0);
  const double* dz = g.dz;
  mz[0] = s * (3.0 * dz[0] + dz[1] + dz[2]);
  mz[1] = s * (dz[0] + 3.0 * dz[1] + dz[2]);
  mz[2] = s * (dz[0] + dz[1] + 3.0 * dz[2]);
  mz[3] = s * (dz[0] + dz[1] + 0.5 * dz[2]);
  mz[4] = s * (dz[0] + dz[2] + 0.5 * dz[1]);
  mz[5] = s * (dz[1] + dz[2] + 0.5 * dz[0]);
}

__device__ __forceinline__ double penalty(double eta, double ka, double kb, double ha, double hb) {
  return eta * 0.5 * (ka + kb) / fmin(ha, hb);
}

// ---------------------------------------------------------------------------
// Transposed column solve: (M - dt A^T) mu = M Z
// ---------------------------------------------------------------------------
// The transposed column matrix has diagonal blocks D_l^T = [TT BT; TB BB]
// (the 3x3 sub-blocks of D_l are symmetric), the block left of the diagonal
// Lo_l = C_{l-1}^T (only columns of the bottom nodes of l-1 nonzero) and the
// block right of it Up_l = B_{l+1}^T (only columns of the top nodes of l+1):
//   Lo_l = dt [kappa_l Kv_l/2 - sig_u S ; -kappa_l Kv_l/2]          (6 x 3)
//   Up_l = dt [-kappa_l Kv_l/2 ; kappa_l Kv_l/2 - sig_d S]          (6 x 3)
// Block Thomas: D'_l = D_l^T - Lo_l G_{l-1}[3:6, :] (columns 0..2 only),
// G_l = D'_l^-1 Up_l and y_l = D'_l^-1 (r_l - Lo_l y_{l-1}[3:6]); back
// substitution mu_l = y_l - G_l mu_{l+1}[0:3].  As in the forward solve, G_l
// depends only on the mesh, kappa, dt and the penalty: a sweep without fields
// (NF = 0) keeps it in its own array, each solve's forward sweep recomputes it
// in registers and stores y_l into the output rows, and the back
// substitution reads the kept G_l and overwrites y_l with mu_l.
struct TSolveArgs {
  DevMesh m;
  const double* Z;     // may be the same array as mu
  double* mu;
  const double* kappa;
  double* gfac;        // [18][n_slots]: the kept G_l
  double dt, eta;
};

template <int NF>
__global__ __launch_bounds__(64) void tsolve_kernel(TSolveArgs a) {
  constexpr int kF = NF > 0 ? NF : 1;   // array extent (the factor sweep has no fields)
  const DevMesh& m = a.m;
  const int cell = m.cell_order[blockIdx.x];   // deepest cells first
  const int lane = threadIdx.x;
  const int c = cell * kCell + lane;
  const int N = m.nlay[c];
  if (N == 0) return;
  const size_t SL = (size_t)m.n_slots;
  const size_t p0 = (size_t)m.cell_base[cell] + lane;
  const size_t lt0 = (size_t)m.cell_lbase[cell] + lane;
  const double Jh = m.geo[G_JH * m.n_col_slots + c];
  const double dt = a.dt, eta = a.eta;
  const double* __restrict__ kap = a.kappa;
  double* __restrict__ Gsc = a.gfac;
  const double sd = Jh * (1.0 / 12.0), so = Jh * (1.0 / 24.0);

  // Each layer's loads are issued one layer ahead of their use (the next
  // layer's Z and the geometry two layers down), so that a column's serial
  // sweep does not wait a memory round trip per layer.
  LayerGeo gc, gn, gp;
  load_layer(m, lt0, gc);
  double kvc[6];
  vertical_stiffness(gc, Jh, kvc);
  double Gp[6][3];
  double yp[kF][6];
  double kp = 0.0;
  gp = gc;
  double zc[kF][6];
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int i = 0; i < 6; ++i) zc[f][i] = a.Z[(size_t)(f * 6 + i) * SL + p0];
  double kn = 0.0;
  if (N > 1) {
    load_layer(m, lt0 + (size_t)kCell, gn);
    kn = kap[1];
  }
  for (int l = 0; l < N; ++l) {
    const size_t p = p0 + (size_t)l * kCell;
    const double kc = kap[l];
    const bool below = l < N - 1;
    double zx[kF][6];
    if (below) {
#pragma unroll
      for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int i = 0; i < 6; ++i) zx[f][i] = a.Z[(size_t)(f * 6 + i) * SL + p + kCell];
    }
    LayerGeo gnn = gn;
    double knn = 0.0;
    if (l + 2 < N) {
      load_layer(m, lt0 + (size_t)(l + 2) * kCell, gnn);
      knn = kap[l + 2];
    }
    double mz[6];
    mass_z(gc, Jh, mz);
    const double sig_u = l > 0 ? penalty(eta, kp, kc, gp.hbar, gc.hbar) : 0.0;
    const double sig_d = below ? penalty(eta, kc, kn, gc.hbar, gn.hbar) : 0.0;
    // forward sub-blocks TT, TB, BT, BB of D_l, then D_l^T = [TT BT; TB BB]
    double d[6][6];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double mm = mz[sidx(i, j)], kk = dt * kc * kvc[sidx(i, j)], hk = 0.5 * kk;
        const double s_ij = (i == j ? sd : so);
        double TT = (2.0 / 3.0) * mm + kk, TB = (1.0 / 3.0) * mm - kk;
        double BT = (1.0 / 3.0) * mm - kk, BB = (2.0 / 3.0) * mm + kk;
        if (l > 0) {
          TT += -hk + dt * sig_u * s_ij;
          TB += hk;
        }
        if (below) {
          BT += hk;
          BB += -hk + dt * sig_d * s_ij;
        }
        d[i][j] = TT;
        d[i][j + 3] = BT;
        d[i + 3][j] = TB;
        d[i + 3][j + 3] = BB;
      }
    // right-hand sides r = M Z
    double r[kF][6];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const double* t = zc[f];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        double at = 0.0, ab = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          at += mz[sidx(i, j)] * t[j];
          ab += mz[sidx(i, j)] * t[j + 3];
        }
        r[f][i] = (2.0 / 3.0) * at + (1.0 / 3.0) * ab;
        r[f][i + 3] = (1.0 / 3.0) * at + (2.0 / 3.0) * ab;
      }
    }
    if (l > 0) {
      double Lo[6][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const double hk = 0.5 * dt * kc * kvc[sidx(i, j)];
          Lo[i][j] = hk - dt * sig_u * (i == j ? sd : so);
          Lo[i + 3][j] = -hk;
        }
#pragma unroll
      for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          double acc = 0.0;
#pragma unroll
          for (int k = 0; k < 3; ++k) acc += Lo[i][k] * Gp[k + 3][j];
          d[i][j] -= acc;
        }
#pragma unroll
      for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int i = 0; i < 6; ++i) {
          double acc = 0.0;
#pragma unroll
          for (int k = 0; k < 3; ++k) acc += Lo[i][k] * yp[f][k + 3];
          r[f][i] -= acc;
        }
    }
    // LU of d without pivoting
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const double inv = 1.0 / d[k][k];
#pragma unroll
      for (int i = k + 1; i < 6; ++i) {
        const double li = d[i][k] * inv;
        d[i][k] = li;
#pragma unroll
        for (int j = k + 1; j < 6; ++j) d[i][j] -= li * d[k][j];
      }
    }
    // G = d^-1 Up (only needed when there is a layer below)
    double Gc[6][3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      double z[6];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        double hk = 0.5 * dt * kc * kvc[sidx(i, q)];
        z[i] = below ? -hk : 0.0;
        z[i + 3] = below ? hk - dt * sig_d * (i == q ? sd : so) : 0.0;
      }
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        double acc = z[i];
#pragma unroll
        for (int k = 0; k < i; ++k) acc -= d[i][k] * z[k];
        z[i] = acc;
      }
#pragma unroll
      for (int i = 5; i >= 0; --i) {
        double acc = z[i];
#pragma unroll
        for (int k = i + 1; k < 6; ++k) acc -= d[i][k] * z[k];
        z[i] = acc / d[i][i];
      }
#pragma unroll
      for (int i = 0; i < 6; ++i) Gc[i][q] = z[i];
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      double z[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        double acc = r[f][i];
#pragma unroll
        for (int k = 0; k < i; ++k) acc -= d[i][k] * z[k];
        z[i] = acc;
      }
#pragma unroll
      for (int i = 5; i >= 0; --i) {
        double acc = z[i];
#pragma unroll
        for (int k = i + 1; k < 6; ++k) acc -= d[i][k] * z[k];
        z[i] = acc / d[i][i];
      }
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        yp[f][i] = z[i];
        a.mu[(size_t)(f * 6 + i) * SL + p] = z[i];   // Z_l has been read: y_l may overwrite it
      }
    }
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        Gp[i][q] = Gc[i][q];
        if (NF == 0) Gsc[(size_t)(i * 3 + q) * SL + p] = Gc[i][q];
      }
    kp = kc;
    gp = gc;
    if (below) {
      gc = gn;
      vertical_stiffness(gc, Jh, kvc);
#pragma unroll
      for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int i = 0; i < 6; ++i) zc[f][i] = zx[f][i];
    }
    gn = gnn;
    kn = knn;
  }
  if (NF == 0) return;
  // back substitution
  double xn[kF][6];
  {
    const size_t p = p0 + (size_t)(N - 1) * kCell;
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        xn[f][i] = yp[f][i];
        a.mu[(size_t)(f * 6 + i) * SL + p] = yp[f][i];
      }
  }
  // G_l and y_l one layer ahead of their use, as in the forward sweep
  double G[6][3], yl[kF][6];
  if (N > 1) {
    const size_t p = p0 + (size_t)(N - 2) * kCell;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int q = 0; q < 3; ++q) G[i][q] = Gsc[(size_t)(i * 3 + q) * SL + p];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int i = 0; i < 6; ++i) yl[f][i] = a.mu[(size_t)(f * 6 + i) * SL + p];
  }
  for (int l = N - 2; l >= 0; --l) {
    const size_t p = p0 + (size_t)l * kCell;
    double Gx[6][3], yx[kF][6];
    if (l > 0) {
#pragma unroll
      for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int q = 0; q < 3; ++q) Gx[i][q] = Gsc[(size_t)(i * 3 + q) * SL + p - kCell];
#pragma unroll
      for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int i = 0; i < 6; ++i) yx[f][i] = a.mu[(size_t)(f * 6 + i) * SL + p - kCell];
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      double xt[3] = {xn[f][0], xn[f][1], xn[f][2]};
#pragma unroll
      for (int i = 0; i < 6; ++i)
        xn[f][i] = yl[f][i] - (G[i][0] * xt[0] + G[i][1] * xt[1] + G[i][2] * xt[2]);
#pragma unroll
      for (int i = 0; i < 6; ++i) a.mu[(size_t)(f * 6 + i) * SL + p] = xn[f][i];
    }
    if (l > 0) {
#pragma unroll
      for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int q = 0; q < 3; ++q) G[i][q] = Gx[i][q];
#pragma unroll
      for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int i = 0; i < 6; ++i) yl[f][i] = yx[f][i];
    }
  }
}

// ---------------------------------------------------------------------------
// kappa gradient: g_l = sum_f mu_f^T (dA/dkappa_l) x_f per column and layer.
// A depends on kappa_l through the volume term of prism l and, on the faces
// above and below it, through {kappa dT/dz} (kappa/2 per side) and the
// penalty (d sigma / d kappa = s' = eta / (2 min(hbar_up, hbar_dn))).  With
// [v] = v_up,bottom - v_dn,top across a face and S = M_h:
//   volume of l:                -(mu_t - mu_b)^T Kv_l (x_t - x_b)
//   each face touching l:       -[mu]^T (s' S [x] + Kv_l (x_l,t - x_l,b) / 2)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double quad3(const double K[6], const double a[3], const double b[3]) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) s += a[i] * K[sidx(i, j)] * b[j];
  return s;
}

__device__ __forceinline__ double quadS(double sd, double so, const double a[3], const double b[3]) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) s += a[i] * (i == j ? sd : so) * b[j];
  return s;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// One thread per prism over the 2-layer tile table, one wavefront per layer
// of a cell: each prism evaluates every term of its own g (its volume and
// both faces touching it; the penalty of a face is evaluated by the prisms on
// both sides), so no column is walked and the loads of all layers are in
// flight at once.  The 64 columns of a cell are summed with a fixed
// butterfly, cells per layer with a fixed tree (kgrad_reduce_kernel).
struct KGradTileArgs {
  DevMesh m;
  const WgTile* tiles;
  const double* mu;
  const double* x;
  double* partial;   // [max_layers][n_cells]
  double eta;
};

template <int NF>
__global__ __launch_bounds__(128) void kgrad_tile_kernel(KGradTileArgs a) {
  const DevMesh& m = a.m;
  const WgTile tile = a.tiles[blockIdx.x];
  const int lane = threadIdx.x & (kCell - 1);
  const int l = tile.layer0 + (threadIdx.x >> 6);
  const int cell = tile.cell;
  const int depth = (m.cell_base[cell + 1] - m.cell_base[cell]) / kCell;
  if (l >= depth) return;                      // uniform per wavefront
  const int c = cell * kCell + lane;
  const int N = m.nlay[c];
  const bool live = l < N;
  const bool up = live && l > 0, dn = live && l + 1 < N;
  const size_t SL = (size_t)m.n_slots;
  const size_t p = (size_t)m.cell_base[cell] + (size_t)l * kCell + lane;
  const size_t pu = up ? p - kCell : p, pd = dn ? p + kCell : p;
  const size_t lt = (size_t)m.cell_lbase[cell] + (size_t)l * kCell + lane;
  double g = 0.0;
  if (live) {
    const double Jh = m.geo[G_JH * m.n_col_slots + c];
    const double sd = Jh * (1.0 / 12.0), so = Jh * (1.0 / 24.0);
    LayerGeo gl, gu, gd;
    load_layer(m, lt, gl);
    load_layer(m, up ? lt - kCell : lt, gu);
    load_layer(m, dn ? lt + kCell : lt, gd);
    double kv[6];
    vertical_stiffness(gl, Jh, kv);
    const double spu = up ? a.eta / (2.0 * fmin(gu.hbar, gl.hbar)) : 0.0;
    const double spd = dn ? a.eta / (2.0 * fmin(gl.hbar, gd.hbar)) : 0.0;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      double mt[3], mb[3], xt[3], xb[3], dm[3], dx[3];
      double mub[3], xub[3], mdt[3], xdt[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const size_t rt = (size_t)(f * 6 + i) * SL, rb = (size_t)(f * 6 + i + 3) * SL;
        mt[i] = a.mu[rt + p];
        mb[i] = a.mu[rb + p];
        xt[i] = a.x[rt + p];
        xb[i] = a.x[rb + p];
        mub[i] = a.mu[rb + pu];
        xub[i] = a.x[rb + pu];
        mdt[i] = a.mu[rt + pd];
        xdt[i] = a.x[rt + pd];
        dm[i] = mt[i] - mb[i];
        dx[i] = xt[i] - xb[i];
      }
      g -= quad3(kv, dm, dx);
      if (up) {                                 // the face above: kappa_l below it
        double jm[3], jx[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          jm[i] = mub[i] - mt[i];
          jx[i] = xub[i] - xt[i];
        }
        g -= quadS(spu * sd, spu * so, jm, jx) + 0.5 * quad3(kv, jm, dx);
      }
      if (dn) {                                 // the face below: kappa_l above it
        double jm[3], jx[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          jm[i] = mb[i] - mdt[i];
          jx[i] = xb[i] - xdt[i];
        }
        g -= quadS(spd * sd, spd * so, jm, jx) + 0.5 * quad3(kv, jm, dx);
      }
    }
  }
  const double v = wave_sum(g);
  if (lane == 0) a.partial[(size_t)l * m.n_cells + cell] = v;
}

// dkappa[l] += dt * sum over cells deeper than l of partial[l][cell]
__global__ __launch_bounds__(256) void kgrad_reduce_kernel(DevMesh m, const double* partial, double dt,
                                                            double* dkappa) {
  const int l = blockIdx.x;
  __shared__ double red[256];
  double acc = 0.0;
  for (int k = threadIdx.x; k < m.n_cells; k += 256) {
    const int depth = (m.cell_base[k + 1] - m.cell_base[k]) / kCell;
    if (l < depth) acc += partial[(size_t)l * m.n_cells + k];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) dkappa[l] += dt * red[0];
}

// ---------------------------------------------------------------------------
// Mass operator: Y = M X or M^-1 X per prism; column partials of X^T M Y.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(64) void mass_apply_kernel(DevMesh m, const R* X, R* Y, int nf, int inverse) {
  const int cell = blockIdx.x;
  const int lane = threadIdx.x;
  const int c = cell * kCell + lane;
  const int N = m.nlay[c];
  if (N == 0) return;
  const size_t SL = (size_t)m.n_slots;
  const double Jh = m.geo[G_JH * m.n_col_slots + c];
  for (int l = 0; l < N; ++l) {
    const size_t p = (size_t)m.cell_base[cell] + (size_t)l * kCell + lane;
    LayerGeo g;
    load_layer(m, (size_t)m.cell_lbase[cell] + (size_t)l * kCell + lane, g);
    double mz[6];
    mass_z(g, Jh, mz);
    double inv[6];
    if (inverse) {
      const double c00 = mz[1] * mz[2] - mz[5] * mz[5], c01 = mz[4] * mz[5] - mz[3] * mz[2];
      const double c02 = mz[3] * mz[5] - mz[4] * mz[1], c11 = mz[0] * mz[2] - mz[4] * mz[4];
      const double c12 = mz[3] * mz[4] - mz[0] * mz[5], c22 = mz[0] * mz[1] - mz[3] * mz[3];
      const double det = mz[0] * c00 + mz[3] * c01 + mz[4] * c02;
      inv[0] = c00 / det; inv[1] = c11 / det; inv[2] = c22 / det;
      inv[3] = c01 / det; inv[4] = c02 / det; inv[5] = c12 / det;
    }
    for (int f = 0; f < nf; ++f) {
      double t[6], o[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) t[i] = (double)X[(size_t)(f * 6 + i) * SL + p];
      // M = [2 1; 1 2]/3 (x) Mz, M^-1 = [2 -1; -1 2] (x) Mz^-1
      double ht[3], hb[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        ht[i] = inverse ? 2.0 * t[i] - t[i + 3] : (2.0 * t[i] + t[i + 3]) * (1.0 / 3.0);
        hb[i] = inverse ? 2.0 * t[i + 3] - t[i] : (t[i] + 2.0 * t[i + 3]) * (1.0 / 3.0);
      }
      const double* K = inverse ? inv : mz;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        o[i] = K[sidx(i, 0)] * ht[0] + K[sidx(i, 1)] * ht[1] + K[sidx(i, 2)] * ht[2];
        o[i + 3] = K[sidx(i, 0)] * hb[0] + K[sidx(i, 1)] * hb[1] + K[sidx(i, 2)] * hb[2];
      }
#pragma unroll
      for (int i = 0; i < 6; ++i) Y[(size_t)(f * 6 + i) * SL + p] = (R)o[i];
    }
  }
}

template <typename R>
__global__ __launch_bounds__(64) void mdot_column_kernel(DevMesh m, const R* X, const R* Y, int nf, double* out) {
  const int cell = blockIdx.x;
  const int lane = threadIdx.x;
  const int c = cell * kCell + lane;
  const int N = m.nlay[c];
  const int CS = m.n_col_slots;
  const size_t SL = (size_t)m.n_slots;
  double acc[kMaxFields] = {0.0, 0.0, 0.0, 0.0};
  if (N > 0) {
    const double Jh = m.geo[G_JH * CS + c];
    for (int l = 0; l < N; ++l) {
      const size_t p = (size_t)m.cell_base[cell] + (size_t)l * kCell + lane;
      LayerGeo g;
      load_layer(m, (size_t)m.cell_lbase[cell] + (size_t)l * kCell + lane, g);
      double mz[6];
      mass_z(g, Jh, mz);
      for (int f = 0; f < nf; ++f) {
        double x[6], y[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) {
          x[i] = (double)X[(size_t)(f * 6 + i) * SL + p];
          y[i] = (double)Y[(size_t)(f * 6 + i) * SL + p];
        }
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            const double mm = mz[sidx(i, j)];
            s += mm * ((2.0 / 3.0) * (x[i] * y[j] + x[i + 3] * y[j + 3]) +
                       (1.0 / 3.0) * (x[i] * y[j + 3] + x[i + 3] * y[j]));
          }
        acc[f] += s;
      }
    }
  }
  for (int f = 0; f < nf; ++f) out[(size_t)f * CS + c] = acc[f];
}

template <int NF>
hipError_t launch_adj_stage_nf(const AdjStageArgs& a, bool w_zero, int tile_layers, hipStream_t s) {
  dim3 grid(a.n_tiles), block(kCell * tile_layers);
  if (w_zero) hipLaunchKernelGGL((adj_stage_kernel<NF, true>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((adj_stage_kernel<NF, false>), grid, block, 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_adjoint_stage(const DevMesh& m, const WgTile* tiles, int n_tiles, int tile_layers, int xcd,
                                int n_fields, bool w_zero, const double* Y, const double* X1, const double* X2,
                                double* out, const double* U, double dt, double b, double a1, double a2,
                                hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  AdjStageArgs a{};
  a.m = m;
  a.tiles = tiles;
  a.n_tiles = n_tiles;
  a.xcd = xcd;
  a.Y = Y;
  a.X1 = X1;
  a.X2 = X2;
  a.out = out;
  a.U = U;
  a.dt = dt;
  a.b = b;
  a.a1 = a1;
  a.a2 = a2;
  switch (n_fields) {
    case 1: return launch_adj_stage_nf<1>(a, w_zero, tile_layers, s);
    case 2: return launch_adj_stage_nf<2>(a, w_zero, tile_layers, s);
    case 3: return launch_adj_stage_nf<3>(a, w_zero, tile_layers, s);
    case 4: return launch_adj_stage_nf<4>(a, w_zero, tile_layers, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_tsolve(const DevMesh& m, int n_fields, const double* Z, double* mu, const double* kappa,
                         double* gfac, double dt, double eta, bool factor, hipStream_t s) {
  if (m.n_cells == 0) return hipSuccess;
  TSolveArgs a{};
  a.m = m;
  a.Z = Z;
  a.mu = mu;
  a.kappa = kappa;
  a.gfac = gfac;
  a.dt = dt;
  a.eta = eta;
  dim3 grid(m.n_cells), block(kCell);
  if (factor) {
    hipLaunchKernelGGL((tsolve_kernel<0>), grid, block, 0, s, a);
    return hipGetLastError();
  }
  switch (n_fields) {
    case 1: hipLaunchKernelGGL((tsolve_kernel<1>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((tsolve_kernel<2>), grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL((tsolve_kernel<3>), grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL((tsolve_kernel<4>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_kappa_gradient(const DevMesh& m, const WgTile* tiles2, int n_tiles2, int n_fields,
                                 const double* mu, const double* x, double* partial, double eta, double dt,
                                 double* dkappa, hipStream_t s) {
  if (m.n_cells == 0) return hipSuccess;
  KGradTileArgs a{};
  a.m = m;
  a.tiles = tiles2;
  a.mu = mu;
  a.x = x;
  a.partial = partial;
  a.eta = eta;
  const dim3 grid(n_tiles2), block(2 * kCell);
  switch (n_fields) {
    case 1: hipLaunchKernelGGL((kgrad_tile_kernel<1>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((kgrad_tile_kernel<2>), grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL((kgrad_tile_kernel<3>), grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL((kgrad_tile_kernel<4>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kgrad_reduce_kernel, dim3(m.max_layers), dim3(256), 0, s, m, partial, dt, dkappa);
  return hipGetLastError();
}

hipError_t launch_mass_apply(const DevMesh& m, const void* X, void* Y, int n_fields, bool fp32, bool inverse,
                             hipStream_t s) {
  if (fp32)
    hipLaunchKernelGGL(mass_apply_kernel<float>, dim3(m.n_cells), dim3(kCell), 0, s, m,
                       static_cast<const float*>(X), static_cast<float*>(Y), n_fields, (int)inverse);
  else
    hipLaunchKernelGGL(mass_apply_kernel<double>, dim3(m.n_cells), dim3(kCell), 0, s, m,
                       static_cast<const double*>(X), static_cast<double*>(Y), n_fields, (int)inverse);
  return hipGetLastError();
}

hipError_t launch_mdot_columns(const DevMesh& m, const void* X, const void* Y, int n_fields, bool fp32,
                               double* col_out, hipStream_t s) {
  if (fp32)
    hipLaunchKernelGGL(mdot_column_kernel<float>, dim3(m.n_cells), dim3(kCell), 0, s, m,
                       static_cast<const float*>(X), static_cast<const float*>(Y), n_fields, col_out);
  else
    hipLaunchKernelGGL(mdot_column_kernel<double>, dim3(m.n_cells), dim3(kCell), 0, s, m,
                       static_cast<const double*>(X), static_cast<const double*>(Y), n_fields, col_out);
  return hipGetLastError();
}

}  // namespace sdg
