// Explicit DG operator and SSP-RK3 stage on extruded linear prisms.
//
// Per prism and field:
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
//
// Two kernels compute the same arithmetic (bitwise: they share every device
// function below and accumulate in the same order):
//
//  * stage_kernel: one thread per prism; a workgroup covers 1, 2 or 4 layers
//    of one cell of 64 columns (one wavefront per layer), so each wavefront
//    reads 64 consecutive slots of every nodal array (the paper's section
//    2.1.1 cell layout, with wavefront-sized cells).  No load depends on
//    control flow: lanes past their column's depth compute on in-bounds
//    padding slots and skip the store, and faces without a neighbour address
//    the prism's own nodes and select the exterior value.
//
//  * walk_kernel: one wavefront walks down a segment of a cell's layers.
//    The next layer's stage input, velocity, bottom level heights (and Tn,
//    where it fits) are copied global -> LDS by the wavefront's own 16-byte
//    direct loads while the current layer computes, so the HBM latency of
//    the streamed data is hidden by the pipeline rather than by occupancy,
//    and the loads take no registers.  The horizontal face between layers l
//    and l+1 is computed once and its contribution to layer l+1's top nodes
//    carried in registers.  Lateral neighbours are read from L2.
#include <atomic>

#include "internal.h"

// Multiply-adds are fused only within one expression, never across
// statements, so the shared device functions below round the same way in
// both kernels whatever the surrounding code.
#pragma clang fp contract(on)

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
// Row r of a [..][6][S] nodal array at byte offset off.  In double the
// address is the base of the row's 6-row block plus a 32-bit offset
// (r mod 6) S + off: one uniform base per block instead of one per row, so
// the FP64 column walk keeps far fewer 64-bit row addresses in scalar
// registers, which it otherwise spills to vector lanes (stages 2% faster).
// In float the per-row form stays: the block form's offsets take the few
// vector registers that keep the float walk at two wavefronts per SIMD.
// A 6-row block is below 4 GiB (checked at mesh upload).
template <typename T>
__device__ __forceinline__ T ldr(const T* __restrict__ arr, size_t S, int r, uint32_t off) {
  if constexpr (sizeof(T) == 8)
    return ldb(arr + (size_t)(r / 6 * 6) * S, (uint32_t)(r % 6) * (uint32_t)(S * sizeof(T)) + off);
  else
    return ldb(arr + (size_t)r * S, off);
}
template <typename T>
__device__ __forceinline__ void str(T* __restrict__ arr, size_t S, int r, uint32_t off, T v) {
  if constexpr (sizeof(T) == 8)
    stb(arr + (size_t)(r / 6 * 6) * S, (uint32_t)(r % 6) * (uint32_t)(S * sizeof(T)) + off, v);
  else
    stb(arr + (size_t)r * S, off, v);
}

template <typename R>
__device__ __forceinline__ R upos(R x) { return x > R(0) ? x : R(0); }
template <typename R>
__device__ __forceinline__ R uneg(R x) { return x < R(0) ? x : R(0); }

// Per-column map derivatives and J_h = 2 area.
template <typename R>
struct ColGeo {
  R xxi, xet, yxi, yet, Jh;
};

template <typename R>
__device__ __forceinline__ ColGeo<R> load_colgeo(const DevMesh& m, uint32_t co) {
  const R* __restrict__ geo = geo_of<R>(m);
  const int CS = m.n_col_slots;
  ColGeo<R> g;
  g.xxi = ldb(geo + G_XXI * CS, co);
  g.xet = ldb(geo + G_XET * CS, co);
  g.yxi = ldb(geo + G_YXI * CS, co);
  g.yet = ldb(geo + G_YET * CS, co);
  g.Jh = ldb(geo + G_JH * CS, co);
  return g;
}

// ===========================================================================
// Per-prism factors (field independent), then one field at a time.
//
// Everything that depends only on geometry and velocity is computed once per
// prism: the volume flux factors at the 12 volume points, the upwind weights
// of the lateral and horizontal faces, and the cofactors of Mz.  Each field
// then needs only its own nodal values and its neighbours' traces, so the
// values live at any time are the factors plus one field's working set.
// ===========================================================================

// No instruction moves across this point.
__device__ __forceinline__ void phase() { __builtin_amdgcn_sched_barrier(0); }

// Volume term factors: with alpha = y_eta u - x_eta v, beta = x_xi v - y_xi u
// at volume point (k, q):
//   Vx = w_q z_zeta alpha, Ve = w_q z_zeta beta,
//   Vz = w_q (J_h w - z_xi alpha - z_eta beta).
// The field's value at the point is sum_a lambda_a(q) ta_k[a] (ta_k: the
// field at the three nodes interpolated to zeta_k), so the sums over q of
// the same quadrature are contracted once per prism into the field-free
//   Px_k[a] = sum_q lambda_a(q) Vx,  Pe_k[a] = sum_q lambda_a(q) Ve,
//   G_k[n][a] = sum_q lambda_n(q) lambda_a(q) Vz   (symmetric),
// and each field only takes ta_k . Px_k, ta_k . Pe_k and G_k ta_k
// (42 multiply-adds a field instead of 108, and 24 values kept instead of 36).
template <typename R>
struct VolF {
  R Px[2][3], Pe[2][3], G[2][6];   // G: symmetric 3x3, entries 00 11 22 01 02 12
};

template <typename R, bool WZ>
__device__ __forceinline__ void volume_factors(const ColGeo<R>& g, const R zt[3], const R zb[3], const R dz[3],
                                               const R u[6], const R v[6], const R w[6], VolF<R>& F) {
  const R xxi = g.xxi, xet = g.xet, yxi = g.yxi, yet = g.yet, Jh = g.Jh;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const R tk = R(kZt[k]), bk = R(kZb[k]);
    R ua[3], va[3], wa[3];
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      ua[n] = tk * u[n] + bk * u[n + 3];
      va[n] = tk * v[n] + bk * v[n + 3];
      wa[n] = WZ ? R(0) : tk * w[n] + bk * w[n + 3];
    }
    const R z_xi = tk * (zt[1] - zt[0]) + bk * (zb[1] - zb[0]);
    const R z_et = tk * (zt[2] - zt[0]) + bk * (zb[2] - zb[0]);
#pragma unroll
    for (int i = 0; i < 3; ++i) F.Px[k][i] = F.Pe[k][i] = R(0);
#pragma unroll
    for (int i = 0; i < 6; ++i) F.G[k][i] = R(0);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const R l0 = R(kL0[q]), l1 = R(kL1[q]), l2 = R(kL2[q]), wq = R(kTw[q]);
      const R uq = l0 * ua[0] + l1 * ua[1] + l2 * ua[2];
      const R vq = l0 * va[0] + l1 * va[1] + l2 * va[2];
      const R zz = R(0.5) * (l0 * dz[0] + l1 * dz[1] + l2 * dz[2]);
      const R al = yet * uq - xet * vq;
      const R be = xxi * vq - yxi * uq;
      const R vx = wq * zz * al;
      const R ve = wq * zz * be;
      R vz = -(z_xi * al + z_et * be);
      if (!WZ) vz += Jh * (l0 * wa[0] + l1 * wa[1] + l2 * wa[2]);
      vz *= wq;
      F.Px[k][0] += l0 * vx;
      F.Px[k][1] += l1 * vx;
      F.Px[k][2] += l2 * vx;
      F.Pe[k][0] += l0 * ve;
      F.Pe[k][1] += l1 * ve;
      F.Pe[k][2] += l2 * ve;
      F.G[k][0] += R(kL0[q] * kL0[q]) * vz;
      F.G[k][1] += R(kL1[q] * kL1[q]) * vz;
      F.G[k][2] += R(kL2[q] * kL2[q]) * vz;
      F.G[k][3] += R(kL0[q] * kL1[q]) * vz;
      F.G[k][4] += R(kL0[q] * kL2[q]) * vz;
      F.G[k][5] += R(kL1[q] * kL2[q]) * vz;
    }
  }
}

// res[i] = int_K T U.grad(phi_i) dV for one field.
template <typename R>
__device__ __forceinline__ void volume_field(const VolF<R>& F, const R T[6], R res[6]) {
  R sx[2], se[2], sz[3] = {R(0), R(0), R(0)};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const R tk = R(kZt[k]), bk = R(kZb[k]);
    R ta[3];
#pragma unroll
    for (int n = 0; n < 3; ++n) ta[n] = tk * T[n] + bk * T[n + 3];
    sx[k] = ta[0] * F.Px[k][0] + ta[1] * F.Px[k][1] + ta[2] * F.Px[k][2];
    se[k] = ta[0] * F.Pe[k][0] + ta[1] * F.Pe[k][1] + ta[2] * F.Pe[k][2];
    sz[0] += F.G[k][0] * ta[0] + F.G[k][3] * ta[1] + F.G[k][4] * ta[2];
    sz[1] += F.G[k][3] * ta[0] + F.G[k][1] * ta[1] + F.G[k][5] * ta[2];
    sz[2] += F.G[k][4] * ta[0] + F.G[k][5] * ta[1] + F.G[k][2] * ta[2];
  }
  // dphi/dxi = dlambda/dxi * (t or b), dphi/dzeta = +-lambda/2
  const R sxt = R(kZt[0]) * sx[0] + R(kZt[1]) * sx[1];
  const R sxb = R(kZb[0]) * sx[0] + R(kZb[1]) * sx[1];
  const R set = R(kZt[0]) * se[0] + R(kZt[1]) * se[1];
  const R seb = R(kZb[0]) * se[0] + R(kZb[1]) * se[1];
  res[0] = -sxt - set + R(0.5) * sz[0];
  res[1] = sxt + R(0.5) * sz[1];
  res[2] = set + R(0.5) * sz[2];
  res[3] = -sxb - seb - R(0.5) * sz[0];
  res[4] = sxb - R(0.5) * sz[1];
  res[5] = seb - R(0.5) * sz[2];
}

// Lateral face e (edge A = e -> B = e+1) of a column: neighbour slot and
// edge, outward normal and length (the same for every layer).
template <typename R>
struct LatMeta {
  int nslot, meta;
  R nx, ny, Le;
};

template <typename R>
__device__ __forceinline__ void lat_meta(const DevMesh& m, int e, uint32_t co, LatMeta<R>& M) {
  const int CS = m.n_col_slots;
  const uint32_t co4 = co / (uint32_t)sizeof(R) * 4u;
  const R* __restrict__ geo = geo_of<R>(m);
  M.nslot = ldb(m.nbr_slot + e * CS, co4);
  M.meta = ldb(m.nbr_meta + e * CS, co4);
  M.nx = ldb(geo + (G_NX + e) * CS, co);
  M.ny = ldb(geo + (G_NY + e) * CS, co);
  M.Le = ldb(geo + (G_LE + e) * CS, co);
}

// At layer l (prism byte offset po): the byte offsets (within a field block)
// of the neighbour's face nodes A top, B top, A bottom, B bottom, and its
// velocity there.  A wall (neighbour shallower than l) or an open boundary
// has no live neighbour: the offsets then point at the prism's own nodes
// (in bounds, unused) so the loads need no branch.
template <typename R>
struct LatNb {
  uint32_t no[4];
  R uo[4], vo[4];
  bool lds;          // column walk: no[] are offsets into the layer's LDS slot
};

template <typename R>
__device__ __forceinline__ void lat_nb(const StageArgs& a, const LatMeta<R>& M, int e, int l, uint32_t po,
                                       LatNb<R>& nb) {
  const size_t S = (size_t)a.m.n_slots;
  const uint32_t rs = (uint32_t)(S * sizeof(R));     // bytes per node row
  const R* __restrict__ U = static_cast<const R*>(a.U);
  const int A = e, B = (e + 1) % 3;
  const bool live = M.nslot >= 0 && l < (M.meta >> 2);
  const int kp = M.meta & 3;
  const uint32_t nA = live ? (uint32_t)((kp + 1) % 3) : (uint32_t)A;
  const uint32_t nB = live ? (uint32_t)kp : (uint32_t)B;
  const uint32_t pno = live ? ((uint32_t)M.nslot + (uint32_t)l * kCell) * (uint32_t)sizeof(R) : po;
  nb.no[0] = nA * rs + pno;
  nb.no[1] = nB * rs + pno;
  nb.no[2] = nb.no[0] + 3u * rs;
  nb.no[3] = nb.no[1] + 3u * rs;
  nb.lds = false;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    nb.uo[j] = ldb(U, nb.no[j]);
    nb.vo[j] = ldb(U + 6 * S, nb.no[j]);
  }
}

// Upwind weights at the 3 x 2 face points from q = u_n dS, u_n the normal
// component of the average of the two velocity traces (a wall carries no
// flux): the flux is q times the inner trace where q > 0, else the outer one.
template <typename R>
struct LatF {
  // FP64 keeps the signed weight q alone, and picks the upwind trace by its
  // sign (the one wavefront per SIMD runs short of registers: 1.5-2% faster);
  // FP32 keeps max(q, 0) and min(q, 0) (2% slower the other way).
  static constexpr bool kSigned = sizeof(R) == 8;
  R up[3][2];                    // q (FP64) or max(q, 0) (FP32)
  R um[kSigned ? 1 : 3][2];      // min(q, 0) (FP32 only)
  uint32_t no[4];
  bool interior;
  bool lds;
};

template <typename R>
__device__ __forceinline__ void lat_factors(const LatMeta<R>& M, const LatNb<R>& nb, int e, int l, const R dz[3],
                                            const R u[6], const R v[6], LatF<R>& F) {
  const int A = e, B = (e + 1) % 3;
  F.interior = M.nslot >= 0;
  const bool wall = F.interior && l >= (M.meta >> 2);
  const bool live = F.interior && !wall;
  const R nx = M.nx, ny = M.ny;
  const R Le = wall ? R(0) : M.Le;
#pragma unroll
  for (int j = 0; j < 4; ++j) F.no[j] = nb.no[j];
  F.lds = nb.lds;
  R un[4] = {nx * u[A] + ny * v[A], nx * u[B] + ny * v[B], nx * u[A + 3] + ny * v[A + 3],
             nx * u[B + 3] + ny * v[B + 3]};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const R avg = R(0.5) * (un[j] + nx * nb.uo[j] + ny * nb.vo[j]);
    un[j] = live ? avg : un[j];
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const R s = R(kS[j]), s1 = R(1) - R(kS[j]);
    const R dS = R(kSw[j]) * Le * R(0.5) * (s1 * dz[A] + s * dz[B]);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const R tk = R(kZt[k]), bk = R(kZb[k]);
      const R q = (s1 * (tk * un[0] + bk * un[2]) + s * (tk * un[1] + bk * un[3])) * dS;
      if constexpr (LatF<R>::kSigned) {
        F.up[j][k] = q;
      } else {
        F.up[j][k] = upos(q);
        F.um[j][k] = uneg(q);
      }
    }
  }
}

// The neighbour's 4 face-node values of field f (stage input), or the
// exterior value on an open boundary.
template <typename R>
__device__ __forceinline__ void lat_neighbour(const StageArgs& a, const LatF<R>& F, int f, R to[4]) {
  const R* fb = static_cast<const R*>(a.Ts) + (size_t)(f * 6) * (size_t)a.m.n_slots;
  const R te = R(a.t_ext[f]);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const R x = ldb(fb, F.no[j]);
    to[j] = F.interior ? x : te;
  }
}

// res[i] -= int_face phi_i Fhat dS for one field.
template <typename R>
__device__ __forceinline__ void lat_field(int e, const LatF<R>& F, const R T[6], const R to[4], R res[6]) {
  const int A = e, B = (e + 1) % 3;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const R s = R(kS[j]), s1 = R(1) - R(kS[j]);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const R tk = R(kZt[k]), bk = R(kZb[k]);
      const R ti = s1 * (tk * T[A] + bk * T[A + 3]) + s * (tk * T[B] + bk * T[B + 3]);
      const R tq = s1 * (tk * to[0] + bk * to[2]) + s * (tk * to[1] + bk * to[3]);
      R fl;
      if constexpr (LatF<R>::kSigned)
        fl = F.up[j][k] * (F.up[j][k] > R(0) ? ti : tq);
      else
        fl = F.up[j][k] * ti + F.um[j][k] * tq;
      res[A] -= s1 * tk * fl;
      res[B] -= s * tk * fl;
      res[A + 3] -= s1 * bk * fl;
      res[B + 3] -= s * bk * fl;
    }
  }
}

// Horizontal face between an upper prism (its bottom nodes 3..5) and a lower
// prism (its top nodes 0..2) of one column, at level heights zf:
//   F_q = w_q lambda(q).un      upward flux (un: upward normal velocity times
//                               J_h at the 3 face nodes, averaged over the
//                               two sides where both exist)
//   h_q = max(F_q, 0) T_lower(q) + min(F_q, 0) T_upper(q)
//   g_n = sum_q lambda_n(q) h_q
// The upper prism adds g to its bottom nodes' residual, the lower prism
// subtracts it from its top nodes'.  A missing side (surface, bottom) takes
// the exterior value and does not enter the velocity average.
// As in the volume term, the sums over q are contracted once per face into
//   Gp[n][a] = sum_q lambda_n(q) lambda_a(q) max(F_q, 0),
//   Gm[n][a] = sum_q lambda_n(q) lambda_a(q) min(F_q, 0)   (both symmetric),
// so g = Gp T_lower + Gm T_upper per field (18 multiply-adds instead of 66).
template <typename R>
struct HorF {
  R gp[6], gm[6];   // symmetric 3x3, entries 00 11 22 01 02 12
  bool has_up, has_lo;
};

template <typename R, bool WZ>
__device__ __forceinline__ void hface_factors(const ColGeo<R>& cg, const R zf[3], bool has_up, const R uu[3],
                                              const R vu[3], const R wu[3], bool has_lo, const R ul[3],
                                              const R vl[3], const R wl[3], HorF<R>& F) {
  const R zxi = zf[1] - zf[0], zet = zf[2] - zf[0];
  const R jzx = zxi * cg.yet - zet * cg.yxi;
  const R jzy = zet * cg.xxi - zxi * cg.xet;
  R un[3];
#pragma unroll
  for (int n = 0; n < 3; ++n) {
    R x = -(uu[n] * jzx + vu[n] * jzy);
    if (!WZ) x += cg.Jh * wu[n];
    R y = -(ul[n] * jzx + vl[n] * jzy);
    if (!WZ) y += cg.Jh * wl[n];
    const R avg = R(0.5) * (x + y);
    un[n] = has_up ? (has_lo ? avg : x) : y;
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) F.gp[i] = F.gm[i] = R(0);
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const R Fq = R(kTw[q]) * (R(kL0[q]) * un[0] + R(kL1[q]) * un[1] + R(kL2[q]) * un[2]);
    const R fp = upos(Fq), fm = uneg(Fq);
    const R c[6] = {R(kL0[q] * kL0[q]), R(kL1[q] * kL1[q]), R(kL2[q] * kL2[q]),
                    R(kL0[q] * kL1[q]), R(kL0[q] * kL2[q]), R(kL1[q] * kL2[q])};
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      F.gp[i] += c[i] * fp;
      F.gm[i] += c[i] * fm;
    }
  }
  F.has_up = has_up;
  F.has_lo = has_lo;
}

template <typename R>
__device__ __forceinline__ void hface_field(const HorF<R>& F, R te, const R Tu[3], const R Tl[3], R g[3]) {
  R tu[3], tl[3];
#pragma unroll
  for (int n = 0; n < 3; ++n) {
    tu[n] = F.has_up ? Tu[n] : te;
    tl[n] = F.has_lo ? Tl[n] : te;
  }
  g[0] = F.gp[0] * tl[0] + F.gp[3] * tl[1] + F.gp[4] * tl[2] + (F.gm[0] * tu[0] + F.gm[3] * tu[1] + F.gm[4] * tu[2]);
  g[1] = F.gp[3] * tl[0] + F.gp[1] * tl[1] + F.gp[5] * tl[2] + (F.gm[3] * tu[0] + F.gm[1] * tu[1] + F.gm[5] * tu[2]);
  g[2] = F.gp[4] * tl[0] + F.gp[5] * tl[1] + F.gp[2] * tl[2] + (F.gm[4] * tu[0] + F.gm[5] * tu[1] + F.gm[2] * tu[2]);
}

// Mz = J_h/120 * m with m_aa = 3 dz_a + dz_b + dz_c, m_ab = dz_a + dz_b + dz_c/2;
// Mz^-1 = sc * cofactors.
template <typename R>
struct MinvF {
  R c00, c01, c02, c11, c12, c22, sc;
};

template <typename R>
__device__ __forceinline__ void minv_factors(const ColGeo<R>& cg, const R dz[3], MinvF<R>& F) {
  const R m00 = R(3) * dz[0] + dz[1] + dz[2];
  const R m11 = dz[0] + R(3) * dz[1] + dz[2];
  const R m22 = dz[0] + dz[1] + R(3) * dz[2];
  const R m01 = dz[0] + dz[1] + R(0.5) * dz[2];
  const R m02 = dz[0] + dz[2] + R(0.5) * dz[1];
  const R m12 = dz[1] + dz[2] + R(0.5) * dz[0];
  F.c00 = m11 * m22 - m12 * m12;
  F.c01 = m02 * m12 - m01 * m22;
  F.c02 = m01 * m12 - m02 * m11;
  F.c11 = m00 * m22 - m02 * m02;
  F.c12 = m01 * m02 - m00 * m12;
  F.c22 = m00 * m11 - m01 * m01;
  const R det = m00 * F.c00 + m01 * F.c01 + m02 * F.c02;
  F.sc = R(120) / (cg.Jh * det);
}

// L = M^-1 res (M^-1 = [2 -1; -1 2] (x) Mz^-1), then out = a Tn + b (T + dt L)
// (or L alone), stored at row f of the output for an active prism.
template <typename R, bool RHS, bool READ_TN, bool OUT2>
__device__ __forceinline__ void finish_field(const StageArgs& a, const MinvF<R>& F, int f, const R T[6],
                                             const R res[6], const R tn[6], uint32_t po, bool active) {
  const R ht[3] = {R(2) * res[0] - res[3], R(2) * res[1] - res[4], R(2) * res[2] - res[5]};
  const R hb[3] = {R(2) * res[3] - res[0], R(2) * res[4] - res[1], R(2) * res[5] - res[2]};
  R L[6];
  L[0] = F.sc * (F.c00 * ht[0] + F.c01 * ht[1] + F.c02 * ht[2]);
  L[1] = F.sc * (F.c01 * ht[0] + F.c11 * ht[1] + F.c12 * ht[2]);
  L[2] = F.sc * (F.c02 * ht[0] + F.c12 * ht[1] + F.c22 * ht[2]);
  L[3] = F.sc * (F.c00 * hb[0] + F.c01 * hb[1] + F.c02 * hb[2]);
  L[4] = F.sc * (F.c01 * hb[0] + F.c11 * hb[1] + F.c12 * hb[2]);
  L[5] = F.sc * (F.c02 * hb[0] + F.c12 * hb[1] + F.c22 * hb[2]);
  const size_t S = (size_t)a.m.n_slots;
  R* __restrict__ Out = static_cast<R*>(a.Tout);
  R* __restrict__ Out2 = static_cast<R*>(a.Tout2);
  const R dt = R(a.dt), ca = R(a.a), cb = R(a.b);
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    R out;
    if (RHS) {
      out = L[i];
    } else {
      out = cb * (T[i] + dt * L[i]);
      if (READ_TN) out += ca * tn[i];
    }
    if (active) {
      str(Out, S, f * 6 + i, po, out);
      // second output T - 2 Tout (the split-IMEX first step)
      if (OUT2) str(Out2, S, f * 6 + i, po, T[i] - R(2) * out);
    }
  }
}

// Which tiles workgroup b processes: one tile, or (a.persistent) a grid sized
// to what the chip holds at once, each workgroup walking tiles with a stride.
// With the XCD remap, tiles are split into 8 contiguous parts and workgroup
// b, which the dispatcher places on XCD b mod 8, takes part b mod 8, so tiles
// that share faces are processed on one XCD and its L2 (the persistent grid is
// a multiple of 8).
struct TileRange {
  int t, end, step;
};

__device__ __forceinline__ TileRange tile_range(const StageArgs& a) {
  const int b = (int)blockIdx.x;
  TileRange r;
  if (!a.persistent) {
    r.t = a.xcd ? xcd_tile(b, a.n_tiles) : b;
    r.end = r.t + 1;
    r.step = 1;
  } else if (a.xcd) {
    const int q = a.n_tiles >> 3, rem = a.n_tiles & 7, x = b & 7;
    const int lo = x * q + (x < rem ? x : rem);
    r.t = lo + (b >> 3);
    r.end = lo + q + (x < rem ? 1 : 0);
    r.step = (int)gridDim.x >> 3;
  } else {
    r.t = b;
    r.end = a.n_tiles;
    r.step = (int)gridDim.x;
  }
  return r;
}

// ===========================================================================
// stage_kernel: one thread per prism.
// ===========================================================================
template <typename R, int NF, bool WZ, bool RHS, bool READ_TN, bool OUT2>
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
  const uint32_t p = (uint32_t)m.cell_base[tile.cell] + (uint32_t)l * kCell + lane;
  const uint32_t lt = (uint32_t)m.cell_lbase[tile.cell] + (uint32_t)l * kCell + lane;
  const uint32_t po = p * (uint32_t)sizeof(R);       // this prism's byte offset in a row
  const uint32_t co = (uint32_t)c * (uint32_t)sizeof(R);
  const R* __restrict__ Ts = static_cast<const R*>(a.Ts);
  const R* __restrict__ U = static_cast<const R*>(a.U);
  const R* __restrict__ Tn = static_cast<const R*>(a.Tn);
  const R* __restrict__ zl = zl_of<R>(m);
  // neighbour layers above and below; the address only needs the
  // (wavefront-uniform) cell depth, the value select the column's own depth
  const uint32_t pup = (l > 0 ? p - kCell : p) * (uint32_t)sizeof(R);
  const uint32_t plo = (l + 1 < depth ? p + kCell : p) * (uint32_t)sizeof(R);

  const ColGeo<R> cg = load_colgeo<R>(m, co);
  R zt[3], zb[3], dz[3];
#pragma unroll
  for (int v3 = 0; v3 < 3; ++v3) {
    zt[v3] = ldb(zl + v3 * LS, lt * (uint32_t)sizeof(R));
    zb[v3] = ldb(zl + v3 * LS, (lt + kCell) * (uint32_t)sizeof(R));
    dz[v3] = zt[v3] - zb[v3];
  }
  VolF<R> vf;
  LatF<R> lf[3];
  HorF<R> top, bot;
  MinvF<R> mf;
  {
    R u[6], v[6], w[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      u[i] = ldr(U, S, 0 * 6 + i, po);
      v[i] = ldr(U, S, 1 * 6 + i, po);
      w[i] = WZ ? R(0) : ldr(U, S, 2 * 6 + i, po);
    }
    volume_factors<R, WZ>(cg, zt, zb, dz, u, v, w, vf);
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      LatMeta<R> M;
      LatNb<R> nb;
      lat_meta<R>(m, e, co, M);
      lat_nb<R>(a, M, e, l, po, nb);
      lat_factors<R>(M, nb, e, l, dz, u, v, lf[e]);
    }
    R ux[3], vx[3], wx[3];
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      ux[n] = ldr(U, S, 0 * 6 + 3 + n, pup);
      vx[n] = ldr(U, S, 1 * 6 + 3 + n, pup);
      wx[n] = WZ ? R(0) : ldr(U, S, 2 * 6 + 3 + n, pup);
    }
    hface_factors<R, WZ>(cg, zt, l > 0, ux, vx, wx, true, u, v, w, top);
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      ux[n] = ldr(U, S, 0 * 6 + n, plo);
      vx[n] = ldr(U, S, 1 * 6 + n, plo);
      wx[n] = WZ ? R(0) : ldr(U, S, 2 * 6 + n, plo);
    }
    hface_factors<R, WZ>(cg, zb, true, u + 3, v + 3, w + 3, l < N - 1, ux, vx, wx, bot);
    minv_factors<R>(cg, dz, mf);
  }
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    R T[6], res[6], tn[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      T[i] = ldr(Ts, S, f * 6 + i, po);
      tn[i] = READ_TN ? ldr(Tn, S, f * 6 + i, po) : R(0);
    }
    volume_field<R>(vf, T, res);
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      R to[4];
      lat_neighbour<R>(a, lf[e], f, to);
      lat_field<R>(e, lf[e], T, to, res);
    }
    const R te = R(a.t_ext[f]);
    R Tx[3], g[3];
#pragma unroll
    for (int n = 0; n < 3; ++n) Tx[n] = ldr(Ts, S, f * 6 + 3 + n, pup);
    hface_field<R>(top, te, Tx, T, g);
#pragma unroll
    for (int n = 0; n < 3; ++n) res[n] -= g[n];
#pragma unroll
    for (int n = 0; n < 3; ++n) Tx[n] = ldr(Ts, S, f * 6 + n, plo);
    hface_field<R>(bot, te, T + 3, Tx, g);
#pragma unroll
    for (int n = 0; n < 3; ++n) res[3 + n] += g[n];
    finish_field<R, RHS, READ_TN, OUT2>(a, mf, f, T, res, tn, po, active);
  }
}

template <typename R, int NF, bool WZ, bool RHS, bool READ_TN, bool OUT2>
__global__ __launch_bounds__(256) void stage_kernel(StageArgs a) {
  TileRange r = tile_range(a);
  for (; r.t < r.end; r.t += r.step) stage_tile<R, NF, WZ, RHS, READ_TN, OUT2>(a, a.tiles[r.t]);
}

// ===========================================================================
// walk_kernel: one wavefront walks a cell's layers l0 .. l0 + nlay - 1 of its tile.
// ===========================================================================
constexpr int kWalkLdsBytes = 40960;   // two layer slots; 4 wavefronts per CU

// LDS slot of one layer: [row][64 lanes] values of type R, in sections
// (stage input, velocity, bottom level heights, Tn where it fits), each
// padded to whole 1 KiB loads.
template <typename R, int NF, bool WZ, bool READ_TN>
struct WalkLayout {
  static constexpr int kPerLoad = 1024 / (kCell * (int)sizeof(R));   // rows per 16 B/lane load
  static constexpr int pad(int r) { return (r + kPerLoad - 1) / kPerLoad * kPerLoad; }
  static constexpr int kNU = WZ ? 12 : 18;            // u 0..5, v 0..5 (, w 0..5)
  static constexpr int kTs = 0;
  static constexpr int kU = pad(6 * NF);
  static constexpr int kZ = kU + pad(kNU);
  static constexpr int kBase = kZ + pad(3);
  // Tn joins the layer copy only where two slots with it stay within one
  // wavefront's share of the CU's LDS: 40 KB in FP64 (one wavefront per
  // SIMD), 20 KB in FP32 (two).  In FP32 with 4 fields it would not, and
  // holding it there cut the residency to five wavefronts per CU (stages 1
  // and 2: 0.94 against 0.72 ms with Tn read from global memory).
  static constexpr bool kTnLds =
      READ_TN && 2 * (kBase + pad(6 * NF)) * kCell * (int)sizeof(R) <= kWalkLdsBytes / (sizeof(R) == 8 ? 1 : 2);
  static constexpr int kTn = kBase;
  static constexpr int kRows = kBase + (kTnLds ? pad(6 * NF) : 0);
  static constexpr int kSlot = kRows * kCell;         // values of type R per slot
  static constexpr int kBytes = 2 * kSlot * (int)sizeof(R);
  static_assert(kBytes <= 65536, "walk LDS above the workgroup limit");
};

typedef __attribute__((address_space(3))) void* lds_ptr_t;

// Copy `count` rows (row stride rowb bytes) starting at `base` + lane offset
// `voff` into LDS rows from `dst`: each 16-byte-per-lane load moves kPerLoad
// rows of kCell values, lane i writing LDS bytes [16 i, 16 i + 16) of the
// load's 1 KiB block; rows past `count` in the last load repeat the last row.
template <typename R, int kPerLoad>
__device__ __forceinline__ void fetch_rows(const char* base, uint32_t rowb, int count, uint32_t voff, int sub,
                                           R* dst) {
#pragma unroll
  for (int k = 0; k < (count + kPerLoad - 1) / kPerLoad; ++k) {
    const int left = count - 1 - k * kPerLoad;
    const uint32_t j = (uint32_t)(sub < left ? sub : left);
    __builtin_amdgcn_global_load_lds(base + (size_t)(k * kPerLoad) * rowb + (j * rowb + voff),
                                     (lds_ptr_t)(dst + k * kPerLoad * kCell), 16, 0, 0);
  }
}

struct WalkCell {
  int cell, N, depth;
  uint32_t base, lbase;
};
// One layer L of this cell into an LDS slot.
template <typename R, int NF, bool WZ, bool READ_TN>
__device__ __forceinline__ void walk_fetch(const StageArgs& a, const WalkCell& wc, int L, R* slot, int lane) {
  using Ly = WalkLayout<R, NF, WZ, READ_TN>;
  constexpr int kLanesPerRow = kCell / Ly::kPerLoad;
  const DevMesh& m = a.m;
  const int sub = lane / kLanesPerRow;
  const uint32_t chunk = (uint32_t)(lane % kLanesPerRow) * 16u;
  const uint32_t rowb = (uint32_t)((size_t)m.n_slots * sizeof(R));
  const uint32_t lrowb = (uint32_t)((size_t)m.n_lslots * sizeof(R));
  const uint32_t pb = (wc.base + (uint32_t)L * kCell) * (uint32_t)sizeof(R) + chunk;
  const uint32_t zb = (wc.lbase + (uint32_t)(L + 1) * kCell) * (uint32_t)sizeof(R) + chunk;
  fetch_rows<R, Ly::kPerLoad>(static_cast<const char*>(a.Ts), rowb, 6 * NF, pb, sub, slot + Ly::kTs * kCell);
  fetch_rows<R, Ly::kPerLoad>(static_cast<const char*>(a.U), rowb, Ly::kNU, pb, sub, slot + Ly::kU * kCell);
  fetch_rows<R, Ly::kPerLoad>(reinterpret_cast<const char*>(zl_of<R>(m)), lrowb, 3, zb, sub, slot + Ly::kZ * kCell);
  if (Ly::kTnLds)
    fetch_rows<R, Ly::kPerLoad>(static_cast<const char*>(a.Tn), rowb, 6 * NF, pb, sub, slot + Ly::kTn * kCell);
}

// vmcnt(0) / lgkmcnt(0) alone (gfx9 s_waitcnt encoding), each also a
// compiler memory barrier so no LDS read is moved above the wait that makes
// its data valid, nor a copy into LDS above the reads it must follow.
__device__ __forceinline__ void wait_vm() {
  __builtin_amdgcn_s_waitcnt(0x0F70);
  asm volatile("" ::: "memory");
}
__device__ __forceinline__ void wait_lgkm() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);
}
// Keeps later LDS reads below a just-issued copy (compiler barrier only).
__device__ __forceinline__ void mem_order() { asm volatile("" ::: "memory"); }

template <typename R>
__device__ __forceinline__ R lds_at(const R* slot, uint32_t byte_off) {
  return *reinterpret_cast<const R*>(reinterpret_cast<const char*>(slot) + byte_off);
}

// Column-walk form of lat_nb.  The layer's stage input and velocity of all
// 64 columns of the cell are already in the LDS slot `cur`, so a neighbour
// column of the same cell (most lateral faces of a locality-ordered mesh) is
// read from there; only a neighbour in another cell is read from global
// memory.  A face without a live neighbour points at the column's own nodes
// in LDS (in bounds, unused).
template <typename R, int kURow>
__device__ __forceinline__ void lat_nb_walk(const StageArgs& a, const LatMeta<R>& M, int e, int l, uint32_t po,
                                            int lane, uint32_t cell_base, const R* cur, LatNb<R>& nb) {
  const size_t S = (size_t)a.m.n_slots;
  const uint32_t rs = (uint32_t)(S * sizeof(R));
  const R* __restrict__ U = static_cast<const R*>(a.U);
  const int A = e, B = (e + 1) % 3;
  const bool live = M.nslot >= 0 && l < (M.meta >> 2);
  const int kp = M.meta & 3;
  const uint32_t nlane = (uint32_t)M.nslot - cell_base;   // < 64 iff the neighbour is in this cell
  nb.lds = !live || nlane < (uint32_t)kCell;
  const uint32_t nA = live ? (uint32_t)((kp + 1) % 3) : (uint32_t)A;
  const uint32_t nB = live ? (uint32_t)kp : (uint32_t)B;
  if (nb.lds) {
    constexpr uint32_t row = kCell * sizeof(R);
    const uint32_t ln = (live ? nlane : (uint32_t)lane) * (uint32_t)sizeof(R);
    nb.no[0] = nA * row + ln;
    nb.no[1] = nB * row + ln;
    nb.no[2] = nb.no[0] + 3u * row;
    nb.no[3] = nb.no[1] + 3u * row;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      nb.uo[j] = lds_at(cur, (uint32_t)kURow * row + nb.no[j]);
      nb.vo[j] = lds_at(cur, (uint32_t)(kURow + 6) * row + nb.no[j]);
    }
  } else {
    const uint32_t pno = ((uint32_t)M.nslot + (uint32_t)l * kCell) * (uint32_t)sizeof(R);
    (void)po;
    nb.no[0] = nA * rs + pno;
    nb.no[1] = nB * rs + pno;
    nb.no[2] = nb.no[0] + 3u * rs;
    nb.no[3] = nb.no[1] + 3u * rs;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      nb.uo[j] = ldb(U, nb.no[j]);
      nb.vo[j] = ldb(U + 6 * S, nb.no[j]);
    }
  }
}

// Column-walk form of lat_neighbour: field f's neighbour traces from the LDS
// slot or from global memory, as lat_nb_walk decided.
template <typename R, int kTsRow>
__device__ __forceinline__ void lat_neighbour_walk(const StageArgs& a, const LatF<R>& F, int f, const R* cur,
                                                   R to[4]) {
  const R* fb = static_cast<const R*>(a.Ts) + (size_t)(f * 6) * (size_t)a.m.n_slots;
  const R te = R(a.t_ext[f]);
  constexpr uint32_t row = kCell * sizeof(R);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    R x;
    if (F.lds)
      x = lds_at(cur, (uint32_t)(kTsRow + f * 6) * row + F.no[j]);
    else
      x = ldb(fb, F.no[j]);
    to[j] = F.interior ? x : te;
  }
}

// State a wavefront carries from one layer of its walk to the next.
template <typename R, int NF>
struct WalkCarry {
  R zt[3];          // heights of the layer's top level
  R gtop[NF][3];    // horizontal-face contribution to the layer's top nodes
};

// One layer l of the walk.  `cur` holds layer l (complete), `nxt` receives
// layer l+1.  cur and nxt are distinct __shared__ arrays, so the compiler
// sees that reading cur does not wait for the copy into nxt.  Loads complete
// in order, so each phase issues the loads it needs before the ones needed
// later: neighbour velocities, then the next layer's copy, then (per field)
// neighbour traces one field ahead.
template <typename R, int NF, bool WZ, bool RHS, bool READ_TN, bool OUT2>
__device__ __forceinline__ void walk_layer(const StageArgs& a, const ColGeo<R>& cg, const LatMeta<R> (&lm)[3],
                                           const WalkCell& wc, int lane, int l, const R* cur, R* nxt,
                                           WalkCarry<R, NF>& cs) {
  const int N = wc.N, depth = wc.depth;
  using Ly = WalkLayout<R, NF, WZ, READ_TN>;
  const DevMesh& m = a.m;
  const size_t S = (size_t)m.n_slots;
  const uint32_t p = wc.base + (uint32_t)l * kCell + lane;
  const uint32_t po = p * (uint32_t)sizeof(R);
  const bool below = l + 1 < depth;   // wavefront-uniform
  const bool active = l < N;
  auto own = [&](int row) { return cur[row * kCell + lane]; };
  auto next = [&](int row, R fallback) { return below ? nxt[row * kCell + lane] : fallback; };

  // In-cell neighbours from LDS: 1.8% faster over a step's three stages in
  // FP64, 9% in FP32 (with two wavefronts per SIMD resident).
  LatNb<R> nb[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) lat_nb_walk<R, Ly::kU>(a, lm[e], e, l, po, lane, wc.base, cur, nb[e]);
  wait_lgkm();
  if (below) walk_fetch<R, NF, WZ, READ_TN>(a, wc, l + 1, nxt, lane);
  mem_order();
  phase();

  R zb[3], dz[3];
#pragma unroll
  for (int v3 = 0; v3 < 3; ++v3) {
    zb[v3] = own(Ly::kZ + v3);
    dz[v3] = cs.zt[v3] - zb[v3];
  }
  VolF<R> vf;
  LatF<R> lf[3];
  HorF<R> bot;
  MinvF<R> mf;
  // Neighbour traces are requested kTA fields ahead of the field being
  // computed: two in FP64 (2.8% faster over a step's three stages, the
  // cross-cell gathers' latency being the longest), one in FP32 (2-4% slower
  // with two).
  constexpr int kTA = (sizeof(R) == 8 && NF > 2) ? 2 : 1;
  R to[3][4], to1[3][4];
  {
    R u[6], v[6], w[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      u[i] = own(Ly::kU + i);
      v[i] = own(Ly::kU + 6 + i);
      w[i] = WZ ? R(0) : own(Ly::kU + 12 + i);
    }
    volume_factors<R, WZ>(cg, cs.zt, zb, dz, u, v, w, vf);
    minv_factors<R>(cg, dz, mf);
    phase();
#pragma unroll
    for (int e = 0; e < 3; ++e) lat_factors<R>(lm[e], nb[e], e, l, dz, u, v, lf[e]);
#pragma unroll
    for (int e = 0; e < 3; ++e) lat_neighbour_walk<R, Ly::kTs>(a, lf[e], 0, cur, to[e]);
    if (kTA == 2) {
#pragma unroll
      for (int e = 0; e < 3; ++e) lat_neighbour_walk<R, Ly::kTs>(a, lf[e], 1, cur, to1[e]);
    }
    phase();
    wait_vm();   // layer l+1 has arrived
    R ul[3], vl[3], wl[3];
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      ul[n] = next(Ly::kU + n, u[3 + n]);
      vl[n] = next(Ly::kU + 6 + n, v[3 + n]);
      wl[n] = WZ ? R(0) : next(Ly::kU + 12 + n, w[3 + n]);
    }
    hface_factors<R, WZ>(cg, zb, true, u + 3, v + 3, w + 3, l < N - 1, ul, vl, wl, bot);
  }
  const R* __restrict__ Tn = static_cast<const R*>(a.Tn);
  R tn[6];
#pragma unroll
  for (int i = 0; i < 6; ++i)
    tn[i] = (READ_TN && !Ly::kTnLds) ? ldr(Tn, S, i, po) : R(0);
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    phase();
    R T[6], res[6], ton[3][4], tnn[6];
    // neighbour traces kTA fields ahead, and the next field's Tn, are
    // requested before this field computes
    if (f + kTA < NF) {
#pragma unroll
      for (int e = 0; e < 3; ++e) lat_neighbour_walk<R, Ly::kTs>(a, lf[e], f + kTA, cur, ton[e]);
    }
    if (f + 1 < NF) {
#pragma unroll
      for (int i = 0; i < 6; ++i)
        tnn[i] = (READ_TN && !Ly::kTnLds) ? ldr(Tn, S, (f + 1) * 6 + i, po) : R(0);
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) T[i] = own(Ly::kTs + f * 6 + i);
    volume_field<R>(vf, T, res);
#pragma unroll
    for (int e = 0; e < 3; ++e) lat_field<R>(e, lf[e], T, to[e], res);
#pragma unroll
    for (int n = 0; n < 3; ++n) res[n] -= cs.gtop[f][n];
    {
      R Tl[3];
#pragma unroll
      for (int n = 0; n < 3; ++n) Tl[n] = next(Ly::kTs + f * 6 + n, T[3 + n]);
      hface_field<R>(bot, R(a.t_ext[f]), T + 3, Tl, cs.gtop[f]);
#pragma unroll
      for (int n = 0; n < 3; ++n) res[3 + n] += cs.gtop[f][n];
    }
    if (Ly::kTnLds) {
#pragma unroll
      for (int i = 0; i < 6; ++i) tn[i] = own(Ly::kTn + f * 6 + i);
    }
    finish_field<R, RHS, READ_TN, OUT2>(a, mf, f, T, res, tn, po, active);
    if (f + 1 < NF) {
#pragma unroll
      for (int e = 0; e < 3; ++e)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (kTA == 2) {
            to[e][j] = to1[e][j];
            to1[e][j] = ton[e][j];
          } else {
            to[e][j] = ton[e][j];
          }
        }
#pragma unroll
      for (int i = 0; i < 6; ++i) tn[i] = tnn[i];
    }
  }
#pragma unroll
  for (int v3 = 0; v3 < 3; ++v3) cs.zt[v3] = zb[v3];
}

template <typename R, int NF, bool WZ, bool RHS, bool READ_TN, bool OUT2>
__global__ __launch_bounds__(64) void walk_kernel(StageArgs a) {
  using Ly = WalkLayout<R, NF, WZ, READ_TN>;
  __shared__ __align__(16) R slot0[Ly::kSlot];
  __shared__ __align__(16) R slot1[Ly::kSlot];
  const DevMesh& m = a.m;
  const int lane = threadIdx.x;
  TileRange r = tile_range(a);
  for (; r.t < r.end; r.t += r.step) {
    const WgTile tile = a.tiles[r.t];
    const int cell = tile.cell;
    const int c = cell * kCell + lane;
    WalkCell wc;
    wc.cell = cell;
    wc.N = m.nlay[c];
    wc.base = (uint32_t)m.cell_base[cell];
    wc.lbase = (uint32_t)m.cell_lbase[cell];
    wc.depth = (int)(((uint32_t)m.cell_base[cell + 1] - wc.base) / kCell);
    const int depth = wc.depth;
    const int l0 = tile.layer0;
    const int l1 = l0 + tile.nlay;
    const size_t S = (size_t)m.n_slots;
    const size_t LS = (size_t)m.n_lslots;
    const uint32_t pc = wc.base + lane;
    const R* __restrict__ Ts = static_cast<const R*>(a.Ts);
    const R* __restrict__ U = static_cast<const R*>(a.U);
    const R* __restrict__ zl = zl_of<R>(m);
    const uint32_t co = (uint32_t)c * (uint32_t)sizeof(R);
    const ColGeo<R> cg = load_colgeo<R>(m, co);
    LatMeta<R> lm[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) lat_meta<R>(m, e, co, lm[e]);

    // layer l0 into slot0; the top face of l0 from the layer above (global)
    wait_lgkm();
    walk_fetch<R, NF, WZ, READ_TN>(a, wc, l0, slot0, lane);
    WalkCarry<R, NF> cs;
    {
      const uint32_t lt = wc.lbase + (uint32_t)l0 * kCell + lane;
#pragma unroll
      for (int v3 = 0; v3 < 3; ++v3) cs.zt[v3] = ldb(zl + v3 * LS, lt * (uint32_t)sizeof(R));
      const uint32_t pup = (l0 > 0 ? pc + (uint32_t)(l0 - 1) * kCell : pc) * (uint32_t)sizeof(R);
      R uu[3], vu[3], wu[3], ul[3], vl[3], wl[3];
#pragma unroll
      for (int n = 0; n < 3; ++n) {
        uu[n] = ldr(U, S, 0 * 6 + 3 + n, pup);
        vu[n] = ldr(U, S, 1 * 6 + 3 + n, pup);
        wu[n] = WZ ? R(0) : ldr(U, S, 2 * 6 + 3 + n, pup);
      }
      // the layer above's bottom values, requested with its velocity before the wait
      R Tu[NF][3];
#pragma unroll
      for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int n = 0; n < 3; ++n) Tu[f][n] = ldr(Ts, S, f * 6 + 3 + n, pup);
      wait_vm();
#pragma unroll
      for (int n = 0; n < 3; ++n) {
        ul[n] = slot0[(Ly::kU + n) * kCell + lane];
        vl[n] = slot0[(Ly::kU + 6 + n) * kCell + lane];
        wl[n] = WZ ? R(0) : slot0[(Ly::kU + 12 + n) * kCell + lane];
      }
      HorF<R> top;
      hface_factors<R, WZ>(cg, cs.zt, l0 > 0, uu, vu, wu, true, ul, vl, wl, top);
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        R Tl[3];
#pragma unroll
        for (int n = 0; n < 3; ++n) Tl[n] = slot0[(Ly::kTs + f * 6 + n) * kCell + lane];
        hface_field<R>(top, R(a.t_ext[f]), Tu[f], Tl, cs.gtop[f]);
      }
    }
    // layers in pairs so that each half names its slots statically
    for (int l = l0; l < l1; l += 2) {
      walk_layer<R, NF, WZ, RHS, READ_TN, OUT2>(a, cg, lm, wc, lane, l, slot0, slot1, cs);
      if (l + 1 < l1) walk_layer<R, NF, WZ, RHS, READ_TN, OUT2>(a, cg, lm, wc, lane, l + 1, slot1, slot0, cs);
    }
    // the last layer may have started a copy into a slot the next tile reuses
    wait_vm();
  }
}

// ---------------------------------------------------------------------------
// Launch.
// ---------------------------------------------------------------------------
// Workgroups of one kernel instance that fit on one CU at once, per tile
// height, queried once.
template <typename Kern>
hipError_t resident_per_cu(Kern kern, int threads, size_t lds, std::atomic<int>* cache, int* out) {
  int v = cache->load(std::memory_order_relaxed);
  if (v == 0) {
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, reinterpret_cast<const void*>(kern), threads,
                                                                 lds);
    if (e != hipSuccess) return e;
    if (v < 1) v = 1;
    cache->store(v, std::memory_order_relaxed);
  }
  *out = v;
  return hipSuccess;
}

template <typename R, int NF, bool WZ, bool RHS, bool READ_TN, bool OUT2>
hipError_t launch_mode(const StageArgs& a, hipStream_t s) {
  const bool walk = a.tile_layers >= kWalkMinLayers;
  const int threads = walk ? kCell : kCell * a.tile_layers;
  int grid = a.n_tiles;
  if (a.persistent) {
    static std::atomic<int> cache[kTileChoices + 1];
    int ci = kTileChoices;   // the per-bucket walk table
    for (int i = 0; i < kTileChoices; ++i)
      if (kTileLayerOptions[i] == a.tile_layers) ci = i;
    int per_cu = 1;
    hipError_t e = walk ? resident_per_cu(&walk_kernel<R, NF, WZ, RHS, READ_TN, OUT2>, threads, 0, &cache[ci], &per_cu)
                        : resident_per_cu(&stage_kernel<R, NF, WZ, RHS, READ_TN, OUT2>, threads, 0, &cache[ci], &per_cu);
    if (e != hipSuccess) return e;
    grid = (per_cu * a.n_cu) & ~7;
    if (grid < 8) grid = 8;
    const int need = (a.n_tiles + 7) & ~7;
    if (grid > need) grid = need;
  }
  if (walk)
    hipLaunchKernelGGL((walk_kernel<R, NF, WZ, RHS, READ_TN, OUT2>), dim3(grid), dim3(threads), 0, s, a);
  else
    hipLaunchKernelGGL((stage_kernel<R, NF, WZ, RHS, READ_TN, OUT2>), dim3(grid), dim3(threads), 0, s, a);
  return hipGetLastError();
}

template <typename R, int NF>
hipError_t launch_nf(const StageArgs& a, bool w_zero, bool rhs_only, bool read_tn, hipStream_t s) {
  if (rhs_only)
    return w_zero ? launch_mode<R, NF, true, true, false, false>(a, s) : launch_mode<R, NF, false, true, false, false>(a, s);
  if (read_tn)
    return w_zero ? launch_mode<R, NF, true, false, true, false>(a, s) : launch_mode<R, NF, false, false, true, false>(a, s);
  if (a.Tout2)
    return w_zero ? launch_mode<R, NF, true, false, false, true>(a, s) : launch_mode<R, NF, false, false, false, true>(a, s);
  return w_zero ? launch_mode<R, NF, true, false, false, false>(a, s) : launch_mode<R, NF, false, false, false, false>(a, s);
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
  if (a.Tout2 && (rhs_only || read_tn)) return hipErrorInvalidValue;
  return fp32 ? launch_r<float>(a, w_zero, rhs_only, read_tn, s)
              : launch_r<double>(a, w_zero, rhs_only, read_tn, s);
}

}  // namespace sdg
