// Implicit vertical diffusion: (M - dt A) Tout = M T* for every column.
//
// One lane per column, one wavefront per cell of 64 columns, so every load
// and store of a layer touches 64 consecutive slots (the paper's cell layout,
// section 2.1.1, with the solve done one thread per column as in section 2.4).
// The column matrix is block tridiagonal with 6x6 blocks.  With the per-prism
// symmetric 3x3 matrices
//
//   Mz_ab = J_h int lambda_a lambda_b z_zeta          (mass, M = H (x) Mz)
//   Kv_ab = J_h sum_q w_q lambda_a lambda_b / D(q),   D = sum_c lambda_c dz_c
//   S_ab  = J_h int lambda_a lambda_b  = M_h          (2D mass, section 2.3)
//
// the interior-penalty operator gives, in (top, bottom) 3x3 blocks:
//
//   diagonal  D_l = M_l + dt kappa_l [Kv -Kv; -Kv Kv]
//                 + dt [-kappa_l Kv/2 + sig_u S, kappa_l Kv/2; 0 0]          (l > 0)
//                 + dt [0 0; kappa_l Kv/2, -kappa_l Kv/2 + sig_d S]          (l < N-1)
//   below     B_l = dt [-kappa_{l-1} Kv_{l-1}/2, kappa_{l-1} Kv_{l-1}/2 - sig_u S]
//             (rows: top nodes of l; columns: nodes of l-1)
//   above     C_l = dt [kappa_{l+1} Kv_{l+1}/2 - sig_d S, -kappa_{l+1} Kv_{l+1}/2]
//             (rows: bottom nodes of l; columns: nodes of l+1)
//
// which is the half-block sparsity drawn in section 2.4.  Block Thomas
// without pivoting: forward sweep D'_l = D_l - B_l D'_{l-1}^-1 C_{l-1}, with
// the LU of D'_l shared by all fields, E_l = D'_l^-1 [:, 3:6] and
// y_l = D'_l^-1 r'_l; back substitution x_l = y_l - E_l (C_l x_{l+1})
// recomputes C_l from the levels.
//
// E_l depends only on the mesh, kappa, dt and the penalty, not on the
// fields, so it is computed once for a given (kappa, dt, eta) by a sweep
// without fields (factor_kernel) and kept in scratch; each solve's forward
// sweep recomputes it in registers (its LU is needed for y) but stores only
// y_l, and the back substitution reads the kept E_l.  That moves 18 values
// per prism slot fewer than storing E with every solve (FP64 solve 1.39 ->
// 1.22 ms on 199,712 x 30 prisms, 4 fields).  Where the state has the solve's
// type, y_l goes into the output rows themselves, where the back
// substitution reads it and writes x_l over it (1.22 -> 1.17 ms: part of the
// y traffic then stays in the cache); otherwise (float state, double solve)
// into scratch.  Scratch values go as 16-byte pairs.  The arithmetic type C
// is double (the FP64 and FP32-state/FP64-solve forms) or float (the
// FP32-everywhere form); the scratch then holds values of type C.
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

// symmetric 3x3 storage: 0:00 1:11 2:22 3:01 4:02 5:12
__device__ __forceinline__ int sidx(int a, int b) {
  return a == b ? a : (a + b == 1 ? 3 : (a + b == 2 ? 4 : 5));
}

template <typename C>
struct LayerGeo {
  C dz[3];
  C hbar;
};

template <typename C>
__device__ __forceinline__ void load_layer(const DevMesh& m, size_t lt, LayerGeo<C>& g) {
  const size_t LS = (size_t)m.n_lslots;
#pragma unroll
  for (int v = 0; v < 3; ++v) g.dz[v] = (C)(m.zl[v * LS + lt] - m.zl[v * LS + lt + kCell]);
  g.hbar = (g.dz[0] + g.dz[1] + g.dz[2]) * (C)(1.0 / 3.0);
}

template <typename C>
__device__ __forceinline__ void vertical_stiffness(const LayerGeo<C>& g, C Jh, C kv[6]) {
#pragma unroll
  for (int i = 0; i < 6; ++i) kv[i] = 0.0;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const C l0 = (C)kL0[q], l1 = (C)kL1[q], l2 = (C)kL2[q];
    const C inv = (C)kTw[q] / (l0 * g.dz[0] + l1 * g.dz[1] + l2 * g.dz[2]);
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

template <typename C>
__device__ __forceinline__ void mass_z(const LayerGeo<C>& g, C Jh, C mz[6]) {
  const C s = Jh * (C)(1.0 / 120.0);
  const C* dz = g.dz;
  mz[0] = s * ((C)3.0 * dz[0] + dz[1] + dz[2]);
  mz[1] = s * (dz[0] + (C)3.0 * dz[1] + dz[2]);
  mz[2] = s * (dz[0] + dz[1] + (C)3.0 * dz[2]);
  mz[3] = s * (dz[0] + dz[1] + (C)0.5 * dz[2]);
  mz[4] = s * (dz[0] + dz[2] + (C)0.5 * dz[1]);
  mz[5] = s * (dz[1] + dz[2] + (C)0.5 * dz[0]);
}

// Scratch entries go in pairs: value pair k of slot p at pair index k * n_slots
// + p, so each lane moves 16 bytes (FP64) per instruction and the
// wavefront's accesses stay contiguous.  Values: E_l row-major (18), then
// y_l field by field (6 each).
template <typename C>
struct alignas(2 * sizeof(C)) CPair {
  C lo, hi;
};

template <typename C>
__device__ __forceinline__ C penalty(C eta, C ka, C kb, C ha, C hb) {
  return eta * (C)0.5 * (ka + kb) / (ha < hb ? ha : hb);
}

// NF = 0: the factor sweep (store E_l only, no back substitution);
// NF > 0: the solve (store y_l only, back substitution with the kept E_l).
template <typename S, typename C, int NF>
__global__ __launch_bounds__(64) void vsolve_kernel(SolveArgs a) {
  const DevMesh& m = a.m;
  const int cell = m.cell_order[blockIdx.x];   // deepest cells first
  const int lane = threadIdx.x;
  const int c = cell * kCell + lane;
  const int N = m.nlay[c];
  if (N == 0) return;

  const size_t SL = (size_t)m.n_slots;
  const size_t p0 = (size_t)m.cell_base[cell] + lane;
  const size_t lt0 = (size_t)m.cell_lbase[cell] + lane;
  const C Jh = (C)m.geo[G_JH * m.n_col_slots + c];
  const C dt = (C)a.dt, eta = (C)a.eta;
  const double* __restrict__ kap = a.kappa;
  // T* and Tout may be the same array (an in-place solve), and the forward
  // sweep writes y_l into Tout: no restrict on either
  const S* Tst = static_cast<const S*>(a.Tstar);
  S* Tout = static_cast<S*>(a.Tout);
  CPair<C>* __restrict__ Psc = reinterpret_cast<CPair<C>*>(a.scratch);   // E_l: pairs 0..8
  CPair<C>* __restrict__ Ysc = Psc + 9 * SL;                              // y_l: pairs 9..9+3NF-1
  constexpr int kNY = 6 * NF;        // y values per slot (even)
  // y_l goes to the output rows (same type), read back and overwritten by x_l
  constexpr bool kYOut = sizeof(S) == sizeof(C);
  const C sd = Jh * (C)(1.0 / 12.0), so = Jh * (C)(1.0 / 24.0);   // M_h diagonal / off-diagonal

  // ---------------- forward sweep ----------------
  // A layer's stage values and the next layer's level heights are loaded
  // one layer ahead (at clamped, always valid slots), before this layer's
  // scratch stores, so their latency is covered by this layer's arithmetic.
  constexpr int kF = NF > 0 ? NF : 1;   // array extent (the factor sweep has no fields)
  auto load_t = [&](int l, C (&t)[kF][6]) {
    const size_t p = p0 + (size_t)l * kCell;
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int i = 0; i < 6; ++i) t[f][i] = (C)Tst[(size_t)(f * 6 + i) * SL + p];
  };
  LayerGeo<C> gc, gn, gpre;
  load_layer(m, lt0, gc);
  load_layer(m, lt0 + (size_t)(N > 1 ? 1 : 0) * kCell, gpre);
  C tpre[kF][6];
  if (NF > 0) load_t(0, tpre);
  C kvp[6], kvc[6];        // Kv of layers l-1 and l
  C Ep[6][3];              // E_{l-1}
  C yp[kF][6];             // y_{l-1}
  C kp = (C)0.0, hp = (C)0.0;    // kappa, hbar of layer l-1
  vertical_stiffness(gc, Jh, kvc);

  for (int l = 0; l < N; ++l) {
    const size_t p = p0 + (size_t)l * kCell;
    const C kc = (C)kap[l];
    const bool below = l < N - 1;
    C t[kF][6];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int i = 0; i < 6; ++i) t[f][i] = tpre[f][i];
    gn = gpre;
    if (NF > 0) load_t(l + 1 < N ? l + 1 : N - 1, tpre);
    load_layer(m, lt0 + (size_t)(l + 2 < N ? l + 2 : N - 1) * kCell, gpre);
    const C kn = below ? (C)kap[l + 1] : (C)0.0;
    C mz[6];
    mass_z(gc, Jh, mz);

    // diagonal block
    C d[6][6];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const C mm = mz[sidx(i, j)], kk = dt * kc * kvc[sidx(i, j)];
        d[i][j] = (C)(2.0 / 3.0) * mm + kk;
        d[i][j + 3] = (C)(1.0 / 3.0) * mm - kk;
        d[i + 3][j] = (C)(1.0 / 3.0) * mm - kk;
        d[i + 3][j + 3] = (C)(2.0 / 3.0) * mm + kk;
      }
    const C sig_u = l > 0 ? penalty(eta, kp, kc, hp, gc.hbar) : (C)0.0;
    const C sig_d = below ? penalty(eta, kc, kn, gc.hbar, gn.hbar) : (C)0.0;
    if (l > 0) {
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const C hk = (C)0.5 * dt * kc * kvc[sidx(i, j)];
          d[i][j] += -hk + dt * sig_u * (i == j ? sd : so);
          d[i][j + 3] += hk;
        }
    }
    if (below) {
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const C hk = (C)0.5 * dt * kc * kvc[sidx(i, j)];
          d[i + 3][j] += hk;
          d[i + 3][j + 3] += -hk + dt * sig_d * (i == j ? sd : so);
        }
    }

    // right-hand sides r = M T*
    C r[kF][6];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        C at = (C)0.0, ab = (C)0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          at += mz[sidx(i, j)] * t[f][j];
          ab += mz[sidx(i, j)] * t[f][j + 3];
        }
        r[f][i] = (C)(2.0 / 3.0) * at + (C)(1.0 / 3.0) * ab;
        r[f][i + 3] = (C)(1.0 / 3.0) * at + (C)(2.0 / 3.0) * ab;
      }
    }

    // Schur complement with the layer above
    if (l > 0) {
      // B_l = dt [-kp Kvp/2 | kp Kvp/2 - sig_u S]  (3 x 6)
      C Bm[3][6];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const C hk = (C)0.5 * dt * kp * kvp[sidx(i, j)];
          Bm[i][j] = -hk;
          Bm[i][j + 3] = hk - dt * sig_u * (i == j ? sd : so);
        }
      // C_{l-1} = dt [kc Kvc/2 - sig_u S | -kc Kvc/2]  (3 x 6)
      C Cm[3][6];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const C hk = (C)0.5 * dt * kc * kvc[sidx(i, j)];
          Cm[i][j] = hk - dt * sig_u * (i == j ? sd : so);
          Cm[i][j + 3] = -hk;
        }
      C P[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          C acc = (C)0.0;
#pragma unroll
          for (int k = 0; k < 6; ++k) acc += Bm[i][k] * Ep[k][j];
          P[i][j] = acc;
        }
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 6; ++j) {
          C acc = (C)0.0;
#pragma unroll
          for (int k = 0; k < 3; ++k) acc += P[i][k] * Cm[k][j];
          d[i][j] -= acc;
        }
#pragma unroll
      for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          C acc = (C)0.0;
#pragma unroll
          for (int k = 0; k < 6; ++k) acc += Bm[i][k] * yp[f][k];
          r[f][i] -= acc;
        }
    }

    // LU of d (no pivoting), in place; the pivots' reciprocals are kept so
    // the triangular solves below multiply instead of divide
    C dinv[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const C inv = (C)1.0 / d[k][k];
      dinv[k] = inv;
#pragma unroll
      for (int i = k + 1; i < 6; ++i) {
        const C li = d[i][k] * inv;
        d[i][k] = li;
#pragma unroll
        for (int j = k + 1; j < 6; ++j) d[i][j] -= li * d[k][j];
      }
    }
    // solve for E = d^-1 e_{3,4,5} and y = d^-1 r
    C Ec[6][3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      C z[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        C acc = (i == q + 3) ? (C)1.0 : (C)0.0;
#pragma unroll
        for (int k = 0; k < i; ++k) acc -= d[i][k] * z[k];
        z[i] = acc;
      }
#pragma unroll
      for (int i = 5; i >= 0; --i) {
        C acc = z[i];
#pragma unroll
        for (int k = i + 1; k < 6; ++k) acc -= d[i][k] * z[k];
        z[i] = acc * dinv[i];
      }
#pragma unroll
      for (int i = 0; i < 6; ++i) Ec[i][q] = z[i];
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      C z[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        C acc = r[f][i];
#pragma unroll
        for (int k = 0; k < i; ++k) acc -= d[i][k] * z[k];
        z[i] = acc;
      }
#pragma unroll
      for (int i = 5; i >= 0; --i) {
        C acc = z[i];
#pragma unroll
        for (int k = i + 1; k < 6; ++k) acc -= d[i][k] * z[k];
        z[i] = acc * dinv[i];
      }
#pragma unroll
      for (int i = 0; i < 6; ++i) yp[f][i] = z[i];
    }
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int q = 0; q < 3; ++q) Ep[i][q] = Ec[i][q];
    if (NF == 0) {
#pragma unroll
      for (int k = 0; k < 9; ++k)
        Psc[(size_t)k * SL + p] = CPair<C>{Ec[(2 * k) / 3][(2 * k) % 3], Ec[(2 * k + 1) / 3][(2 * k + 1) % 3]};
    } else if (kYOut) {
#pragma unroll
      for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int i = 0; i < 6; ++i) Tout[(size_t)(f * 6 + i) * SL + p] = (S)yp[f][i];
    } else {
      C sv[kNY > 0 ? kNY : 2];
#pragma unroll
      for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int i = 0; i < 6; ++i) sv[f * 6 + i] = yp[f][i];
#pragma unroll
      for (int k = 0; k < kNY / 2; ++k) Ysc[(size_t)k * SL + p] = CPair<C>{sv[2 * k], sv[2 * k + 1]};
    }
    // advance the carried layer quantities
#pragma unroll
    for (int i = 0; i < 6; ++i) kvp[i] = kvc[i];
    kp = kc;
    hp = gc.hbar;
    if (below) {
      gc = gn;
      vertical_stiffness(gc, Jh, kvc);
    }
  }

  if (NF == 0) return;

  // ---------------- back substitution ----------------
  // x_{N-1} = y_{N-1} (still in yp)
  C xn[kF][6];
  {
    const size_t p = p0 + (size_t)(N - 1) * kCell;
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        xn[f][i] = yp[f][i];
        Tout[(size_t)(f * 6 + i) * SL + p] = (S)yp[f][i];
      }
  }
  // kvp, kp, hp describe layer N-1 now.  E_l, y_l and the layer's levels
  // are loaded one layer ahead.
  constexpr int kNV = 18 + kNY;
  auto load_sv = [&](int l, C (&sv)[kNV], LayerGeo<C>& g) {
    const size_t p = p0 + (size_t)l * kCell;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const CPair<C> v = Psc[(size_t)k * SL + p];
      sv[2 * k] = v.lo;
      sv[2 * k + 1] = v.hi;
    }
    if (kYOut) {
#pragma unroll
      for (int k = 0; k < kNY; ++k) sv[18 + k] = (C)Tout[(size_t)k * SL + p];
    } else {
#pragma unroll
      for (int k = 0; k < kNY / 2; ++k) {
        const CPair<C> v = Ysc[(size_t)k * SL + p];
        sv[18 + 2 * k] = v.lo;
        sv[18 + 2 * k + 1] = v.hi;
      }
    }
    load_layer(m, lt0 + (size_t)l * kCell, g);
  };
  C svpre[kNV];
  LayerGeo<C> glpre;
  load_sv(N > 1 ? N - 2 : 0, svpre, glpre);
  for (int l = N - 2; l >= 0; --l) {
    const size_t p = p0 + (size_t)l * kCell;
    C sv[kNV];
#pragma unroll
    for (int k = 0; k < kNV; ++k) sv[k] = svpre[k];
    const LayerGeo<C> gl = glpre;
    load_sv(l > 0 ? l - 1 : 0, svpre, glpre);
    const C kl = (C)kap[l];
    const C sig_d = penalty(eta, kl, kp, gl.hbar, hp);
    // C_l = dt [kp Kv_{l+1}/2 - sig_d S | -kp Kv_{l+1}/2]
    C Cm[3][6];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const C hk = (C)0.5 * dt * kp * kvp[sidx(i, j)];
        Cm[i][j] = hk - dt * sig_d * (i == j ? sd : so);
        Cm[i][j + 3] = -hk;
      }
    C E[6][3];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int q = 0; q < 3; ++q) E[i][q] = sv[i * 3 + q];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      C cx[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        C acc = (C)0.0;
#pragma unroll
        for (int j = 0; j < 6; ++j) acc += Cm[i][j] * xn[f][j];
        cx[i] = acc;
      }
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        xn[f][i] = sv[18 + f * 6 + i] - (E[i][0] * cx[0] + E[i][1] * cx[1] + E[i][2] * cx[2]);
      }
    }
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int i = 0; i < 6; ++i) Tout[(size_t)(f * 6 + i) * SL + p] = (S)xn[f][i];
    vertical_stiffness(gl, Jh, kvp);
    kp = kl;
    hp = gl.hbar;
  }
}

template <typename S, typename C>
hipError_t launch_s(const SolveArgs& a, bool factor, hipStream_t s) {
  dim3 grid(a.m.n_cells), block(kCell);
  if (factor) {
    hipLaunchKernelGGL((vsolve_kernel<S, C, 0>), grid, block, 0, s, a);
    return hipGetLastError();
  }
  switch (a.n_fields) {
    case 1: hipLaunchKernelGGL((vsolve_kernel<S, C, 1>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((vsolve_kernel<S, C, 2>), grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL((vsolve_kernel<S, C, 3>), grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL((vsolve_kernel<S, C, 4>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_vsolve(const SolveArgs& a, bool fp32_state, bool fp32_solve, bool factor, hipStream_t s) {
  if (a.m.n_cells == 0) return hipSuccess;
  if (!fp32_state) return launch_s<double, double>(a, factor, s);
  return fp32_solve ? launch_s<float, float>(a, factor, s) : launch_s<float, double>(a, factor, s);
}

}  // namespace sdg
