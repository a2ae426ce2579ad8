// Matrix-free column solvers of the two vertical-derivative systems of the
// paper's section 2.3: D_vu x = F (the horizontal pressure gradient system,
// integrated from the surface down) and D_vd x = F (the vertical velocity
// system, integrated from the seabed up).
//
// Derivation from the printed block rows.  Both matrices are (1/2) P (x) M_h
// with P a pattern of small integers and M_h = J_h/24 [2 1 1; 1 2 1; 1 1 2],
// so D x = F is P x = 2 f per node triple with f = M_h^-1 F, and
// M_h^-1 F_i = (6/J_h) (4 F_i - (F_0 + F_1 + F_2)).  Per layer l, with t and b
// the top- and bottom-face node triples:
//   D_vu:  x_t(l) - x_b(l) = 2 f_b(l)  and  2 x_b(l-1) - x_t(l) - x_b(l) = 2 f_t(l),
//          hence x_b(l) = x_b(l-1) - (f_t(l) + f_b(l)) from x_b(-1) = 0 at the
//          surface, and x_t(l) = x_b(l) + 2 f_b(l);
//   D_vd:  x_t(l) - x_b(l) = 2 f_t(l)  and  x_t(l) + x_b(l) - 2 x_t(l+1) = 2 f_b(l),
//          hence x_t(l) = x_t(l+1) + (f_t(l) + f_b(l)) from x_t(N) = 0 at the
//          seabed, and x_b(l) = x_t(l) - 2 f_t(l).
// Each lane carries one value per node of its column: the solution on the
// face the sweep crosses into the next layer (x_b going down, x_t going up).
//
// One wavefront per cell, one lane per column: every layer's six values per
// component are six coalesced 64-wide loads.  The loads do not depend on the
// carried value, so the loop keeps kAhead layers in flight ahead of the one it
// finishes.  Values are read before they are written, by the same lane, so F
// and x may be the same buffer.
#include "internal.h"

namespace sdg {
namespace {

// Layers loaded ahead of the one being finished: about 48 loads in flight per
// wavefront whatever the component count.
constexpr int ahead_layers(int nc) { return nc >= 4 ? 2 : 8 / nc; }

template <typename T, int NC>
struct Layer {
  T v[NC][6];
};

// Load one layer of the column (zeros where the lane's column has no such layer).
template <typename T, int NC>
__device__ __forceinline__ void load_layer(Layer<T, NC>& L, const T* F, size_t SL, int64_t slot, bool live) {
#pragma unroll
  for (int k = 0; k < NC; ++k)
#pragma unroll
    for (int a = 0; a < 6; ++a) L.v[k][a] = live ? F[(k * 6 + a) * SL + slot] : (T)0;
}

template <typename T, typename C, int NC, bool DOWN>
__global__ __launch_bounds__(64) void column_dv_kernel(DevMesh m, const T* F, T* X, const C* jh) {
  const int cell = blockIdx.x;
  const int lane = threadIdx.x;
  const int c = cell * kCell + lane;
  const int N = m.nlay[c];
  const int64_t base = (int64_t)m.cell_base[cell] + lane;
  const int D = (m.cell_base[cell + 1] - m.cell_base[cell]) / kCell;   // deepest column of the cell
  const size_t SL = (size_t)m.n_slots;
  const C minv = N > 0 ? (C)6 / jh[c] : (C)0;

  // traversal step i visits layer i (DOWN) or D-1-i (up)
  auto layer_of = [&](int i) { return DOWN ? i : D - 1 - i; };

  constexpr int kAhead = ahead_layers(NC);
  Layer<T, NC> q[kAhead];
#pragma unroll
  for (int i = 0; i < kAhead; ++i) {
    const int l = layer_of(i);
    load_layer(q[i], F, SL, base + (int64_t)l * kCell, i < D && l < N);
  }

  // solution on the face shared with the previously visited layer (zero at
  // the surface for D_vu, at the seabed for D_vd)
  C xf[NC][3];
#pragma unroll
  for (int k = 0; k < NC; ++k)
#pragma unroll
    for (int n = 0; n < 3; ++n) xf[k][n] = (C)0;

  for (int i0 = 0; i0 < D; i0 += kAhead) {
#pragma unroll
    for (int j = 0; j < kAhead; ++j) {
      const int i = i0 + j;
      if (i >= D) break;
      const int l = layer_of(i);
      const Layer<T, NC> cur = q[j];
      const int ip = i + kAhead;
      const int lp = layer_of(ip);
      if (ip < D) load_layer(q[j], F, SL, base + (int64_t)lp * kCell, lp < N);
      if (l < N) {
        const int64_t slot = base + (int64_t)l * kCell;
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          C v[6];
#pragma unroll
          for (int a = 0; a < 6; ++a) v[a] = (C)cur.v[k][a];
          const C st = v[0] + v[1] + v[2];
          const C sb = v[3] + v[4] + v[5];
#pragma unroll
          for (int n = 0; n < 3; ++n) {
            const C ft = minv * ((C)4 * v[n] - st);
            const C fb = minv * ((C)4 * v[3 + n] - sb);
            C xt, xb;
            if (DOWN) {
              xb = xf[k][n] - (ft + fb);
              xt = xb + (C)2 * fb;
              xf[k][n] = xb;
            } else {
              xt = xf[k][n] + (ft + fb);
              xb = xt - (C)2 * ft;
              xf[k][n] = xt;
            }
            X[(k * 6 + n) * SL + slot] = (T)xt;
            X[(k * 6 + 3 + n) * SL + slot] = (T)xb;
          }
        }
      }
    }
  }
}

template <typename T, typename C, bool DOWN>
hipError_t launch_typed(const DevMesh& m, int nc, const void* F, void* X, const C* jh, hipStream_t s) {
  const T* f = static_cast<const T*>(F);
  T* x = static_cast<T*>(X);
  const dim3 grid(m.n_cells), block(kCell);
  switch (nc) {
    case 1: column_dv_kernel<T, C, 1, DOWN><<<grid, block, 0, s>>>(m, f, x, jh); break;
    case 2: column_dv_kernel<T, C, 2, DOWN><<<grid, block, 0, s>>>(m, f, x, jh); break;
    case 3: column_dv_kernel<T, C, 3, DOWN><<<grid, block, 0, s>>>(m, f, x, jh); break;
    case 4: column_dv_kernel<T, C, 4, DOWN><<<grid, block, 0, s>>>(m, f, x, jh); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_column_dv(const DevMesh& m, bool down, int n_comp, const void* F, void* X, bool fp32_state,
                            bool fp32_arith, hipStream_t s) {
  if (m.n_cells == 0) return hipSuccess;
  const double* jh = m.geo + (size_t)G_JH * m.n_col_slots;
  const float* jh32 = m.geo32 + (size_t)G_JH * m.n_col_slots;
  if (!fp32_state) {
    return down ? launch_typed<double, double, true>(m, n_comp, F, X, jh, s)
                : launch_typed<double, double, false>(m, n_comp, F, X, jh, s);
  }
  if (fp32_arith) {
    return down ? launch_typed<float, float, true>(m, n_comp, F, X, jh32, s)
                : launch_typed<float, float, false>(m, n_comp, F, X, jh32, s);
  }
  return down ? launch_typed<float, double, true>(m, n_comp, F, X, jh, s)
              : launch_typed<float, double, false>(m, n_comp, F, X, jh, s);
}

}  // namespace sdg
