// Setup and diagnostic kernels: per-column geometry, FP32 copies of the
// levels, mass sums (fixed-order, deterministic) and a non-finite check.
#include "internal.h"

namespace sdg {
namespace {

// Per column: map derivatives, J_h = 2 * area, outward unit normals and
// lengths of the three edges (edge k runs from vertex k to vertex k+1).
__global__ __launch_bounds__(256) void geometry_kernel(DevMesh m, double* geo, float* geo32) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int CS = m.n_col_slots;
  if (c >= CS) return;
  double g[kGeoRows];
#pragma unroll
  for (int r = 0; r < kGeoRows; ++r) g[r] = 0.0;
  if (m.nlay[c] > 0) {
    double x[3], y[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      x[v] = m.xy[(2 * v) * CS + c];
      y[v] = m.xy[(2 * v + 1) * CS + c];
    }
    g[G_XXI] = x[1] - x[0];
    g[G_XET] = x[2] - x[0];
    g[G_YXI] = y[1] - y[0];
    g[G_YET] = y[2] - y[0];
    g[G_JH] = g[G_XXI] * g[G_YET] - g[G_XET] * g[G_YXI];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const int b = (e + 1) % 3;
      const double dx = x[b] - x[e], dy = y[b] - y[e];
      const double len = sqrt(dx * dx + dy * dy);
      g[G_NX + e] = dy / len;
      g[G_NY + e] = -dx / len;
      g[G_LE + e] = len;
    }
  }
#pragma unroll
  for (int r = 0; r < kGeoRows; ++r) {
    geo[r * CS + c] = g[r];
    geo32[r * CS + c] = (float)g[r];
  }
}

__global__ __launch_bounds__(256) void to_float_kernel(const double* src, float* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

// Per column and field: sum over layers of 1^T M T.  1^T M = [w w] with
// w_b = sum_a Mz_ab = J_h (2 dz_b + dz_others) / 48.
template <typename R>
__global__ __launch_bounds__(64) void column_mass_kernel(DevMesh m, const R* T, int nf, double* out) {
  const int cell = blockIdx.x;
  const int lane = threadIdx.x;
  const int c = cell * kCell + lane;
  const int N = m.nlay[c];
  const int CS = m.n_col_slots;
  const size_t SL = (size_t)m.n_slots, LS = (size_t)m.n_lslots;
  double acc[kMaxFields] = {0.0, 0.0, 0.0, 0.0};
  if (N > 0) {
    const double Jh = m.geo[G_JH * CS + c];
    for (int l = 0; l < N; ++l) {
      const size_t p = (size_t)m.cell_base[cell] + (size_t)l * kCell + lane;
      const size_t lt = (size_t)m.cell_lbase[cell] + (size_t)l * kCell + lane;
      double dz[3];
#pragma unroll
      for (int v = 0; v < 3; ++v) dz[v] = m.zl[v * LS + lt] - m.zl[v * LS + lt + kCell];
      const double s = dz[0] + dz[1] + dz[2];
      for (int f = 0; f < nf; ++f) {
        double sum = 0.0;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          const double wb = Jh * (dz[b] + s) * (1.0 / 48.0);
          sum += wb * ((double)T[(size_t)(f * 6 + b) * SL + p] + (double)T[(size_t)(f * 6 + b + 3) * SL + p]);
        }
        acc[f] += sum;
      }
    }
  }
  for (int f = 0; f < nf; ++f) out[(size_t)f * CS + c] = acc[f];
}

// One block per (member, field): each thread sums a fixed strided subset of
// the member's columns, then a fixed tree in LDS.
__global__ __launch_bounds__(256) void member_sum_kernel(const double* colm, int CS, int nf,
                                                         const int32_t* moff, double* out) {
  const int mem = blockIdx.x / nf, f = blockIdx.x % nf;
  __shared__ double red[256];
  double acc = 0.0;
  for (int c = moff[mem] + threadIdx.x; c < moff[mem + 1]; c += 256) acc += colm[(size_t)f * CS + c];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// Live slots only: padding slots of caller buffers are never inspected.
template <typename R>
__global__ __launch_bounds__(64) void finite_kernel(DevMesh m, const R* T, int nf, int32_t* flag) {
  const int cell = blockIdx.x;
  const int c = cell * kCell + threadIdx.x;
  const int N = m.nlay[c];
  const size_t SL = (size_t)m.n_slots;
  bool bad = false;
  for (int l = 0; l < N; ++l) {
    const size_t p = (size_t)m.cell_base[cell] + (size_t)l * kCell + threadIdx.x;
    for (int k = 0; k < 6 * nf; ++k) bad |= !isfinite(T[(size_t)k * SL + p]);
  }
  if (bad) flag[0] = 1;
}

__global__ void clear_kernel(int32_t* flag) { flag[0] = 0; }

}  // namespace

hipError_t launch_geometry(const DevMesh& m, double* geo, float* geo32, hipStream_t s) {
  const int n = m.n_col_slots;
  hipLaunchKernelGGL(geometry_kernel, dim3((n + 255) / 256), dim3(256), 0, s, m, geo, geo32);
  return hipGetLastError();
}

hipError_t launch_z32(const DevMesh& m, float* zl32, hipStream_t s) {
  const int64_t n = 3 * m.n_lslots;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(to_float_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, m.zl, zl32, n);
  return hipGetLastError();
}

hipError_t launch_column_mass(const DevMesh& m, const void* T, int n_fields, bool fp32,
                              double* col_mass, hipStream_t s) {
  if (fp32)
    hipLaunchKernelGGL(column_mass_kernel<float>, dim3(m.n_cells), dim3(kCell), 0, s, m,
                       static_cast<const float*>(T), n_fields, col_mass);
  else
    hipLaunchKernelGGL(column_mass_kernel<double>, dim3(m.n_cells), dim3(kCell), 0, s, m,
                       static_cast<const double*>(T), n_fields, col_mass);
  return hipGetLastError();
}

hipError_t launch_member_sum(const double* col_mass, int n_col_slots, int n_fields,
                             const int32_t* member_off, int n_members, double* out,
                             hipStream_t s) {
  hipLaunchKernelGGL(member_sum_kernel, dim3(n_members * n_fields), dim3(256), 0, s, col_mass,
                     n_col_slots, n_fields, member_off, out);
  return hipGetLastError();
}

hipError_t launch_finite_check(const DevMesh& m, const void* T, int n_fields, bool fp32,
                               int32_t* flag, hipStream_t s) {
  hipLaunchKernelGGL(clear_kernel, dim3(1), dim3(1), 0, s, flag);
  if (fp32)
    hipLaunchKernelGGL(finite_kernel<float>, dim3(m.n_cells), dim3(kCell), 0, s, m,
                       static_cast<const float*>(T), n_fields, flag);
  else
    hipLaunchKernelGGL(finite_kernel<double>, dim3(m.n_cells), dim3(kCell), 0, s, m,
                       static_cast<const double*>(T), n_fields, flag);
  return hipGetLastError();
}

}  // namespace sdg
