// Kernels of the ULV-like factorization (Alg. 3) and solve (Alg. 4): the
// generators' V^T at the leaves, 64-wide triangular block solves with many
// right-hand sides, application of the LQ reflectors, and the partial-pivoting
// LU of the root block (panel factorization and row interchanges; the
// trailing updates run on the batched GEMM).
#include <climits>
#include <cmath>

#include "hss_internal.h"
#include "hss_ulv_kernels.h"

namespace hss {
namespace {

constexpr int NT = 256;

// V^T of a leaf as rows of Z: Z[a][J[a]] = 1, Z[a][rest[j]] = E[j][a].
__global__ __launch_bounds__(NT) void vt_leaf_kernel(const VtLeafDesc* __restrict__ d) {
  const VtLeafDesc g = d[blockIdx.y];
  const int a = blockIdx.x;
  if (a >= g.k) return;
  double* row = g.Z + (long long)a * g.ldz;
  for (int c = threadIdx.x; c < g.m; c += NT) row[c] = 0.0;
  __syncthreads();
  if (threadIdx.x == 0) row[g.perm[a]] = 1.0;
  for (int j = threadIdx.x; j < g.m - g.k; j += NT) row[g.perm[g.k + j]] = g.E[(long long)j * g.k + a];
}

// One diagonal block of a triangular solve, in place on X (nb rows, nrhs
// columns): lower: X = T^{-1} X with T lower triangular (unit diagonal if
// unit); upper: likewise with T upper triangular.  One workgroup per problem;
// each thread owns right-hand-side columns.
__global__ __launch_bounds__(NT) void tri_block_kernel(const TriDesc* __restrict__ d) {
  __shared__ double T[64][65];
  const TriDesc g = d[blockIdx.x];
  const int nb = g.nb;
  for (int e = threadIdx.x; e < nb * nb; e += NT) {
    const int r = e / nb, c = e % nb;
    T[r][c] = g.T[(long long)r * g.ldt + c];
  }
  __syncthreads();
  for (int col = threadIdx.x; col < g.nrhs; col += NT) {
    double x[64];
#pragma unroll
    for (int r = 0; r < 64; ++r) x[r] = (r < nb) ? g.X[(long long)r * g.ldx + col] : 0.0;
    if (g.lower) {
#pragma unroll
      for (int r = 0; r < 64; ++r) {
        if (r < nb) {
          double s = x[r];
#pragma unroll
          for (int c = 0; c < 64; ++c)
            if (c < r) s = fma(-T[r][c], x[c], s);
          x[r] = g.unit ? s : s / T[r][r];
        }
      }
    } else {
#pragma unroll
      for (int r = 63; r >= 0; --r) {
        if (r < nb) {
          double s = x[r];
#pragma unroll
          for (int c = 0; c < 64; ++c)
            if (c > r && c < nb) s = fma(-T[r][c], x[c], s);
          x[r] = g.unit ? s : s / T[r][r];
        }
      }
    }
#pragma unroll
    for (int r = 0; r < 64; ++r)
      if (r < nb) g.X[(long long)r * g.ldx + col] = x[r];
  }
}

// v <- H_0 H_1 ... H_{r-1} v (transpose = 1, i.e. Q^T v) or
// v <- H_{r-1} ... H_0 v (transpose = 0, Q v) with H_i = I - tau_i u_i u_i^T,
// u_i = (1, Z[i][i+1..m-1]).  One workgroup per problem; every wavefront
// handles right-hand-side columns.
__global__ __launch_bounds__(NT) void reflect_kernel(const ReflDesc* __restrict__ d) {
  const ReflDesc g = d[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int col = wave; col < g.nrhs; col += NT / 64) {
    for (int s = 0; s < g.r; ++s) {
      const int i = g.transpose ? g.r - 1 - s : s;
      const double* u = g.Z + (long long)i * g.ldz;
      double dot = 0.0;
      for (int q = i + lane; q < g.m; q += 64) {
        const double ui = (q == i) ? 1.0 : u[q];
        dot = fma(ui, g.V[(long long)q * g.ldv + col], dot);
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) dot += __shfl_xor(dot, o, 64);
      const double f = g.tau[i] * dot;
      for (int q = i + lane; q < g.m; q += 64) {
        const double ui = (q == i) ? 1.0 : u[q];
        g.V[(long long)q * g.ldv + col] = fma(-f, ui, g.V[(long long)q * g.ldv + col]);
      }
    }
  }
}

// Unblocked partial-pivoting LU of the panel A[j0:n, j0:j0+nb] (row-major,
// ld), one workgroup.  Pivot rows are chosen by largest magnitude (lowest
// index on ties) and swapped inside the panel; piv[j0 + c] = absolute row
// chosen for column j0 + c.  info is set to the first zero pivot (1-based) or
// left untouched.
__global__ __launch_bounds__(1024) void lu_panel_kernel(double* __restrict__ A, long long ld, int n,
                                                       int j0, int nb, int* __restrict__ piv,
                                                       int* __restrict__ info) {
  __shared__ double rv[16];
  __shared__ int ri[16];
  __shared__ int s_p;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int c = 0; c < nb; ++c) {
    const int col = j0 + c;
    double bv = -1.0;
    int bi = INT_MAX;
    for (int r = col + tid; r < n; r += 1024) {
      const double v = fabs(A[(long long)r * ld + col]);
      if (v > bv) {
        bv = v;
        bi = r;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(bv, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ov > bv || (ov == bv && oi < bi)) {
        bv = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      rv[wave] = bv;
      ri[wave] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      double v = rv[0];
      int ix = ri[0];
      for (int q = 1; q < 16; ++q)
        if (rv[q] > v || (rv[q] == v && ri[q] < ix)) {
          v = rv[q];
          ix = ri[q];
        }
      s_p = ix;
      piv[col] = ix;
      if (!(v > 0.0) && *info == 0) *info = col + 1;
    }
    __syncthreads();
    const int p = s_p;
    if (p != col) {
      for (int q = j0 + tid; q < j0 + nb; q += 1024) {
        const double t = A[(long long)col * ld + q];
        A[(long long)col * ld + q] = A[(long long)p * ld + q];
        A[(long long)p * ld + q] = t;
      }
    }
    __syncthreads();
    const double d = A[(long long)col * ld + col];
    const double inv = (d != 0.0) ? 1.0 / d : 0.0;
    for (int r = col + 1 + tid; r < n; r += 1024) {
      double* ar = A + (long long)r * ld;
      const double l = ar[col] * inv;
      ar[col] = l;
      for (int q = col + 1; q < j0 + nb; ++q) ar[q] = fma(-l, A[(long long)col * ld + q], ar[q]);
    }
    __syncthreads();
  }
}

// Row interchanges of the panel's pivots applied to the columns outside
// [j0, j0+nb) (or to a right-hand side with cols = its width, c_skip0 = 0,
// c_skip1 = 0).  Sequential over the pivots, parallel over columns.
__global__ __launch_bounds__(NT) void lu_swap_kernel(double* __restrict__ A, long long ld, int ncols,
                                                    const int* __restrict__ piv, int j0, int nb,
                                                    int skip0, int skip1) {
  const int c = blockIdx.x * NT + threadIdx.x;
  if (c >= ncols || (c >= skip0 && c < skip1)) return;
  for (int q = j0; q < j0 + nb; ++q) {
    const int p = piv[q];
    if (p != q) {
      const double t = A[(long long)q * ld + c];
      A[(long long)q * ld + c] = A[(long long)p * ld + c];
      A[(long long)p * ld + c] = t;
    }
  }
}

}  // namespace

hipError_t launch_vt_leaf(const VtLeafDesc* d, int nd, int kmax, Staging& st, hipStream_t s) {
  if (nd <= 0 || kmax <= 0) return hipSuccess;
  const VtLeafDesc* dd = static_cast<const VtLeafDesc*>(st.push(d, sizeof(VtLeafDesc) * nd));
  if (!dd) return hipErrorOutOfMemory;
  hipLaunchKernelGGL(vt_leaf_kernel, dim3(kmax, nd), dim3(NT), 0, s, dd);
  return hipGetLastError();
}

hipError_t launch_tri_block(const TriDesc* d, int nd, Staging& st, hipStream_t s) {
  if (nd <= 0) return hipSuccess;
  const TriDesc* dd = static_cast<const TriDesc*>(st.push(d, sizeof(TriDesc) * nd));
  if (!dd) return hipErrorOutOfMemory;
  hipLaunchKernelGGL(tri_block_kernel, dim3(nd), dim3(NT), 0, s, dd);
  return hipGetLastError();
}

hipError_t launch_reflect(const ReflDesc* d, int nd, Staging& st, hipStream_t s) {
  if (nd <= 0) return hipSuccess;
  const ReflDesc* dd = static_cast<const ReflDesc*>(st.push(d, sizeof(ReflDesc) * nd));
  if (!dd) return hipErrorOutOfMemory;
  hipLaunchKernelGGL(reflect_kernel, dim3(nd), dim3(NT), 0, s, dd);
  return hipGetLastError();
}

hipError_t launch_lu_panel(double* A, long long ld, int n, int j0, int nb, int* piv, int* info,
                           hipStream_t s) {
  hipLaunchKernelGGL(lu_panel_kernel, dim3(1), dim3(1024), 0, s, A, ld, n, j0, nb, piv, info);
  return hipGetLastError();
}

hipError_t launch_lu_swap(double* A, long long ld, int ncols, const int* piv, int j0, int nb,
                          int skip0, int skip1, hipStream_t s) {
  if (ncols <= 0 || nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(lu_swap_kernel, dim3((ncols + NT - 1) / NT), dim3(NT), 0, s, A, ld, ncols, piv,
                     j0, nb, skip0, skip1);
  return hipGetLastError();
}

}  // namespace hss
