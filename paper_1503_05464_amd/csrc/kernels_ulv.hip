// Kernels of the ULV-like factorization (Alg. 3) and solve (Alg. 4): the
// generators' V^T at the leaves, 64-wide triangular block solves with many
// right-hand sides, the dense reflector matrix and block triangular factors
// of the compact WY form of the LQ reflectors, and the partial-pivoting
// LU of the root block (panel factorization and row interchanges; the
// trailing updates run on the batched GEMM).
#include <climits>
#include <cmath>

#include "hss_internal.h"
#include "hss_ulv_kernels.h"

namespace hss {
namespace {

constexpr int NT = 256;
// widest batch of right-hand sides solved by tri_wave_kernel
constexpr int kTriWaveMaxRhs = 64;

// Wavefront argmax of (|value|, row) for the pivot search: the larger value,
// the lower row on ties.  Butterfly of four DPP levels (quad permutes, then
// half-row and row mirrors) and two cross-row shuffles; the order is total,
// so every lane ends with the same pair.
template <int CTRL>
__device__ __forceinline__ int piv_dpp(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double piv_dpp_d(double v) {
  return __hiloint2double(piv_dpp<CTRL>(__double2hiint(v)), piv_dpp<CTRL>(__double2loint(v)));
}
__device__ __forceinline__ void piv_better(double& bv, int& bi, double ov, int oi) {
  if (ov > bv || (ov == bv && oi < bi)) {
    bv = ov;
    bi = oi;
  }
}
__device__ __forceinline__ void pivot_argmax(double& bv, int& bi) {
  piv_better(bv, bi, piv_dpp_d<0xB1>(bv), piv_dpp<0xB1>(bi));
  piv_better(bv, bi, piv_dpp_d<0x4E>(bv), piv_dpp<0x4E>(bi));
  piv_better(bv, bi, piv_dpp_d<0x141>(bv), piv_dpp<0x141>(bi));
  piv_better(bv, bi, piv_dpp_d<0x140>(bv), piv_dpp<0x140>(bi));
  piv_better(bv, bi, __shfl_xor(bv, 16, 64), __shfl_xor(bi, 16, 64));
  piv_better(bv, bi, __shfl_xor(bv, 32, 64), __shfl_xor(bi, 32, 64));
}

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
// unit); upper: likewise with T upper triangular.  One workgroup per problem
// and block of NT right-hand-side columns (grid y); each thread owns one
// column, all NB rows of it in registers.  The LDS copy of T is padded to
// NB x NB with the identity, so the padded rows solve to zero and the
// unrolled loops need no test against nb: with one, the compiler kept the
// column in scratch memory.  NB is 64, or 32 when every block of the launch
// has at most 32 rows (the root LU's panels): half the steps and registers.
template <int NB>
__global__ __launch_bounds__(NT) void tri_block_kernel(const TriDesc* __restrict__ d) {
  __shared__ double T[NB][NB + 1];
  const TriDesc g = d[blockIdx.x];
  const int nb = g.nb;
  const int cbeg = blockIdx.y * NT;
  if (cbeg >= g.nrhs) return;
  for (int e = threadIdx.x; e < NB * NB; e += NT) {  // a unit diagonal is stored as 1: s / 1 = s exactly
    const int r = e / NB, c = e % NB;
    T[r][c] = (r < nb && c < nb && !(g.unit && r == c)) ? g.T[(long long)r * g.ldt + c] : (r == c ? 1.0 : 0.0);
  }
  __syncthreads();
  const int col = cbeg + threadIdx.x;
  if (col >= g.nrhs) return;
  double x[NB];
#pragma unroll
  for (int r = 0; r < NB; ++r) {  // rows past nb read row 0 and are zeroed
    const double v = g.X[(long long)(r < nb ? r : 0) * g.ldx + col];
    x[r] = r < nb ? v : 0.0;
  }
  // column by column: once x[c] is final, the updates of the other rows are
  // independent of each other
  if (g.lower) {
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      x[c] = x[c] / T[c][c];
#pragma unroll
      for (int r = c + 1; r < NB; ++r) x[r] = fma(-T[r][c], x[c], x[r]);
    }
  } else {
#pragma unroll
    for (int c = NB - 1; c >= 0; --c) {
      x[c] = x[c] / T[c][c];
#pragma unroll
      for (int r = 0; r < c; ++r) x[r] = fma(-T[r][c], x[c], x[r]);
    }
  }
#pragma unroll
  for (int r = 0; r < NB; ++r)
    if (r < nb) g.X[(long long)r * g.ldx + col] = x[r];
}

// The value lane l of the wavefront holds, in every lane (l uniform).
__device__ __forceinline__ double lane_bcast(double v, int l) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The same block solve for few right-hand sides: one wavefront per column,
// lane r holding x[r].  Column c of T is applied once x[c] is final, which
// is then read from its lane by all others, so a column takes nb dependent
// steps across the wavefront instead of nb^2 / 2 in one thread (the
// arithmetic, and so the rounding, is that of the kernel above).  Four
// columns per workgroup (grid y).
__global__ __launch_bounds__(NT) void tri_wave_kernel(const TriDesc* __restrict__ d) {
  __shared__ double T[64][65];
  constexpr int CPB = NT / 64;
  const TriDesc g = d[blockIdx.x];
  const int nb = g.nb;
  if ((int)blockIdx.y * CPB >= g.nrhs) return;
  for (int e = threadIdx.x; e < 64 * 64; e += NT) {
    const int r = e >> 6, c = e & 63;
    T[r][c] = (r < nb && c < nb && !(g.unit && r == c)) ? g.T[(long long)r * g.ldt + c] : (r == c ? 1.0 : 0.0);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int col = blockIdx.y * CPB + (threadIdx.x >> 6);
  if (col >= g.nrhs) return;
  double* xp = g.X + (long long)(lane < nb ? lane : 0) * g.ldx + col;
  double x = lane < nb ? *xp : 0.0;
  if (g.lower) {
    for (int c = 0; c < nb; ++c) {
      const double xc = lane_bcast(x, c) / T[c][c];
      x = lane == c ? xc : (lane > c ? fma(-T[lane][c], xc, x) : x);
    }
  } else {
    for (int c = nb - 1; c >= 0; --c) {
      const double xc = lane_bcast(x, c) / T[c][c];
      x = lane == c ? xc : (lane < c ? fma(-T[lane][c], xc, x) : x);
    }
  }
  if (lane < nb) *xp = x;
}

// Y = [u_0 .. u_{r-1}] (m x r, row-major, ld r) with u_i = (0.., 1, Z[i][i+1..m-1]):
// 64 x 64 tiles transposed through LDS, so both Z rows and Y rows are read
// and written contiguously.  grid: (ceil(m/64) * ceil(rmax/64), problems).
__global__ __launch_bounds__(NT) void refl_y_kernel(const ReflYDesc* __restrict__ d) {
  __shared__ double tile[64][65];
  const ReflYDesc g = d[blockIdx.y];
  const int tq = (g.m + 63) / 64, ti = (g.r + 63) / 64;
  if ((int)blockIdx.x >= tq * ti) return;
  const int q0 = (blockIdx.x % tq) * 64, i0 = (blockIdx.x / tq) * 64;
  // read: rows i of Z (reflector i), columns q
  for (int e = threadIdx.x; e < 64 * 64; e += NT) {
    const int il = e / 64, ql = e % 64;
    const int i = i0 + il, q = q0 + ql;
    double v = 0.0;
    if (i < g.r && q < g.m) v = (q < i) ? 0.0 : (q == i ? 1.0 : g.Z[(long long)i * g.ldz + q]);
    tile[il][ql] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += NT) {
    const int ql = e / 64, il = e % 64;
    const int i = i0 + il, q = q0 + ql;
    if (i < g.r && q < g.m) g.Y[(long long)q * g.r + i] = tile[il][ql];
  }
}

// out = the sum of `parts` partial products (rows x cols, ld cols, `stride`
// apart), added in the order of the parts: the second stage of a product
// whose long inner dimension was split over workgroups.  One thread per
// output element; grid (element blocks, problems).
__global__ __launch_bounds__(NT) void sum_partials_kernel(const SumDesc* __restrict__ d) {
  const SumDesc g = d[blockIdx.y];
  const int e = blockIdx.x * NT + threadIdx.x;
  if (e >= g.rows * g.cols) return;
  const int r = e / g.cols, c = e % g.cols;
  double v = 0.0;
  for (int q = 0; q < g.parts; ++q) v += g.part[q * g.stride + (long long)r * g.cols + c];
  g.out[(long long)r * g.ldo + c] = v;
}

// Forward triangular factor of a block of kb reflectors, H_0 ... H_{kb-1} =
// I - Y T Y^T: T[j][j] = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] G[0:j, j] with
// G = Y^T Y.  One workgroup of 64 threads per block; thread l owns row l.
// G and tau are staged in LDS first (rows of G read contiguously), so the
// serial recurrence reads LDS only; T is upper triangular and zero below the
// diagonal, so every thread sums over all p < j and the loop is uniform.
__global__ __launch_bounds__(64) void larft_kernel(const LarftDesc* __restrict__ d) {
  __shared__ double T[64][65];
  __shared__ double G[64][65];
  __shared__ double tau[64];
  const LarftDesc g = d[blockIdx.x];
  const int l = threadIdx.x, kb = g.kb;
  for (int r = 0; r < kb; ++r) G[r][l] = l < kb ? g.G[(long long)r * 64 + l] : 0.0;
  tau[l] = l < kb ? g.tau[l] : 0.0;
  for (int c = 0; c < 64; ++c) T[l][c] = 0.0;
  __syncthreads();
  for (int j = 0; j < kb; ++j) {
    double s = 0.0;
    for (int p = 0; p < j; ++p) s = fma(T[l][p], G[p][j], s);
    __syncthreads();
    if (l < j) T[l][j] = -tau[j] * s;
    if (l == j) T[j][j] = tau[j];
    __syncthreads();
  }
  if (l < kb)
    for (int c = 0; c < kb; ++c) g.T[(long long)l * 64 + c] = T[l][c];
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
    pivot_argmax(bv, bi);
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

// The same panel factorization with the panel's rows split over NTH threads
// (thread t owns rows j0 + t + NTH k, k < R; panels of at most 512 rows take
// 256 threads: 184 against about 300 us per 64-column panel of 230 rows,
// while 128 and 64 threads were slower again) and the columns taken
// eight at a time: a sub-panel of 8 columns lives in registers while its
// pivots are chosen (largest magnitude, lowest row on ties), its rows are
// interchanged (through LDS, and in global memory for the panel's other
// columns) and its multipliers are applied; then the panel's columns to the
// right get the 8 rows of U (a unit-lower solve) and the rank-8 update of
// the rows below, with the multipliers still in registers.
constexpr int LW = 8;  // sub-panel width

template <int R, int NTH = 1024>
__global__ __launch_bounds__(NTH) void lu_panel_reg_kernel(double* __restrict__ A, long long ld, int n,
                                                          int j0, int nb, int* __restrict__ piv,
                                                          int* __restrict__ info) {
  constexpr int NW = NTH / 64;  // wavefronts
  __shared__ double rv[NW];
  __shared__ int ri[NW];
  __shared__ int s_p;
  __shared__ double xr[2][LW];
  __shared__ double ub[LW][64];
  __shared__ double l11[LW][LW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int j1 = j0 + nb;
  for (int c0 = j0; c0 < j1; c0 += LW) {
    const int w = min(LW, j1 - c0);
    double a[R][LW];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int r = j0 + tid + NTH * k;
#pragma unroll
      for (int q = 0; q < LW; ++q) a[k][q] = (r >= c0 && r < n && q < w) ? A[(long long)r * ld + c0 + q] : 0.0;
    }
    for (int cc = 0; cc < w; ++cc) {
      const int col = c0 + cc;
      double bv = -1.0;
      int bi = INT_MAX;
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const int r = j0 + tid + NTH * k;
        double x = 0.0;
#pragma unroll
        for (int q = 0; q < LW; ++q)
          if (q == cc) x = a[k][q];
        if (r >= col && r < n && fabs(x) > bv) {
          bv = fabs(x);
          bi = r;
        }
      }
      pivot_argmax(bv, bi);
      if (lane == 0) {
        rv[wave] = bv;
        ri[wave] = bi;
      }
      __syncthreads();
      if (tid == 0) {
        double v = rv[0];
        int ix = ri[0];
        for (int q = 1; q < NW; ++q)
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
      // rows col and p: exchange the sub-panel part through LDS
      const int oc = col - j0, op = p - j0;
      const bool own_c = oc % NTH == tid, own_p = op % NTH == tid;
      if (own_c || own_p) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
          if (own_c && oc / NTH == k)
#pragma unroll
            for (int q = 0; q < LW; ++q) xr[0][q] = a[k][q];
          if (own_p && op / NTH == k)
#pragma unroll
            for (int q = 0; q < LW; ++q) xr[1][q] = a[k][q];
        }
      }
      // ... and the panel's other columns in global memory
      if (p != col && tid < nb) {
        const int q = j0 + tid;
        if (q < c0 || q >= c0 + w) {
          const double t = A[(long long)col * ld + q];
          A[(long long)col * ld + q] = A[(long long)p * ld + q];
          A[(long long)p * ld + q] = t;
        }
      }
      __syncthreads();
      if (p != col && (own_c || own_p)) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
          if (own_c && oc / NTH == k)
#pragma unroll
            for (int q = 0; q < LW; ++q) a[k][q] = xr[1][q];
          if (own_p && op / NTH == k)
#pragma unroll
            for (int q = 0; q < LW; ++q) a[k][q] = xr[0][q];
        }
      }
      // the pivot row (after the interchange) is xr[1]
      const double d = xr[1][cc];
      const double inv = (d != 0.0) ? 1.0 / d : 0.0;
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const int r = j0 + tid + NTH * k;
        if (r > col && r < n) {
          double l = 0.0;
#pragma unroll
          for (int q = 0; q < LW; ++q)
            if (q == cc) l = a[k][q] * inv;
#pragma unroll
          for (int q = 0; q < LW; ++q) {
            if (q == cc) a[k][q] = l;
            else if (q > cc) a[k][q] = fma(-l, xr[1][q], a[k][q]);
          }
        }
      }
      __syncthreads();  // xr is rewritten by the next column
    }
    // the sub-panel back to global memory, and its unit-lower L11 into LDS
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int r = j0 + tid + NTH * k;
      if (r >= c0 && r < n)
#pragma unroll
        for (int q = 0; q < LW; ++q)
          if (q < w) A[(long long)r * ld + c0 + q] = a[k][q];
      if (r >= c0 && r < c0 + w)
#pragma unroll
        for (int q = 0; q < LW; ++q) l11[r - c0][q] = a[k][q];
    }
    const int q0 = c0 + w, nr = j1 - q0;  // the panel's columns to the right
    if (nr <= 0) break;
    __syncthreads();
    // U rows c0..c0+w-1 of those columns: unit-lower solve with L11, one
    // column per thread, its w entries loaded together
    if (tid < nr) {
      const int q = q0 + tid;
      double x[LW];
#pragma unroll
      for (int i = 0; i < LW; ++i) x[i] = i < w ? A[(long long)(c0 + i) * ld + q] : 0.0;
#pragma unroll
      for (int i = 0; i < LW; ++i) {
#pragma unroll
        for (int k = 0; k < i; ++k) x[i] = fma(-l11[i][k], x[k], x[i]);
        if (i < w) {
          A[(long long)(c0 + i) * ld + q] = x[i];
          ub[i][tid] = x[i];
        }
      }
    }
    __syncthreads();
    // rows below: A[r][q] -= L[r][c0..c0+w) U[c0..c0+w)[q], CH columns at a
    // time with their loads in flight together (a column at a time, each
    // load waited for the previous update)
    constexpr int CH = R >= 4 ? 4 : 8;  // four rows per thread: registers
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int r = j0 + tid + NTH * k;
      if (r >= q0 && r < n) {
        double* ar = A + (long long)r * ld + q0;
        for (int t0 = 0; t0 < nr; t0 += CH) {
          double x[CH];
#pragma unroll
          for (int e = 0; e < CH; ++e) x[e] = t0 + e < nr ? ar[t0 + e] : 0.0;
#pragma unroll
          for (int e = 0; e < CH; ++e)
#pragma unroll
            for (int i = 0; i < LW; ++i)
              if (i < w) x[e] = fma(-a[k][i], ub[i][t0 + e], x[e]);
#pragma unroll
          for (int e = 0; e < CH; ++e)
            if (t0 + e < nr) ar[t0 + e] = x[e];
        }
      }
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
  int cmax = 1, nbmax = 1;
  for (int i = 0; i < nd; ++i) {
    cmax = d[i].nrhs > cmax ? d[i].nrhs : cmax;
    nbmax = d[i].nb > nbmax ? d[i].nb : nbmax;
  }
  const TriDesc* dd = static_cast<const TriDesc*>(st.push(d, sizeof(TriDesc) * nd));
  if (!dd) return hipErrorOutOfMemory;
  if (cmax <= kTriWaveMaxRhs)
    hipLaunchKernelGGL(tri_wave_kernel, dim3(nd, (cmax + 3) / 4), dim3(NT), 0, s, dd);
  else if (nbmax <= 32)
    hipLaunchKernelGGL(tri_block_kernel<32>, dim3(nd, (cmax + NT - 1) / NT), dim3(NT), 0, s, dd);
  else
    hipLaunchKernelGGL(tri_block_kernel<64>, dim3(nd, (cmax + NT - 1) / NT), dim3(NT), 0, s, dd);
  return hipGetLastError();
}

hipError_t launch_refl_y(const ReflYDesc* d, int nd, int rmax, int mmax, Staging& st, hipStream_t s) {
  if (nd <= 0 || rmax <= 0 || mmax <= 0) return hipSuccess;
  const ReflYDesc* dd = static_cast<const ReflYDesc*>(st.push(d, sizeof(ReflYDesc) * nd));
  if (!dd) return hipErrorOutOfMemory;
  const int tiles = ((mmax + 63) / 64) * ((rmax + 63) / 64);
  hipLaunchKernelGGL(refl_y_kernel, dim3(tiles, nd), dim3(NT), 0, s, dd);
  return hipGetLastError();
}

hipError_t launch_sum_partials(const SumDesc* d, int nd, Staging& st, hipStream_t s) {
  if (nd <= 0) return hipSuccess;
  int emax = 1;
  for (int i = 0; i < nd; ++i) emax = std::max(emax, d[i].rows * d[i].cols);
  const SumDesc* dd = static_cast<const SumDesc*>(st.push(d, sizeof(SumDesc) * nd));
  if (!dd) return hipErrorOutOfMemory;
  hipLaunchKernelGGL(sum_partials_kernel, dim3((emax + NT - 1) / NT, nd), dim3(NT), 0, s, dd);
  return hipGetLastError();
}

hipError_t launch_larft(const LarftDesc* d, int nd, Staging& st, hipStream_t s) {
  if (nd <= 0) return hipSuccess;
  const LarftDesc* dd = static_cast<const LarftDesc*>(st.push(d, sizeof(LarftDesc) * nd));
  if (!dd) return hipErrorOutOfMemory;
  hipLaunchKernelGGL(larft_kernel, dim3(nd), dim3(64), 0, s, dd);
  return hipGetLastError();
}

hipError_t launch_lu_panel(double* A, long long ld, int n, int j0, int nb, int* piv, int* info,
                           hipStream_t s) {
  const int rows = n - j0;
  if (nb > 64 || rows > 4096)
    hipLaunchKernelGGL(lu_panel_kernel, dim3(1), dim3(1024), 0, s, A, ld, n, j0, nb, piv, info);
  else if (rows > 2048)
    hipLaunchKernelGGL(lu_panel_reg_kernel<4>, dim3(1), dim3(1024), 0, s, A, ld, n, j0, nb, piv, info);
  else if (rows > 1024)
    hipLaunchKernelGGL(lu_panel_reg_kernel<2>, dim3(1), dim3(1024), 0, s, A, ld, n, j0, nb, piv, info);
  else if (rows > 512)
    hipLaunchKernelGGL(lu_panel_reg_kernel<1>, dim3(1), dim3(1024), 0, s, A, ld, n, j0, nb, piv, info);
  else if (rows > 256)
    hipLaunchKernelGGL((lu_panel_reg_kernel<2, 256>), dim3(1), dim3(256), 0, s, A, ld, n, j0, nb, piv, info);
  else
    hipLaunchKernelGGL((lu_panel_reg_kernel<1, 256>), dim3(1), dim3(256), 0, s, A, ld, n, j0, nb, piv, info);
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
