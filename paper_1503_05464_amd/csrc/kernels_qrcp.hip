// Batched interpolative decomposition [X, J] = ID(Y, eps) by Householder QR
// with column pivoting, stopped at the first pivot with
// |R_ii| <= eps |R_11| (Sec. 2.2; the modified xGEQP3 of Sec. 3.2).
//
// Problem p holds Y_p (d x m) as the m rows of a row-major matrix (the rows
// of the local sample S_loc, so "column j of Y" is a contiguous row).  The
// kernel works on a copy W.  One workgroup per problem:
//   * pivot = largest remaining column norm, lowest index on ties (block
//     reduction);
//   * the reflector of the pivot column is staged in LDS and applied to all
//     unselected columns, one column per wavefront at a time (wavefront dot
//     product, update, and an exact recomputation of the remaining norm --
//     no downdating, so small tolerances stay accurate);
//   * columns are not swapped: a per-column step number marks the pivots,
//     so R(i, j) stays in row i of column j's storage.
// A second kernel forms J (pivot order) and the other columns in increasing
// order, and E = (R1^{-1} R2)^T by back substitution, one thread per
// unselected column.
//
// Early exit: when the caller's fail rule (rank above d - p_margin and
// below m) is already certain -- more than kfail pivots accepted and m > d,
// so the rank cannot reach m -- the factorization stops; the reported rank
// is then a lower bound that still trips the rule.
#include <cmath>

#include "hss_internal.h"

namespace hss {
namespace {

constexpr int NT = 256;
constexpr int NW = NT / 64;

struct DevIdProblem {
  IdProblem p;
  long long off;
  int allow_early;
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(NT) void qrcp_kernel(const DevIdProblem* __restrict__ probs,
                                                  double rtol, int* __restrict__ kout,
                                                  int* __restrict__ step_all,
                                                  double* __restrict__ nrm_all) {
  extern __shared__ double u[];  // reflector, length d
  __shared__ double red_v[NT / 64];
  __shared__ int red_i[NT / 64];
  __shared__ double s_best;
  __shared__ int s_p;

  const DevIdProblem dp = probs[blockIdx.x];
  const IdProblem& P = dp.p;
  const int m = P.m, d = P.d;
  const long long ldw = P.ldw;
  double* __restrict__ W = P.W;
  int* __restrict__ step = step_all + dp.off;
  double* __restrict__ nrm = nrm_all + dp.off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  // copy and initial norms
  for (int j = wave; j < m; j += NW) {
    const double* y = P.Y + (long long)j * P.ldy;
    double* w = W + (long long)j * ldw;
    double s = 0.0;
    for (int r = lane; r < d; r += 64) {
      const double v = y[r];
      w[r] = v;
      s = fma(v, v, s);
    }
    s = wave_sum(s);
    if (lane == 0) {
      nrm[j] = sqrt(s);
      step[j] = -1;
    }
  }
  __threadfence_block();
  __syncthreads();

  const int kmax = min(m, d);
  double nu0 = 0.0;
  int k = 0;
  for (int i = 0; i < kmax; ++i) {
    // pivot: largest norm among unselected columns, lowest index on ties
    double bv = -1.0;
    int bi = m;
    for (int j = tid; j < m; j += NT) {
      if (step[j] < 0) {
        const double v = nrm[j];
        if (v > bv) {  // j increases, so ties keep the lowest index
          bv = v;
          bi = j;
        }
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
      red_v[wave] = bv;
      red_i[wave] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      double v = red_v[0];
      int ix = red_i[0];
      for (int q = 1; q < NW; ++q) {
        if (red_v[q] > v || (red_v[q] == v && red_i[q] < ix)) {
          v = red_v[q];
          ix = red_i[q];
        }
      }
      s_best = v;
      s_p = ix;
    }
    __syncthreads();
    const double best = s_best;
    const int p = s_p;
    if (i == 0) nu0 = best;
    if (best <= 0.0 || best <= rtol * nu0) break;
    if (dp.allow_early && i > P.kfail && m > d) break;

    // Householder reflector of column p, rows i..d-1: H = I - tau u u^T,
    // u_0 = 1, H x = alpha e_1 with alpha = -sign(x_0) ||x||.
    double* wp = W + (long long)p * ldw;
    const double x0 = wp[i];
    const double alpha = -copysign(best, x0);
    const double v0 = x0 - alpha;
    const double tau = -v0 / alpha;
    const double inv_v0 = 1.0 / v0;
    for (int r = i + tid; r < d; r += NT) u[r - i] = (r == i) ? 1.0 : wp[r] * inv_v0;
    __syncthreads();
    if (tid == 0) {
      wp[i] = alpha;
      step[p] = i;
    }
    __threadfence_block();
    __syncthreads();

    for (int j = wave; j < m; j += NW) {
      if (step[j] >= 0) continue;
      double* w = W + (long long)j * ldw;
      double dot = 0.0;
      for (int r = i + lane; r < d; r += 64) dot = fma(u[r - i], w[r], dot);
      dot = wave_sum(dot);
      const double f = tau * dot;
      double s = 0.0;
      for (int r = i + lane; r < d; r += 64) {
        const double v = fma(-f, u[r - i], w[r]);
        w[r] = v;
        if (r > i) s = fma(v, v, s);
      }
      s = wave_sum(s);
      if (lane == 0) nrm[j] = sqrt(s);
    }
    __threadfence_block();
    __syncthreads();
    k = i + 1;
  }
  if (tid == 0) kout[blockIdx.x] = k;
}

// J / rest permutation and E = (R1^{-1} R2)^T.  grid: (problem, chunk of
// NT unselected columns).  Chunk 0 also writes the permutation.
__global__ __launch_bounds__(NT) void id_finish_kernel(const DevIdProblem* __restrict__ probs,
                                                      const int* __restrict__ kin,
                                                      const int* __restrict__ step_all) {
  __shared__ int cnt[NT];
  const DevIdProblem dp = probs[blockIdx.x];
  const IdProblem& P = dp.p;
  const int m = P.m;
  const int k = kin[blockIdx.x];
  const int* __restrict__ step = step_all + dp.off;
  const int tid = threadIdx.x;
  int* perm = P.perm;

  // ranks of the unselected columns among themselves (block scan over
  // contiguous chunks)
  const int per = (m + NT - 1) / NT;
  const int j0 = tid * per;
  const int j1 = min(m, j0 + per);
  int c = 0;
  for (int j = j0; j < j1; ++j) c += (step[j] < 0 || step[j] >= k) ? 1 : 0;
  cnt[tid] = c;
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int q = 0; q < NT; ++q) {
      const int t = cnt[q];
      cnt[q] = acc;
      acc += t;
    }
  }
  __syncthreads();
  int pos = cnt[tid];
  for (int j = j0; j < j1; ++j) {
    const int s = step[j];
    if (s >= 0 && s < k) perm[s] = j;
    else perm[k + pos++] = j;
  }
  __threadfence_block();
  __syncthreads();

  // back substitution for every unselected column c: R1 t = R2(:, c)
  const double* W = P.W;
  const long long ldw = P.ldw;
  for (int cidx = tid; cidx < m - k; cidx += NT) {
    const int jc = perm[k + cidx];
    const double* wc = W + (long long)jc * ldw;
    double* t = P.E + (long long)cidx * k;
    for (int a = k - 1; a >= 0; --a) {
      double s = wc[a];
      for (int b = a + 1; b < k; ++b) s = fma(-W[(long long)perm[b] * ldw + a], t[b], s);
      t[a] = s / W[(long long)perm[a] * ldw + a];
    }
  }
}

}  // namespace

hipError_t launch_id_batched(const IdProblem* probs, int nprob, double rtol, int* k_dev,
                             int* step_dev, double* nrm_dev, const long long* offs, Staging& st,
                             hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  DevIdProblem* h = new DevIdProblem[nprob];
  int dmax = 1;
  for (int q = 0; q < nprob; ++q) {
    h[q].p = probs[q];
    h[q].off = offs[q];
    h[q].allow_early = probs[q].kfail >= 0 ? 1 : 0;
    if (probs[q].d > dmax) dmax = probs[q].d;
  }
  // the reflector is staged in LDS: d doubles per workgroup
  if ((size_t)dmax * sizeof(double) > 64 * 1024) {
    delete[] h;
    return hipErrorInvalidValue;
  }
  void* dd = st.push(h, sizeof(DevIdProblem) * nprob);
  delete[] h;
  if (!dd) return hipErrorOutOfMemory;
  const DevIdProblem* d = static_cast<const DevIdProblem*>(dd);
  hipLaunchKernelGGL(qrcp_kernel, dim3(nprob), dim3(NT), (size_t)dmax * sizeof(double), s, d, rtol,
                     k_dev, step_dev, nrm_dev);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(id_finish_kernel, dim3(nprob), dim3(NT), 0, s, d, k_dev, step_dev);
  return hipGetLastError();
}

}  // namespace hss
