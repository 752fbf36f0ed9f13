// Batched FP64 GEMM with row gathers and scatters, for the small per-node
// products of compression (Alg. 1: S_a - B_ab R_b, V^T R_in), matvec
// (Alg. 2: V^T x, B y, U z) and the ULV factors (Alg. 3/4).
//
//   D[rowD(r), c] = beta * C[rowC(r), c] + alpha * sum_k Aop(r, k) * B[rowB(k), c]
//
// Every problem of a batch has its own sizes and pointers; one launch covers
// all of them, one 64 x 64 output tile per workgroup.  The problem of a tile
// is found by a binary search over the tile prefix sums.  Row maps let the
// ID-structured generators U = Pi [I; E] act without forming U: rows J are
// gathered or scattered and E multiplies the other rows.  A source may be
// split in two segments (rows below `split` from one buffer, the rest from
// another), which stacks the two children's blocks [X_a; X_b] without a copy.
//
// Arithmetic: FP64 FMA on the vector ALU (on gfx950 FP64 vector and matrix
// peaks are equal), 4 x 4 register blocking per thread, k-slices of 16
// staged through LDS.
#include <climits>

#include "hss_internal.h"

namespace hss {
namespace {

constexpr int TM = 64, TN = 64, TK = 16, NTH = 256;

struct DevDesc {
  GemmDesc g;
  long long tile0;  // first flattened tile of this problem
  int tiles_n;      // tiles along N
};

__device__ __forceinline__ const double* seg_row(const Seg& s, int q) {
  int qq = s.map ? s.map[q] : q;
  return (qq < s.split) ? s.p0 + (long long)qq * s.ld : s.p1 + (long long)(qq - s.split) * s.ld;
}
__device__ __forceinline__ double* seg_row_out(const SegOut& s, int q) {
  int qq = s.map ? s.map[q] : q;
  return (qq < s.split) ? s.p0 + (long long)qq * s.ld : s.p1 + (long long)(qq - s.split) * s.ld;
}

__global__ __launch_bounds__(NTH) void gemm_batched_kernel(const DevDesc* __restrict__ descs,
                                                           int nprob) {
  // locate the problem of this tile
  const long long t = blockIdx.x;
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (descs[mid].tile0 <= t) lo = mid;
    else hi = mid - 1;
  }
  const DevDesc& dd = descs[lo];
  const GemmDesc& g = dd.g;
  const long long local = t - dd.tile0;
  const int r0 = (int)(local / dd.tiles_n) * TM;
  const int c0 = (int)(local % dd.tiles_n) * TN;

  __shared__ double As[TK][TM + 4];
  __shared__ double Bs[TK][TN + 4];

  const int tid = threadIdx.x;
  const int tx = tid & 15;  // columns c0 + 4*tx ..
  const int ty = tid >> 4;  // rows r0 + 4*ty ..
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;

  for (int k0 = 0; k0 < g.K; k0 += TK) {
    // A slice: TM x TK, 4 per thread
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + q * NTH;
      int rr, kk;
      if (!g.transA) {
        rr = e / TK;
        kk = e % TK;
      } else {
        kk = e / TM;
        rr = e % TM;
      }
      const int r = r0 + rr, k = k0 + kk;
      double v = 0.0;
      if (r < g.M && k < g.K)
        v = g.transA ? g.A[(long long)k * g.lda + r] : g.A[(long long)r * g.lda + k];
      As[kk][rr] = v;
    }
    // B slice: TK x TN, gathered rows
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + q * NTH;
      const int kk = e / TN, cc = e % TN;
      const int k = k0 + kk, c = c0 + cc;
      double v = 0.0;
      if (k < g.K && c < g.N) v = seg_row(g.B, k)[c];
      Bs[kk][cc] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = r0 + ty * 4 + i;
    if (r >= g.M) continue;
    const double* crow = (g.beta != 0.0) ? seg_row(g.C, r) : nullptr;
    double* drow = seg_row_out(g.D, r);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = c0 + tx * 4 + j;
      if (c >= g.N) continue;
      double v = g.alpha * acc[i][j];
      if (crow) v += g.beta * crow[c];
      drow[c] = v;
    }
  }
}

}  // namespace

hipError_t launch_gemm_batched(const GemmDesc* descs, int nprob, Staging& st, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  DevDesc* h = new DevDesc[nprob];
  long long tiles = 0;
  int kept = 0;
  for (int p = 0; p < nprob; ++p) {
    const GemmDesc& g = descs[p];
    if (g.M <= 0 || g.N <= 0) continue;
    DevDesc& d = h[kept++];
    d.g = g;
    if (d.g.B.p1 == nullptr) d.g.B.split = INT_MAX;
    if (d.g.C.p1 == nullptr) d.g.C.split = INT_MAX;
    if (d.g.D.p1 == nullptr) d.g.D.split = INT_MAX;
    d.tiles_n = (g.N + TN - 1) / TN;
    d.tile0 = tiles;
    tiles += (long long)((g.M + TM - 1) / TM) * d.tiles_n;
  }
  hipError_t err = hipSuccess;
  if (kept > 0 && tiles > 0) {
    void* dd = st.push(h, sizeof(DevDesc) * kept);
    if (!dd) {
      err = hipErrorOutOfMemory;
    } else {
      hipLaunchKernelGGL(gemm_batched_kernel, dim3((unsigned)tiles), dim3(NTH), 0, s,
                         static_cast<const DevDesc*>(dd), kept);
      err = hipGetLastError();
    }
  }
  delete[] h;
  return err;
}

}  // namespace hss
