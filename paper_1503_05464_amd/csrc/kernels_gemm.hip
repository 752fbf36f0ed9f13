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
// Arithmetic: the 16x16x4 FP64 MFMA, each of the four wavefronts of a
// workgroup owning a 32 x 32 sub-tile (2 x 2 MFMA blocks).  A and B are
// staged through LDS in k-slices of 16, both k-major so that the MFMA
// operands are read conflict-free; the next slice is loaded into registers
// while the current one is multiplied.  (A vector-FMA version with 4 x 4
// outputs per thread took 1.2 to 1.4 times as long, on large and on small
// batched products alike.)
#include <climits>

#include "hss_internal.h"

namespace hss {
namespace {

constexpr int TM = 64, TN = 64, TK = 16, NTH = 256;

typedef double dbl4 __attribute__((ext_vector_type(4)));

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

// held to four wavefronts per SIMD (at most 128 registers; it needs 94)
__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(4))) void gemm_batched_kernel(
    const DevDesc* __restrict__ descs, int nprob) {
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
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;  // this wavefront's 32 x 32 sub-tile

  // this thread's share of a k-slice: 4 entries of A and 4 of B
  double va[4], vb[4];
  auto load = [&](int k0) {
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
      va[q] = (r < g.M && k < g.K) ? (g.transA ? g.A[(long long)k * g.lda + r] : g.A[(long long)r * g.lda + k])
                                   : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + q * NTH;
      const int kk = e / TN, cc = e % TN;
      const int k = k0 + kk, c = c0 + cc;
      vb[q] = (k < g.K && c < g.N) ? seg_row(g.B, k)[c] : 0.0;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + q * NTH;
      if (!g.transA) As[e % TK][e / TK] = va[q];
      else As[e / TM][e % TM] = va[q];
      Bs[e / TN][e % TN] = vb[q];
    }
  };

  dbl4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};

  if (g.K > 0) {
    load(0);
    store();
  }
  __syncthreads();
  for (int k0 = 0; k0 < g.K; k0 += TK) {
    const int kn = k0 + TK;
    if (kn < g.K) load(kn);  // next slice in flight while this one is multiplied
    __builtin_amdgcn_s_setprio(1);  // multiplying wavefronts issue first
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      const int kr = kk + (lane >> 4);
      double a[2], b[2];
#pragma unroll
      for (int mb = 0; mb < 2; ++mb) a[mb] = As[kr][wm * 32 + mb * 16 + (lane & 15)];
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) b[nb] = Bs[kr][wn * 32 + nb * 16 + (lane & 15)];
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
          acc[mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mb], b[nb], acc[mb][nb], 0, 0, 0);
    }
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();
    if (kn < g.K) store();
    __syncthreads();
  }

  // D layout of the 16x16x4 f64 MFMA: lane l, register q -> row l/16 + 4q,
  // column l%16 of the 16 x 16 block
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = r0 + wm * 32 + mb * 16 + (lane >> 4) + 4 * q;
      if (r >= g.M) continue;
      const double* crow = (g.beta != 0.0) ? seg_row(g.C, r) : nullptr;
      double* drow = seg_row_out(g.D, r);
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        const int c = c0 + wn * 32 + nb * 16 + (lane & 15);
        if (c >= g.N) continue;
        double v = g.alpha * acc[mb][nb][q];
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
