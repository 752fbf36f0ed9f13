// Batched FP64 GEMM with row gathers and scatters, for the small per-node
// products of compression (Alg. 1: S_a - B_ab R_b, V^T R_in), matvec
// (Alg. 2: V^T x, B y, U z) and the ULV factors (Alg. 3/4).
//
//   D[rowD(r), c] = beta * C[rowC(r), c] + alpha * sum_k Aop(r, k) * B[rowB(k), c]
//
// Every problem of a batch has its own sizes and pointers; one launch covers
// all of them, one output tile per workgroup.  The tile shape of a launch is
// picked from a table indexed by the batch's size class (widest N, largest
// M), written by the project's autotuner (paper_1503_05464_amd/autotune.py)
// from measured launch times.  The problem of a tile is found by a binary
// search over the tile prefix sums.  Row maps let the
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
#include <algorithm>
#include <climits>
#include <cstdlib>
#include <vector>

#include "hss_internal.h"

namespace hss {
namespace {

constexpr int TK = 16, NTH = 256;

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

// Tile shapes: the four wavefronts form a WGM x WGN grid, each owning MB x NB
// blocks of 16 x 16 (one 16x16x4 FP64 MFMA accumulator each), so a tile is
// TM = 16 WGM MB rows by TN = 16 WGN NB columns.  Wide tiles suit the
// compression's products (N = the new sample columns); narrow ones the
// matvec and solve with few right-hand sides, where a 64-column tile would
// leave most of its columns empty.
template <int WGM, int WGN, int MB, int NB>
struct Tile {
  static_assert(WGM * WGN == 4, "four wavefronts");
  static constexpr int TM = 16 * WGM * MB, TN = 16 * WGN * NB;
  static constexpr int LA = TK * TM / NTH, LB = TK * TN / NTH;  // slice entries per thread
  static_assert(LA >= 1 && LB >= 1 && TK * TM % NTH == 0 && TK * TN % NTH == 0, "whole slices");
};

// held to four wavefronts per SIMD (at most 128 registers)
template <int WGM, int WGN, int MB, int NB>
__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(4))) void gemm_batched_kernel(
    const DevDesc* __restrict__ descs, int nprob) {
  using TL = Tile<WGM, WGN, MB, NB>;
  constexpr int TM = TL::TM, TN = TL::TN, LA = TL::LA, LB = TL::LB;
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
  const int wm = wave / WGN, wn = wave % WGN;  // this wavefront's sub-tile

  // this thread's share of a k-slice: LA entries of A and LB of B
  double va[LA], vb[LB];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < LA; ++q) {
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
    for (int q = 0; q < LB; ++q) {
      const int e = tid + q * NTH;
      const int kk = e / TN, cc = e % TN;
      const int k = k0 + kk, c = c0 + cc;
      vb[q] = (k < g.K && c < g.N) ? seg_row(g.B, k)[c] : 0.0;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int q = 0; q < LA; ++q) {
      const int e = tid + q * NTH;
      if (!g.transA) As[e % TK][e / TK] = va[q];
      else As[e / TM][e % TM] = va[q];
    }
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      const int e = tid + q * NTH;
      Bs[e / TN][e % TN] = vb[q];
    }
  };

  dbl4 acc[MB][NB];
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};

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
      double a[MB], b[NB];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) a[mb] = As[kr][wm * 16 * MB + mb * 16 + (lane & 15)];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) b[nb] = Bs[kr][wn * 16 * NB + nb * 16 + (lane & 15)];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
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
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = r0 + wm * 16 * MB + mb * 16 + (lane >> 4) + 4 * q;
      if (r >= g.M) continue;
      const double* crow = (g.beta != 0.0) ? seg_row(g.C, r) : nullptr;
      double* drow = seg_row_out(g.D, r);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int c = c0 + wn * 16 * NB + nb * 16 + (lane & 15);
        if (c >= g.N) continue;
        double v = g.alpha * acc[mb][nb][q];
        if (crow) v += g.beta * crow[c];
        drow[c] = v;
      }
    }
}

struct GVariant {
  int tm, tn;
  void (*fn)(const DevDesc*, int);
};
// the tile shapes (index = variant number of the tuning table)
const GVariant kGVariants[] = {
    {64, 64, gemm_batched_kernel<2, 2, 2, 2>},
    {64, 16, gemm_batched_kernel<4, 1, 1, 1>},
    {128, 16, gemm_batched_kernel<4, 1, 2, 1>},
    {32, 32, gemm_batched_kernel<2, 2, 1, 1>},
    {64, 32, gemm_batched_kernel<4, 1, 1, 2>},
    {128, 32, gemm_batched_kernel<4, 1, 2, 2>},
    {16, 64, gemm_batched_kernel<1, 4, 1, 1>},
};
constexpr int kNumGVariants = sizeof(kGVariants) / sizeof(kGVariants[0]);

#include "gemm_tiles.inc"  // kGemmTileTable[class] = variant (written by autotune.py)
static_assert(sizeof(kGemmTileTable) / sizeof(kGemmTileTable[0]) == kGemmClasses, "one entry per class");

}  // namespace

// The size class of a launch: its widest N and its largest M, bucketed.
static int gemm_class(const GemmDesc* descs, int nprob) {
  int nmax = 0, mmax = 0;
  for (int p = 0; p < nprob; ++p)
    if (descs[p].M > 0 && descs[p].N > 0) {
      nmax = std::max(nmax, descs[p].N);
      mmax = std::max(mmax, descs[p].M);
    }
  const int nb = nmax <= 16 ? 0 : nmax <= 32 ? 1 : nmax <= 64 ? 2 : 3;
  const int mb = mmax <= 32 ? 0 : mmax <= 128 ? 1 : 2;
  return nb * 3 + mb;
}

hipError_t launch_gemm_batched(const GemmDesc* descs, int nprob, Staging& st, hipStream_t s, int variant) {
  if (nprob <= 0) return hipSuccess;
  if (variant < 0 || variant >= kNumGVariants) {
    variant = kGemmTileTable[gemm_class(descs, nprob)];
    static const int forced = [] {  // tuning and tests: one variant for every launch
      const char* v = std::getenv("HSS_GEMM_VARIANT");
      return v && v[0] ? std::atoi(v) : -1;
    }();
    if (forced >= 0 && forced < kNumGVariants) variant = forced;
  }
  const GVariant& gv = kGVariants[variant];
  std::vector<DevDesc> h;
  h.reserve(nprob);
  long long tiles = 0;
  for (int p = 0; p < nprob; ++p) {
    const GemmDesc& g = descs[p];
    if (g.M <= 0 || g.N <= 0) continue;
    DevDesc d;
    d.g = g;
    if (d.g.B.p1 == nullptr) d.g.B.split = INT_MAX;
    if (d.g.C.p1 == nullptr) d.g.C.split = INT_MAX;
    if (d.g.D.p1 == nullptr) d.g.D.split = INT_MAX;
    d.tiles_n = (g.N + gv.tn - 1) / gv.tn;
    d.tile0 = tiles;
    tiles += (long long)((g.M + gv.tm - 1) / gv.tm) * d.tiles_n;
    h.push_back(d);
  }
  if (h.empty() || tiles <= 0) return hipSuccess;
  void* dd = st.push(h.data(), sizeof(DevDesc) * h.size());
  if (!dd) return hipErrorOutOfMemory;
  hipLaunchKernelGGL(gv.fn, dim3((unsigned)tiles), dim3(NTH), 0, s, static_cast<const DevDesc*>(dd), (int)h.size());
  return hipGetLastError();
}

int gemm_variants() { return kNumGVariants; }

}  // namespace hss
