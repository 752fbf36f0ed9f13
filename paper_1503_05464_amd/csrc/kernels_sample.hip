// Sampling products of randomized HSS compression (Sec. 2.2) on FP64 MFMA:
//   S^r = (A - M) R^r      and      S^c = (A - M)^T R^c,
// where M is either zero or the block-diagonal part of A formed by the leaf
// diagonal blocks.  With M the leaf blocks, S^(l) = (A - D^(l)) R at the
// leaf level is exactly the leaves' local sample S_loc = S(I,:) - D R(I,:)
// of Alg. 1, so the leaf step is fused into the sampling product.
//
// A may be stored in FP32 (widened exactly to FP64 when read from LDS) or
// FP64.  Both products are tall-skinny GEMMs (n x n times n x ncols, ncols =
// d0 or the growth step dd) and are MFMA-bound for ncols >= 32 on gfx950
// (FP64: ~9.8 flop/B ridge against 2*ncols/sizeof(A) flop per byte of A).
//
// Tiling: a 256-thread workgroup computes a 128 x 64 tile of S; its four
// wavefronts each own a 64 x 32 sub-tile as 4 x 2 blocks of the 16x16x4 f64
// MFMA.  A and R are staged through LDS in k-slices of BK rows (BK = 32 for
// FP32 A, 16 for FP64 A); the A slice is stored k-major so that both the
// plain and the transposed product read MFMA operands conflict-free, and
// only the global->LDS copy differs between them.  The next slice is
// prefetched into registers while the current one is multiplied.  When the
// tile count is too small to give every CU its four resident workgroups, K
// is split over workgroups and
// the partial sums are added in a fixed order by a second kernel
// (deterministic, no atomics).  Consecutive tiles are mapped to the same XCD
// so that the column tiles sharing an A slice meet in one L2.
#include "hss_internal.h"

namespace hss {
namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 128;
constexpr int BN = 64;
constexpr int NT = 256;

template <typename TA>
struct Cfg;
template <>
struct Cfg<float> {
  static constexpr int BK = 32;
  static constexpr int PAD = 16;
};
template <>
struct Cfg<double> {
  static constexpr int BK = 16;
  static constexpr int PAD = 8;
};

template <typename TA>
__device__ __forceinline__ double widen(TA v) {
  return (double)v;
}

// Loads this thread's share (64 bytes) of the A slice into registers.
// NN: A[i0 + r][k0 + kseg + e]; TN: A[k0 + kk][i0 + cseg + e].
template <typename TA, bool TRANS>
__device__ __forceinline__ void load_a(TA (&v)[64 / sizeof(TA)], const TA* __restrict__ A,
                                       long long lda, int n, int i0, int k0, int kend,
                                       const int* __restrict__ leaf_of, bool vec_ok,
                                       bool need_mask) {
  constexpr int E = 64 / sizeof(TA);
  constexpr int BK = Cfg<TA>::BK;
  const int tid = threadIdx.x;
  int row, col;  // indices into A
  int ie, ke;    // (i, k) of element 0; element e adds to k (NN) or i (TN)
  if (!TRANS) {
    const int r = tid / (BK / E);
    const int kseg = (tid % (BK / E)) * E;
    row = i0 + r;
    col = k0 + kseg;
    ie = row;
    ke = col;
  } else {
    const int kk = tid / (BM / E);
    const int cseg = (tid % (BM / E)) * E;
    row = k0 + kk;
    col = i0 + cseg;
    ie = col;
    ke = row;
  }
  const bool full = !TRANS ? (row < n && col + E <= kend) : (row < kend && col + E <= n);
  if (full && vec_ok) {
    const u32x4* p = reinterpret_cast<const u32x4*>(A + (long long)row * lda + col);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      u32x4 w = __builtin_nontemporal_load(p + q);
      TA* t = reinterpret_cast<TA*>(&w);
#pragma unroll
      for (int e = 0; e < (int)(16 / sizeof(TA)); ++e) v[q * (16 / sizeof(TA)) + e] = t[e];
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const bool ok = !TRANS ? (row < n && col + e < kend) : (row < kend && col + e < n);
      v[e] = ok ? A[(long long)row * lda + col + e] : (TA)0;
    }
  }
  if (need_mask) {
    // zero the entries of the leaf diagonal blocks: leaf_of[i] == leaf_of[k]
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = !TRANS ? ie : ie + e;
      const int k = !TRANS ? ke + e : ke;
      if (i < n && k < n && leaf_of[i] == leaf_of[k]) v[e] = (TA)0;
    }
  }
}

template <typename TA, bool TRANS>
__device__ __forceinline__ void store_a(TA (*As)[BM + Cfg<TA>::PAD], const TA (&v)[64 / sizeof(TA)]) {
  constexpr int E = 64 / sizeof(TA);
  constexpr int BK = Cfg<TA>::BK;
  const int tid = threadIdx.x;
  if (!TRANS) {
    const int r = tid / (BK / E);
    const int kseg = (tid % (BK / E)) * E;
#pragma unroll
    for (int e = 0; e < E; ++e) As[kseg + e][r] = v[e];
  } else {
    const int kk = tid / (BM / E);
    const int cseg = (tid % (BM / E)) * E;
#pragma unroll
    for (int e = 0; e < E; ++e) As[kk][cseg + e] = v[e];
  }
}

// R slice: rows k0 .. k0+BK-1, columns c0 .. c0+BN-1; ER doubles per thread.
template <int BK>
__device__ __forceinline__ void load_r(double (&v)[BK / 4], const double* __restrict__ R,
                                       long long ldr, int k0, int kend, int c0, int ncols,
                                       bool vec_ok) {
  constexpr int ER = BK / 4;
  const int tid = threadIdx.x;
  const int rr = tid / (BN / ER);
  const int cc = (tid % (BN / ER)) * ER;
  const int k = k0 + rr;
  const int c = c0 + cc;
  if (k < kend && c + ER <= ncols && vec_ok) {
    const double2* p = reinterpret_cast<const double2*>(R + (long long)k * ldr + c);
#pragma unroll
    for (int q = 0; q < ER / 2; ++q) {
      double2 w = p[q];
      v[2 * q] = w.x;
      v[2 * q + 1] = w.y;
    }
  } else {
#pragma unroll
    for (int e = 0; e < ER; ++e) v[e] = (k < kend && c + e < ncols) ? R[(long long)k * ldr + c + e] : 0.0;
  }
}

template <int BK>
__device__ __forceinline__ void store_r(double (*Bs)[BN + 4], const double (&v)[BK / 4]) {
  constexpr int ER = BK / 4;
  const int tid = threadIdx.x;
  const int rr = tid / (BN / ER);
  const int cc = (tid % (BN / ER)) * ER;
#pragma unroll
  for (int e = 0; e < ER; ++e) Bs[rr][cc + e] = v[e];
}

template <typename TA, bool TRANS>
__global__ __launch_bounds__(NT) void sample_kernel(
    const TA* __restrict__ A, long long lda, int n, const int* __restrict__ leaf_of,
    const double* __restrict__ R, long long ldr, double* __restrict__ S, long long lds, int ncols,
    int n_nt, int ksplit, int kchunk, double* __restrict__ work) {
  constexpr int BK = Cfg<TA>::BK;
  constexpr int E = 64 / sizeof(TA);
  __shared__ TA As[BK][BM + Cfg<TA>::PAD];
  __shared__ double Bs[BK][BN + 4];

  // tile of this workgroup; consecutive logical tiles share an XCD
  const int nblk = gridDim.x;
  int L = blockIdx.x;
  if ((nblk & 7) == 0) L = (blockIdx.x & 7) * (nblk >> 3) + (blockIdx.x >> 3);
  const int nt = L % n_nt;
  const int rest = L / n_nt;
  const int ks = rest % ksplit;
  const int mt = rest / ksplit;
  const int i0 = mt * BM;
  const int c0 = nt * BN;
  const int kbeg = ks * kchunk;
  const int kend = min(n, kbeg + kchunk);

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = wave >> 1;
  const int wn = wave & 1;

  const bool vec_a = ((lda * (long long)sizeof(TA)) % 16 == 0) &&
                     ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
  const bool vec_r = (ldr % 2 == 0) && ((reinterpret_cast<uintptr_t>(R) & 15) == 0);

  // Does the leaf mask touch rows [i0, i0+BM) x k-range [k0, k0+BK)?
  // leaf_of holds leaf ordinals in index order (non-decreasing), so the
  // blocks meet iff the leaf ranges of the two index ranges overlap.
  int li0 = 0, li1 = -1;
  if (leaf_of) {
    li0 = leaf_of[min(i0, n - 1)];
    li1 = leaf_of[min(i0 + BM, n) - 1];
  }

  dbl4 acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};

  TA va[E];
  double vr[BK / 4];
  auto mask_for = [&](int k0) -> bool {
    if (!leaf_of || k0 >= kend) return false;
    const int lk0 = leaf_of[k0];
    const int lk1 = leaf_of[min(k0 + BK, kend) - 1];
    return !(lk1 < li0 || li1 < lk0);
  };

  int k0 = kbeg;
  if (k0 < kend) {
    load_a<TA, TRANS>(va, A, lda, n, i0, k0, kend, leaf_of, vec_a, mask_for(k0));
    load_r<BK>(vr, R, ldr, k0, kend, c0, ncols, vec_r);
    store_a<TA, TRANS>(As, va);
    store_r<BK>(Bs, vr);
  }
  __syncthreads();
  for (; k0 < kend; k0 += BK) {
    const int kn = k0 + BK;
    if (kn < kend) {
      load_a<TA, TRANS>(va, A, lda, n, i0, kn, kend, leaf_of, vec_a, mask_for(kn));
      load_r<BK>(vr, R, ldr, kn, kend, c0, ncols, vec_r);
    }
    // the wavefronts multiplying take issue priority over those still
    // loading or storing the next slice (8.99 -> 8.36 ms per launch at
    // n = 65536, 64 columns)
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      double a[4], b[2];
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) a[mb] = widen(As[kr][wm * 64 + mb * 16 + (lane & 15)]);
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) b[nb] = Bs[kr][wn * 32 + nb * 16 + (lane & 15)];
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
          acc[mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mb], b[nb], acc[mb][nb], 0, 0, 0);
    }
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();
    if (kn < kend) {
      store_a<TA, TRANS>(As, va);
      store_r<BK>(Bs, vr);
    }
    __syncthreads();
  }

  // D layout of the 16x16x4 f64 MFMA on gfx950 (checked on the device):
  // lane l, register r -> row l/16 + 4r, column l%16.
  double* out = S;
  long long ldo = lds;
  if (ksplit > 1) {
    out = work + (long long)ks * n * ncols;
    ldo = ncols;
  }
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
      const int c = c0 + wn * 32 + nb * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wm * 64 + mb * 16 + (lane >> 4) + 4 * r;
        if (i < n && c < ncols) out[(long long)i * ldo + c] = acc[mb][nb][r];
      }
    }
}

__global__ void reduce_splits_kernel(const double* __restrict__ work, int ksplit, long long n,
                                     int ncols, double* __restrict__ S, long long lds) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = n * ncols;
  if (idx >= total) return;
  const long long i = idx / ncols;
  const int c = (int)(idx % ncols);
  double s = 0.0;
  for (int q = 0; q < ksplit; ++q) s += work[(long long)q * total + idx];
  S[i * lds + c] = s;
}

struct Plan {
  int n_mt, n_nt, ksplit, kchunk;
};

Plan make_plan(long long n, int ncols, int bk) {
  Plan p;
  p.n_mt = (int)((n + BM - 1) / BM);
  p.n_nt = (ncols + BN - 1) / BN;
  const long long tiles = (long long)p.n_mt * p.n_nt;
  long long want = (1024 + tiles - 1) / tiles;  // 4 workgroups per CU (the resident maximum)
  long long maxs = n / 1024;                   // keep >= 1024 k per split
  if (maxs < 1) maxs = 1;
  if (want > maxs) want = maxs;
  if (want < 1) want = 1;
  long long chunk = (n + want - 1) / want;
  chunk = (chunk + bk - 1) / bk * bk;
  p.ksplit = (int)((n + chunk - 1) / chunk);
  p.kchunk = (int)chunk;
  return p;
}

template <typename TA, bool TRANS>
void run(const TA* A, long long lda, long long n, const int* leaf_of, int ncols, const double* R,
         long long ldr, double* S, long long lds, double* work, hipStream_t s) {
  Plan p = make_plan(n, ncols, Cfg<TA>::BK);
  const long long nblocks = (long long)p.n_mt * p.n_nt * p.ksplit;
  hipLaunchKernelGGL((sample_kernel<TA, TRANS>), dim3((unsigned)nblocks), dim3(NT), 0, s, A, lda,
                     (int)n, leaf_of, R, ldr, S, lds, ncols, p.n_nt, p.ksplit, p.kchunk, work);
  if (p.ksplit > 1) {
    const long long total = n * ncols;
    hipLaunchKernelGGL(reduce_splits_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       work, p.ksplit, n, ncols, S, lds);
  }
}

}  // namespace

long long sample_workspace_doubles(long long n, int ncols) {
  // the FP64 plan needs at least as many splits as the FP32 one
  Plan a = make_plan(n, ncols, Cfg<float>::BK);
  Plan b = make_plan(n, ncols, Cfg<double>::BK);
  int ks = a.ksplit > b.ksplit ? a.ksplit : b.ksplit;
  return ks > 1 ? (long long)ks * n * ncols : 0;
}

void launch_sample(const void* A, int dtype, long long n, long long lda, const int* leaf_of,
                   int ncols, const double* Rr, const double* Rc, long long ldr, double* Sr,
                   double* Sc, long long lds, double* work, hipStream_t s) {
  if (n <= 0 || ncols <= 0) return;
  if (dtype == 1) {
    const float* a = static_cast<const float*>(A);
    if (Sr) run<float, false>(a, lda, n, leaf_of, ncols, Rr, ldr, Sr, lds, work, s);
    if (Sc) run<float, true>(a, lda, n, leaf_of, ncols, Rc, ldr, Sc, lds, work, s);
  } else {
    const double* a = static_cast<const double*>(A);
    if (Sr) run<double, false>(a, lda, n, leaf_of, ncols, Rr, ldr, Sr, lds, work, s);
    if (Sc) run<double, true>(a, lda, n, leaf_of, ncols, Rc, ldr, Sc, lds, work, s);
  }
}

}  // namespace hss
