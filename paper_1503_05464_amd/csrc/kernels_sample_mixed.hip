// Sampling products of randomized HSS compression (Sec. 2.2) in reduced
// precision, for A stored in FP32:
//   S^r = (A - M) R^r      and      S^c = (A - M)^T R^c
// (M: zero or the leaf diagonal blocks, as in the FP64 kernel).
//
// R has already been rounded to the precision of the products (FP32 or
// BF16) when it was drawn, and the rest of the compression uses that same R,
// so the products below differ from the FP64 products of the same A and R
// only by the rounding of their accumulation.
//
// Two modes:
//  * F32: the 16x16x4 FP32 MFMA on FP32 A and R;
//  * BF16X3: every FP32 entry of A is split exactly into three BF16 terms,
//    a = h1 + h2 + h3 (h1 = bf16(a), h2 = bf16(a - h1), h3 = a - h1 - h2), and
//    the three products h_t R run on the 16x16x32 BF16 MFMA.  Each product of
//    two BF16 numbers is exact in FP32.
// In both modes the MFMA accumulates in FP32 over a chunk of KF = 256 values
// of k; the chunk sum is then added into an FP64 accumulator, so rounding
// grows with the chunk length rather than with n.
//
// Tiling: a 256-thread workgroup computes a 128 x 64 tile of S, its four
// wavefronts 64 x 32 each as 4 x 2 blocks of 16 x 16.  A passes through LDS
// in k-slices of 32, stored with k contiguous per row (split into its three
// BF16 planes on the way in), so that a lane reads its eight k values for
// one MFMA operand in a single 16-byte access: lane l takes
// k = 8 (l / 16) + e, e < 8, of row l % 16 -- the same k for A and R, which is
// all the product needs.  A is written to LDS in packed pieces: a thread
// holds 4 consecutive k of each of 4 rows of the tile, loaded as four rows
// of 4 k (plain product; eight consecutive lanes cover a row of the slice)
// or as a 4 x 4 block of A (transposed product).  R comes from a transposed
// copy in the products' precision (R^T: columns of R contiguous, zero-padded
// to whole slices and tiles), made once per call; its slice passes through
// LDS beside A's.  The output layout of both MFMAs (checked on the
// device): lane l, register r -> row 4 (l / 16) + r, column l % 16.  The
// single-matrix kernel is held to 168 registers so that three workgroups
// share a CU, and K is split to fill two whole rounds of them.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "hss_internal.h"

namespace hss {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 128;
constexpr int BN = 64;
constexpr int BK = 32;
constexpr int NT = 256;
constexpr int KF = 256;        // k values accumulated in FP32 before the FP64 carry
// LDS row pitches (elements) chosen so that the 16 rows read by one 16-byte
// access per lane start on distinct bank groups: 144 B rows for FP32, 80 B
// rows for BF16
constexpr int AP1 = BK + 4;
constexpr int AP2 = BK + 8;

// round-to-nearest-even FP32 -> BF16 (finite inputs)
__device__ __forceinline__ unsigned short bf16_rn(float x) {
  unsigned int u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

template <int MODE>
struct Smem;
template <>
struct alignas(16) Smem<1> {  // FP32
  float A[BM][AP1];
  float R[BN][AP1];  // R^T slice: column c of R, k contiguous
};
template <>
struct alignas(16) Smem<2> {  // BF16 x 3
  unsigned short A[3][BM][AP2];
  unsigned short R[BN][AP2];
};

template <int MODE>
struct RtType;
template <>
struct RtType<1> {
  typedef float T;
};
template <>
struct RtType<2> {
  typedef unsigned short T;
};

// This thread's 16 entries of the A slice, stored in v[4 q + e].  NN: row
// i0 + 32 q + tid / 8, k = k0 + 4 (tid % 8) + e, so that eight consecutive
// lanes read one row's 128 bytes of the slice in one instruction (with two
// lanes per row, each reading 64 bytes in four instructions, the loads of a
// wavefront touched 32 rows per instruction and A streamed at 3.8 TB/s
// against 7.1 TB/s).  TN (element (i, k) is A[k][i]): k = k0 + 4 (tid / 32)
// + q, i = i0 + 4 (tid % 32) + e.  Either way the thread holds 4 consecutive
// k of each of 4 rows of the tile.
template <bool TRANS>
__device__ __forceinline__ void load_a(float (&v)[16], const float* __restrict__ A, long long lda,
                                       int n, int i0, int k0, int kend,
                                       const int* __restrict__ leaf_of, bool vec_ok,
                                       bool need_mask) {
  const int tid = threadIdx.x;
  if (!TRANS) {
    const int rb = i0 + (tid >> 3), col = k0 + 4 * (tid & 7);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = rb + 32 * q;
      if (row < n && col + 4 <= kend && vec_ok) {
        const u32x4 w = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(A + (long long)row * lda + col));
#pragma unroll
        for (int e = 0; e < 4; ++e) v[4 * q + e] = __uint_as_float(w[e]);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          v[4 * q + e] = (row < n && col + e < kend) ? A[(long long)row * lda + col + e] : 0.0f;
      }
    }
    if (need_mask) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (rb + 32 * q < n && col + e < n && leaf_of[rb + 32 * q] == leaf_of[col + e]) v[4 * q + e] = 0.0f;
    }
  } else {
    const int kb = k0 + 4 * (tid >> 5), ib = i0 + 4 * (tid & 31);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = kb + q;
      if (k < kend && ib + 4 <= n && vec_ok) {
        const u32x4 w = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(A + (long long)k * lda + ib));
#pragma unroll
        for (int e = 0; e < 4; ++e) v[4 * q + e] = __uint_as_float(w[e]);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[4 * q + e] = (k < kend && ib + e < n) ? A[(long long)k * lda + ib + e] : 0.0f;
      }
    }
    if (need_mask) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (kb + q < n && ib + e < n && leaf_of[kb + q] == leaf_of[ib + e]) v[4 * q + e] = 0.0f;
    }
  }
}

// Three-term split of an FP32 value into BF16 by truncation, a = h1 + h2 + h3
// exactly: h1 keeps the top 8 significant bits of a (its upper 16 bits), the
// remainder r1 = a - h1 is exact in FP32 and has at most 16 significant bits,
// h2 keeps its top 8, and r2 = r1 - h2 (exact) has at most 8, so it is a BF16
// value itself.  Exact for every normal a whose remainders stay normal
// (|a| >= 2^-103); below that an entry loses at most its own magnitude.  Each
// term is returned as FP32 bits whose low 16 bits are zero.  Four VALU
// operations, against about fifteen for a split by rounding to nearest: 5.64
// -> 5.48 ms per BF16x3 launch at n = 65536 with 64 columns, once the terms
// are packed two k at a time (holding all 48 terms of a thread unpacked
// spilled registers and took 8.7 ms).
__device__ __forceinline__ void split3(float a, unsigned int& h1, unsigned int& h2, unsigned int& h3) {
  h1 = __float_as_uint(a) & 0xFFFF0000u;
  const float r1 = a - __uint_as_float(h1);
  h2 = __float_as_uint(r1) & 0xFFFF0000u;
  h3 = __float_as_uint(r1 - __uint_as_float(h2));
}

// two BF16 terms (the upper halves of lo and hi) in one 32-bit word, lo first
__device__ __forceinline__ unsigned int pack2(unsigned int lo, unsigned int hi) {
  return __builtin_amdgcn_perm(hi, lo, 0x07060302u);
}

// Position of k offset kk (a multiple of 4) in row `row` of the A slice in
// LDS: the 16-byte pieces of a row (four in a BF16 plane, eight in FP32) are
// permuted by bits 4.. of the row.  In the transposed product the 32 lanes
// of a store write rows 4 apart, which without the permutation fall on a
// quarter of the LDS banks (a modelled 16 passes per store instead of 4
// for BF16 and 8 for FP32); the reads of a 16-row MFMA block see the same
// permutation in every row, so they stay conflict-free.
template <int MODE>
__device__ __forceinline__ int swz(int row, int kk) {
  if constexpr (MODE == 2) return (((kk >> 3) ^ ((row >> 4) & 3)) << 3) | (kk & 7);
  else return (((kk >> 2) ^ ((row >> 4) & 7)) << 2) | (kk & 3);
}

template <int MODE, bool TRANS>
__device__ __forceinline__ void store_a(Smem<MODE>& sm, const float (&v)[16]) {
  const int tid = threadIdx.x;
  if (!TRANS) {  // rows 32 q + tid / 8, k = 4 (tid % 8) + e
    const int rb = tid >> 3, kq = 4 * (tid & 7);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if constexpr (MODE == 1) {
        *reinterpret_cast<float4*>(&sm.A[rb + 32 * q][swz<1>(rb + 32 * q, kq)]) =
            make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
      } else {
        unsigned int w[3][2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          unsigned int a1, a2, a3, b1, b2, b3;
          split3(v[4 * q + 2 * h], a1, a2, a3);
          split3(v[4 * q + 2 * h + 1], b1, b2, b3);
          w[0][h] = pack2(a1, b1);
          w[1][h] = pack2(a2, b2);
          w[2][h] = pack2(a3, b3);
        }
#pragma unroll
        for (int t = 0; t < 3; ++t)
          *reinterpret_cast<uint2*>(&sm.A[t][rb + 32 * q][swz<2>(rb + 32 * q, kq)]) = make_uint2(w[t][0], w[t][1]);
      }
    }
  } else {  // 4 rows of the tile (columns of A), 4 consecutive k each
    const int kq = 4 * (tid >> 5), rb = 4 * (tid & 31);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if constexpr (MODE == 1) {
        *reinterpret_cast<float4*>(&sm.A[rb + e][swz<1>(rb + e, kq)]) = make_float4(v[e], v[4 + e], v[8 + e], v[12 + e]);
      } else {
        unsigned int w[3][2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          unsigned int a1, a2, a3, b1, b2, b3;
          split3(v[8 * q + e], a1, a2, a3);
          split3(v[8 * q + 4 + e], b1, b2, b3);
          w[0][q] = pack2(a1, b1);
          w[1][q] = pack2(a2, b2);
          w[2][q] = pack2(a3, b3);
        }
#pragma unroll
        for (int t = 0; t < 3; ++t)
          *reinterpret_cast<uint2*>(&sm.A[t][rb + e][swz<2>(rb + e, kq)]) = make_uint2(w[t][0], w[t][1]);
      }
    }
  }
}

// This thread's piece of the R^T slice (columns c0 .. c0 + 63 of R, k0 ..
// k0 + 31): column c0 + tid / 4, k = k0 + 8 (tid % 4) + e, e < 8 -- 16 bytes
// in BF16, 32 in FP32, four consecutive lanes reading one column's slice.
// The workgroup stages the slice in LDS once for its four wavefronts (each
// loading its own operands from R^T read twice as many bytes, in pieces
// scattered over 16 columns per instruction).
template <int MODE>
struct RPiece {
  u32x4 w[MODE == 1 ? 2 : 1];
};

template <int MODE>
__device__ __forceinline__ void load_r(RPiece<MODE>& f, const typename RtType<MODE>::T* __restrict__ Rt,
                                       long long ldrt, int c0, int k0) {
  const int tid = threadIdx.x;
  const u32x4* p = reinterpret_cast<const u32x4*>(Rt + (long long)(c0 + (tid >> 2)) * ldrt + k0 + 8 * (tid & 3));
#pragma unroll
  for (int h = 0; h < (MODE == 1 ? 2 : 1); ++h) f.w[h] = p[h];
}

template <int MODE>
__device__ __forceinline__ void store_r(Smem<MODE>& sm, const RPiece<MODE>& f) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int h = 0; h < (MODE == 1 ? 2 : 1); ++h)
    *reinterpret_cast<u32x4*>(&sm.R[tid >> 2][8 * (tid & 3) + 4 * h]) = f.w[h];
}

// One 128 x 64 tile of S (rows i0.., columns c0..) over k in [kbeg, kend),
// written to out (leading dimension ldo).  Rt: R^T in the products'
// precision, ldrt >= kend rounded up to BK, columns up to c0 + BN present.
template <int MODE, bool TRANS>
__device__ __forceinline__ void sample_tile(Smem<MODE>& sm, const float* __restrict__ A,
                                            long long lda, int n, const int* __restrict__ leaf_of,
                                            const typename RtType<MODE>::T* __restrict__ Rt,
                                            long long ldrt, int ncols, int i0, int c0, int kbeg,
                                            int kend, double* __restrict__ out, long long ldo) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 15, lk = (lane >> 4) * 8;
  const int cbase = c0 + wn * 32;

  const bool vec_a = ((lda * 4) % 16 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
  int li0 = 0, li1 = -1;
  if (leaf_of) {
    li0 = leaf_of[min(i0, n - 1)];
    li1 = leaf_of[min(i0 + BM, n) - 1];
  }
  auto mask_for = [&](int k0) -> bool {
    if (!leaf_of || k0 >= kend) return false;
    const int lk0 = leaf_of[k0];
    const int lk1 = leaf_of[min(k0 + BK, kend) - 1];
    return !(lk1 < li0 || li1 < lk0);
  };

  f32x4 acc[4][2];
  double accd[4][2][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int r = 0; r < 4; ++r) accd[a][b][r] = 0.0;
    }

  float va[16];
  RPiece<MODE> rp;
  int k0 = kbeg;
  if (k0 < kend) {
    load_a<TRANS>(va, A, lda, n, i0, k0, kend, leaf_of, vec_a, mask_for(k0));
    load_r<MODE>(rp, Rt, ldrt, c0, k0);
    store_a<MODE, TRANS>(sm, va);
    store_r<MODE>(sm, rp);
  }
  __syncthreads();
  int since = 0;  // k values accumulated in FP32 since the last carry
  for (; k0 < kend; k0 += BK) {
    const int kn = k0 + BK;
    if (kn < kend) {
      load_a<TRANS>(va, A, lda, n, i0, kn, kend, leaf_of, vec_a, mask_for(kn));
      load_r<MODE>(rp, Rt, ldrt, c0, kn);
    }
    if constexpr (MODE == 1) {
      float b[2][8];
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        const float4 x = *reinterpret_cast<const float4*>(&sm.R[wn * 32 + nb * 16 + lr][lk]);
        const float4 y = *reinterpret_cast<const float4*>(&sm.R[wn * 32 + nb * 16 + lr][lk + 4]);
        b[nb][0] = x.x; b[nb][1] = x.y; b[nb][2] = x.z; b[nb][3] = x.w;
        b[nb][4] = y.x; b[nb][5] = y.y; b[nb][6] = y.z; b[nb][7] = y.w;
      }
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) {
        const int row = wm * 64 + mb * 16 + lr;
        const float4 x = *reinterpret_cast<const float4*>(&sm.A[row][swz<1>(row, lk)]);
        const float4 y = *reinterpret_cast<const float4*>(&sm.A[row][swz<1>(row, lk + 4)]);
        const float a[8] = {x.x, x.y, x.z, x.w, y.x, y.y, y.z, y.w};
#pragma unroll
        for (int e = 0; e < 8; ++e)
#pragma unroll
          for (int nb = 0; nb < 2; ++nb)
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e], b[nb][e], acc[mb][nb], 0, 0, 0);
      }
    } else {
      // multiplying wavefronts issue first (5.72 -> 5.62 ms per launch; the
      // FP32 mode runs slower with it: 6.71 -> 6.87 ms)
      bf16x8 b[2];
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) b[nb] = *reinterpret_cast<const bf16x8*>(&sm.R[wn * 32 + nb * 16 + lr][lk]);
      __builtin_amdgcn_s_setprio(1);
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        bf16x8 a[4];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
          a[mb] = *reinterpret_cast<const bf16x8*>(&sm.A[t][wm * 64 + mb * 16 + lr][swz<2>(wm * 64 + mb * 16 + lr, lk)]);
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
          for (int nb = 0; nb < 2; ++nb)
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mb], b[nb], acc[mb][nb], 0, 0, 0);
      }
      __builtin_amdgcn_s_setprio(0);
    }
    since += BK;
    if (since >= KF || kn >= kend) {  // carry the FP32 chunk sums into FP64
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
#pragma unroll
          for (int r = 0; r < 4; ++r) accd[mb][nb][r] += (double)acc[mb][nb][r];
          acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
      since = 0;
    }
    __syncthreads();
    if (kn < kend) {
      store_a<MODE, TRANS>(sm, va);
      store_r<MODE>(sm, rp);
    }
    __syncthreads();
  }

#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
      const int c = cbase + nb * 16 + lr;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wm * 64 + mb * 16 + 4 * (lane >> 4) + r;
        if (i < n && c < ncols) out[(long long)i * ldo + c] = accd[mb][nb][r];
      }
    }
}

template <int MODE, bool TRANS>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void sample_mixed_kernel(
    const float* __restrict__ A, long long lda, int n, const int* __restrict__ leaf_of,
    const typename RtType<MODE>::T* __restrict__ Rt, long long ldrt, double* __restrict__ S,
    long long lds, int ncols, int n_nt, int ksplit, int kchunk, double* __restrict__ work) {
  __shared__ Smem<MODE> sm;
  // consecutive logical tiles share an XCD
  const int nblk = gridDim.x;
  int L = blockIdx.x;
  if ((nblk & 7) == 0) L = (blockIdx.x & 7) * (nblk >> 3) + (blockIdx.x >> 3);
  const int nt = L % n_nt;
  const int rest = L / n_nt;
  const int ks = rest % ksplit;
  const int mt = rest / ksplit;
  const int kbeg = ks * kchunk;
  double* out = S;
  long long ldo = lds;
  if (ksplit > 1) {
    out = work + (long long)ks * n * ncols;
    ldo = ncols;
  }
  sample_tile<MODE, TRANS>(sm, A, lda, n, leaf_of, Rt, ldrt, ncols, mt * BM, nt * BN, kbeg,
                           min(n, kbeg + kchunk), out, ldo);
}

// Many matrices in one launch: descriptor q covers the tiles
// [tile0, tile0 + n_mt * n_nt) of its product; no split of k.
struct GroupDesc {
  const float* A;
  long long lda;
  int n, ncols, n_nt;
  const int* leaf_of;
  const void* Rt;
  long long ldrt;
  double* S;
  long long lds;
  long long tile0;
};

template <int MODE, bool TRANS>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void sample_mixed_grouped_kernel(const GroupDesc* __restrict__ g,
                                                                  int ng) {
  __shared__ Smem<MODE> sm;
  const long long b = blockIdx.x;
  int lo = 0, hi = ng - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (g[mid].tile0 <= b) lo = mid;
    else hi = mid - 1;
  }
  const GroupDesc d = g[lo];
  const int t = (int)(b - d.tile0);
  sample_tile<MODE, TRANS>(sm, d.A, d.lda, d.n, d.leaf_of,
                           static_cast<const typename RtType<MODE>::T*>(d.Rt), d.ldrt, d.ncols,
                           (t / d.n_nt) * BM, (t % d.n_nt) * BN, 0, d.n, d.S, d.lds);
}

__global__ void reduce_splits_mixed_kernel(const double* __restrict__ work, int ksplit, long long n,
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

// R^T in the products' precision: Rt[c][k] = R[k][c] for c < ncols, k < n,
// zero in the padding (columns up to whole tiles, k up to whole slices).
// R already holds values representable in that precision.
struct PrepDesc {
  const double* R;
  long long ldr;
  int n, ncols, cpad;
  long long ldrt;
  void* Rt;
  long long e0;  // first element of this descriptor in the launch
};

template <int MODE>
__global__ void prep_rt_kernel(const PrepDesc* __restrict__ g, int ng, long long total) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int lo = 0, hi = ng - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (g[mid].e0 <= e) lo = mid;
    else hi = mid - 1;
  }
  const PrepDesc d = g[lo];
  const long long x = e - d.e0;
  const int c = (int)(x / d.ldrt);
  const long long k = x % d.ldrt;
  const double v = (c < d.ncols && k < d.n) ? d.R[k * d.ldr + c] : 0.0;
  if constexpr (MODE == 1) static_cast<float*>(d.Rt)[x] = (float)v;
  else static_cast<unsigned short*>(d.Rt)[x] = bf16_rn((float)v);
}

// The same copy for at most two descriptors passed by value (one matrix, one
// or both sides): no table in device memory.
struct PrepPair {
  PrepDesc d[2];
};

template <int MODE>
__global__ void prep_rt_pair_kernel(PrepPair g, int ng, long long total) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const PrepDesc& d = (ng > 1 && g.d[1].e0 <= e) ? g.d[1] : g.d[0];
  const long long x = e - d.e0;
  const int c = (int)(x / d.ldrt);
  const long long k = x % d.ldrt;
  const double v = (c < d.ncols && k < d.n) ? d.R[k * d.ldr + c] : 0.0;
  if constexpr (MODE == 1) static_cast<float*>(d.Rt)[x] = (float)v;
  else static_cast<unsigned short*>(d.Rt)[x] = bf16_rn((float)v);
}

long long rt_ld(long long n) { return (n + BK - 1) / BK * BK; }
int rt_cols(int ncols) { return (ncols + BN - 1) / BN * BN; }
// doubles of workspace for one R^T copy (4-byte elements: enough for both modes)
long long rt_doubles(long long n, int ncols) { return (rt_ld(n) * rt_cols(ncols) * 4 + 7) / 8; }

hipError_t prep_rt(std::vector<PrepDesc>& g, int mode, Staging& st, hipStream_t s) {
  if (g.empty()) return hipSuccess;
  long long total = 0;
  for (PrepDesc& d : g) {
    d.e0 = total;
    total += (long long)d.cpad * d.ldrt;
  }
  const PrepDesc* dg = static_cast<const PrepDesc*>(st.push(g.data(), g.size() * sizeof(PrepDesc)));
  if (!dg) return hipErrorOutOfMemory;
  const dim3 grid((unsigned)((total + 255) / 256));
  if (mode == 1) hipLaunchKernelGGL(prep_rt_kernel<1>, grid, dim3(256), 0, s, dg, (int)g.size(), total);
  else hipLaunchKernelGGL(prep_rt_kernel<2>, grid, dim3(256), 0, s, dg, (int)g.size(), total);
  return hipGetLastError();
}

// R rounded in place to the precision of the products: FP32 (mode 1) or
// BF16 (mode 2), round to nearest even from the FP64 value itself.
__global__ void round_r_kernel(double* __restrict__ R, long long ld, long long n, int col0, int col1,
                               int mode) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int w = col1 - col0;
  if (idx >= n * w) return;
  double* p = R + (idx / w) * ld + col0 + (int)(idx % w);
  // BF16: keep 8 significant bits, rounding away the low 45 bits of the FP64
  // fraction (bias of half minus one, plus the kept lowest bit for ties)
  *p = round_sample_prec(*p, mode);
}

struct Plan {
  int n_mt, n_nt, ksplit, kchunk;
};

// Workgroups of the mixed kernel resident on the device at once (three per
// CU: the kernel is held to 168 registers for that).
int mixed_slots() {
  static const int v = [] {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per, reinterpret_cast<const void*>(&sample_mixed_kernel<2, false>), NT, 0) != hipSuccess)
      return 768;
    return std::max(1, per * cus);
  }();
  return v;
}

// The product streams A from HBM, so what counts is how many loads are in
// flight: K is split until the workgroups fill two whole rounds of the
// resident slots (n = 65536, 64 columns: 512 tiles x 3 splits = 1536
// workgroups on 768 slots; 6.47 -> 5.64 ms per BF16x3 launch together with
// the third resident workgroup per CU).
Plan make_plan(long long n, int ncols) {
  Plan p;
  p.n_mt = (int)((n + BM - 1) / BM);
  p.n_nt = (ncols + BN - 1) / BN;
  const long long tiles = (long long)p.n_mt * p.n_nt;
  long long want = (2LL * mixed_slots() + tiles - 1) / tiles;
  long long maxs = n / 1024;
  if (maxs < 1) maxs = 1;
  if (want > maxs) want = maxs;
  if (want < 1) want = 1;
  long long chunk = (n + want - 1) / want;
  chunk = (chunk + KF - 1) / KF * KF;  // split boundaries on carry boundaries
  p.ksplit = (int)((n + chunk - 1) / chunk);
  p.kchunk = (int)chunk;
  return p;
}

template <int MODE, bool TRANS>
void run(const float* A, long long lda, long long n, const int* leaf_of, int ncols, const void* Rt,
         double* S, long long lds, double* work, hipStream_t s) {
  Plan p = make_plan(n, ncols);
  const long long nblocks = (long long)p.n_mt * p.n_nt * p.ksplit;
  hipLaunchKernelGGL((sample_mixed_kernel<MODE, TRANS>), dim3((unsigned)nblocks), dim3(NT), 0, s, A,
                     lda, (int)n, leaf_of, static_cast<const typename RtType<MODE>::T*>(Rt), rt_ld(n),
                     S, lds, ncols, p.n_nt, p.ksplit, p.kchunk, work);
  if (p.ksplit > 1) {
    const long long total = n * ncols;
    hipLaunchKernelGGL(reduce_splits_mixed_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256),
                       0, s, work, p.ksplit, n, ncols, S, lds);
  }
}

}  // namespace

long long sample_mixed_workspace_doubles(long long n, int ncols) {
  Plan p = make_plan(n, ncols);
  return 2 * rt_doubles(n, ncols) + (p.ksplit > 1 ? (long long)p.ksplit * n * ncols : 0);
}

hipError_t launch_sample_mixed(const float* A, long long n, long long lda, const int* leaf_of,
                               int ncols, int mode, const double* Rr, const double* Rc,
                               long long ldr, double* Sr, double* Sc, long long lds, double* work,
                               hipStream_t s) {
  if (n <= 0 || ncols <= 0) return hipSuccess;
  // work: [R^T of R^r | R^T of R^c | split-k partials]
  double* rt_r = work;
  double* rt_c = work + rt_doubles(n, ncols);
  double* part = work + 2 * rt_doubles(n, ncols);
  PrepPair g{};
  int ng = 0;
  long long total = 0;
  for (int side = 0; side < 2; ++side) {
    if (!(side ? Sc : Sr)) continue;
    g.d[ng] = PrepDesc{side ? Rc : Rr, ldr, (int)n, ncols, rt_cols(ncols), rt_ld(n), side ? rt_c : rt_r, total};
    total += (long long)g.d[ng].cpad * g.d[ng].ldrt;
    ++ng;
  }
  if (ng == 0) return hipSuccess;
  const dim3 pgrid((unsigned)((total + 255) / 256));
  if (mode == 1) hipLaunchKernelGGL(prep_rt_pair_kernel<1>, pgrid, dim3(256), 0, s, g, ng, total);
  else hipLaunchKernelGGL(prep_rt_pair_kernel<2>, pgrid, dim3(256), 0, s, g, ng, total);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (mode == 1) {
    if (Sr) run<1, false>(A, lda, n, leaf_of, ncols, rt_r, Sr, lds, part, s);
    if (Sc) run<1, true>(A, lda, n, leaf_of, ncols, rt_c, Sc, lds, part, s);
  } else {
    if (Sr) run<2, false>(A, lda, n, leaf_of, ncols, rt_r, Sr, lds, part, s);
    if (Sc) run<2, true>(A, lda, n, leaf_of, ncols, rt_c, Sc, lds, part, s);
  }
  return hipGetLastError();
}

long long sample_mixed_grouped_workspace_doubles(const SampleJob* jobs, int njob) {
  long long t = 0;
  for (int q = 0; q < njob; ++q)
    if (jobs[q].n > 0 && jobs[q].ncols > 0) t += 2 * rt_doubles(jobs[q].n, jobs[q].ncols);
  return t;
}

hipError_t launch_sample_mixed_grouped(const SampleJob* jobs, int njob, int mode, double* work,
                                       Staging& st, hipStream_t s) {
  if (njob <= 0) return hipSuccess;
  // the R^T copies of every job and side, then one launch per side
  std::vector<PrepDesc> pd;
  std::vector<double*> rts(2 * (size_t)njob, nullptr);
  long long off = 0;
  for (int q = 0; q < njob; ++q) {
    const SampleJob& j = jobs[q];
    if (j.n <= 0 || j.ncols <= 0) continue;
    for (int side = 0; side < 2; ++side) {
      rts[2 * q + side] = work + off;
      pd.push_back(PrepDesc{side == 0 ? j.Rr : j.Rc, j.ldr, (int)j.n, j.ncols, rt_cols(j.ncols),
                            rt_ld(j.n), work + off, 0});
      off += rt_doubles(j.n, j.ncols);
    }
  }
  hipError_t e = prep_rt(pd, mode, st, s);
  if (e != hipSuccess) return e;
  for (int side = 0; side < 2; ++side) {
    std::vector<GroupDesc> g;
    long long tiles = 0;
    for (int q = 0; q < njob; ++q) {
      const SampleJob& j = jobs[q];
      if (j.n <= 0 || j.ncols <= 0) continue;
      GroupDesc d{};
      d.A = j.A;
      d.lda = j.lda;
      d.n = (int)j.n;
      d.ncols = j.ncols;
      d.n_nt = (j.ncols + BN - 1) / BN;
      d.leaf_of = j.leaf_of;
      d.Rt = rts[2 * q + side];
      d.ldrt = rt_ld(j.n);
      d.S = side == 0 ? j.Sr : j.Sc;
      d.lds = j.lds;
      d.tile0 = tiles;
      tiles += (long long)((j.n + BM - 1) / BM) * d.n_nt;
      g.push_back(d);
    }
    if (g.empty()) return hipSuccess;
    const GroupDesc* dg = static_cast<const GroupDesc*>(st.push(g.data(), g.size() * sizeof(GroupDesc)));
    if (!dg) return hipErrorOutOfMemory;
    const int ng = (int)g.size();
    if (mode == 1) {
      if (side == 0) hipLaunchKernelGGL((sample_mixed_grouped_kernel<1, false>), dim3((unsigned)tiles), dim3(NT), 0, s, dg, ng);
      else hipLaunchKernelGGL((sample_mixed_grouped_kernel<1, true>), dim3((unsigned)tiles), dim3(NT), 0, s, dg, ng);
    } else {
      if (side == 0) hipLaunchKernelGGL((sample_mixed_grouped_kernel<2, false>), dim3((unsigned)tiles), dim3(NT), 0, s, dg, ng);
      else hipLaunchKernelGGL((sample_mixed_grouped_kernel<2, true>), dim3((unsigned)tiles), dim3(NT), 0, s, dg, ng);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

void launch_round_r(double* R, long long ld, long long n, int col0, int col1, int mode,
                    hipStream_t s) {
  const long long total = n * (long long)(col1 - col0);
  if (total <= 0 || mode == 0) return;
  hipLaunchKernelGGL(round_r_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, R, ld,
                     n, col0, col1, mode);
}

}  // namespace hss
