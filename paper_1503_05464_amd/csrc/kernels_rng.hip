// Gaussian random matrices R^r, R^c from Philox4x64-10 (Salmon, Moraes,
// Dror, Shaw, SC'11) and the Box-Muller transform.
//
// The paper draws its random vectors with rand() or a Mersenne Twister
// (Sec. 3.2); both are sequential.  A counter-based generator gives entry
// (i, j) of R from its address alone, so every thread fills its own entries
// and the columns appended when d grows (Sec. 3.3) never depend on what was
// drawn before.
//
// Entry (i, j) of stream `which`: key (seed, 0), counter (i/4, j, which, 0);
// the four 64-bit output words w0..w3 become u = ((w >> 12) + 1/2) 2^-52 and
// rows 4q, 4q+1 take the Box-Muller pair of (u0, u1), rows 4q+2, 4q+3 that of
// (u2, u3): sqrt(-2 ln ua) cos(2 pi ub), sqrt(-2 ln ua) sin(2 pi ub).
#include <vector>

#include "hss_internal.h"

namespace hss {
namespace {

struct U64x4 {
  unsigned long long v[4];
};

__device__ __forceinline__ U64x4 philox4x64_10(unsigned long long c0, unsigned long long c1,
                                               unsigned long long c2, unsigned long long c3,
                                               unsigned long long k0, unsigned long long k1) {
  const unsigned long long M0 = 0xD2E7470EE14C6C93ull;
  const unsigned long long M1 = 0xCA5A826395121157ull;
  const unsigned long long W0 = 0x9E3779B97F4A7C15ull;
  const unsigned long long W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    unsigned long long hi0 = __umul64hi(M0, c0);
    unsigned long long lo0 = M0 * c0;
    unsigned long long hi1 = __umul64hi(M1, c2);
    unsigned long long lo1 = M1 * c2;
    unsigned long long n0 = hi1 ^ c1 ^ k0;
    unsigned long long n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  U64x4 o;
  o.v[0] = c0;
  o.v[1] = c1;
  o.v[2] = c2;
  o.v[3] = c3;
  return o;
}

__device__ __forceinline__ double to_unit(unsigned long long w) {
  return ((double)(w >> 12) + 0.5) * 0x1p-52;
}

// grid: x covers columns (fastest, coalesced row writes), y covers row quads.
__global__ void random_normal_kernel(unsigned long long seed, int which, long long n, int col0,
                                     int ncol, double* __restrict__ R, long long ld, int ncb) {
  const int cb = blockIdx.x % ncb;
  const long long qb = blockIdx.x / ncb;
  const int c = cb * blockDim.x + threadIdx.x;
  const long long q = qb * blockDim.y + threadIdx.y;
  if (c >= ncol || 4 * q >= n) return;
  U64x4 w = philox4x64_10((unsigned long long)q, (unsigned long long)(col0 + c),
                          (unsigned long long)which, 0ull, seed, 0ull);
  const double two_pi = 2.0 * 3.14159265358979323846;
  double u0 = to_unit(w.v[0]), u1 = to_unit(w.v[1]);
  double u2 = to_unit(w.v[2]), u3 = to_unit(w.v[3]);
  double r01 = sqrt(-2.0 * log(u0));
  double r23 = sqrt(-2.0 * log(u2));
  double t01 = two_pi * u1, t23 = two_pi * u3;
  double z[4] = {r01 * cos(t01), r01 * sin(t01), r23 * cos(t23), r23 * sin(t23)};
  const long long row0 = 4 * q;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if (row0 + r < n) R[(row0 + r) * ld + c] = z[r];
  }
}

// Many (matrix, side) column ranges in one launch: job q covers the flattened
// blocks [b0, b0 + nb) of the layout above; entries rounded to `mode`.
struct RngDesc {
  RngJob j;
  long long b0;
  int ncb;
};

__global__ void random_normal_batched_kernel(const RngDesc* __restrict__ jobs, int njob, int mode) {
  const long long b = blockIdx.x;
  int lo = 0, hi = njob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].b0 <= b) lo = mid;
    else hi = mid - 1;
  }
  const RngDesc& d = jobs[lo];
  const long long local = b - d.b0;
  const int cb = (int)(local % d.ncb);
  const long long qb = local / d.ncb;
  const int c = cb * blockDim.x + threadIdx.x;
  const long long q = qb * blockDim.y + threadIdx.y;
  const long long n = d.j.n;
  if (c >= d.j.ncol || 4 * q >= n) return;
  U64x4 w = philox4x64_10((unsigned long long)q, (unsigned long long)(d.j.col0 + c),
                          (unsigned long long)d.j.which, 0ull, d.j.seed, 0ull);
  const double two_pi = 2.0 * 3.14159265358979323846;
  double u0 = to_unit(w.v[0]), u1 = to_unit(w.v[1]);
  double u2 = to_unit(w.v[2]), u3 = to_unit(w.v[3]);
  double r01 = sqrt(-2.0 * log(u0));
  double r23 = sqrt(-2.0 * log(u2));
  double t01 = two_pi * u1, t23 = two_pi * u3;
  double z[4] = {r01 * cos(t01), r01 * sin(t01), r23 * cos(t23), r23 * sin(t23)};
  const long long row0 = 4 * q;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if (row0 + r < n) d.j.R[(row0 + r) * d.j.ld + c] = round_sample_prec(z[r], mode);
  }
}

}  // namespace

hipError_t launch_random_normal_batched(const RngJob* jobs, int njob, int mode, Staging& st,
                                        hipStream_t s) {
  std::vector<RngDesc> h;
  h.reserve(njob);
  long long blocks = 0;
  for (int q = 0; q < njob; ++q) {
    const RngJob& j = jobs[q];
    if (j.ncol <= 0 || j.n <= 0) continue;
    RngDesc d;
    d.j = j;
    d.ncb = (j.ncol + 63) / 64;
    d.b0 = blocks;
    blocks += (long long)d.ncb * (((j.n + 3) / 4 + 3) / 4);
    h.push_back(d);
  }
  if (h.empty()) return hipSuccess;
  const RngDesc* dd = static_cast<const RngDesc*>(st.push(h.data(), h.size() * sizeof(RngDesc)));
  if (!dd) return hipErrorOutOfMemory;
  hipLaunchKernelGGL(random_normal_batched_kernel, dim3((unsigned)blocks), dim3(64, 4), 0, s, dd, (int)h.size(),
                     mode);
  return hipGetLastError();
}

void launch_random_normal(unsigned long long seed, int which, long long n, int col0, int col1,
                          double* R, long long ld, hipStream_t s) {
  const int ncol = col1 - col0;
  if (ncol <= 0 || n <= 0) return;
  dim3 block(64, 4);
  long long nq = (n + 3) / 4;
  int ncb = (ncol + 63) / 64;
  long long nblocks = (long long)ncb * ((nq + 3) / 4);
  hipLaunchKernelGGL(random_normal_kernel, dim3((unsigned)nblocks), block, 0, s, seed, which, n, col0,
                     ncol, R, ld, ncb);
}

}  // namespace hss
