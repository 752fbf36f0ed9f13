// Small data-movement kernels of compression: extraction of the leaf
// diagonal blocks D = A(I, I) and of the coupling blocks
// B_ab = A(I^r_a, I^c_b), B_ba = A(I^r_b, I^c_a) (Alg. 1), composition of the
// skeleton index sets I_tau = I_in(J) (Alg. 1), and the leaf ordinal of
// every index (used to mask the leaf diagonal blocks out of the sampling
// product).
#include "hss_internal.h"

namespace hss {
namespace {

constexpr int NT = 256;

struct DevGather {
  GatherDesc g;
  long long row0;  // first flattened output row of this problem
};

// one workgroup per output row; threads over the columns
template <typename TA>
__global__ __launch_bounds__(NT) void gather_kernel(const TA* __restrict__ A, long long lda,
                                                    const DevGather* __restrict__ descs,
                                                    int nprob) {
  const long long t = blockIdx.x;
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].row0 <= t) lo = mid;
    else hi = mid - 1;
  }
  const GatherDesc& g = descs[lo].g;
  const int r = (int)(t - descs[lo].row0);
  const long long ar = g.rows ? g.rows[r] : (long long)g.row_off + r;
  const TA* arow = g.A ? static_cast<const TA*>(g.A) + ar * g.lda : A + ar * lda;
  double* out = g.out + (long long)r * g.ldo;
  for (int c = threadIdx.x; c < g.nc; c += NT) {
    const long long ac = g.cols ? g.cols[c] : (long long)g.col_off + c;
    out[c] = (double)arow[ac];
  }
}

__global__ __launch_bounds__(NT) void index_kernel(const IndexDesc* __restrict__ descs) {
  const IndexDesc g = descs[blockIdx.x];
  for (int a = threadIdx.x; a < g.k; a += NT) {
    const int q = g.perm[a];
    int v;
    if (q < g.split) v = g.b0 ? g.b0[q] : g.off0 + q;
    else v = g.b1[q - g.split];
    g.out[a] = v;
  }
}

__global__ void leaf_of_kernel(const int* __restrict__ lo, const int* __restrict__ hi,
                               int* __restrict__ leaf_of) {
  const int l = blockIdx.x;
  for (int i = lo[l] + threadIdx.x; i < hi[l]; i += blockDim.x) leaf_of[i] = l;
}

}  // namespace

hipError_t launch_gather(const void* A, int dtype, long long lda, const GatherDesc* descs,
                         int nprob, Staging& st, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  DevGather* h = new DevGather[nprob];
  long long rows = 0;
  int kept = 0;
  for (int p = 0; p < nprob; ++p) {
    if (descs[p].nr <= 0 || descs[p].nc <= 0) continue;
    h[kept].g = descs[p];
    h[kept].row0 = rows;
    rows += descs[p].nr;
    ++kept;
  }
  hipError_t err = hipSuccess;
  if (kept > 0) {
    void* dd = st.push(h, sizeof(DevGather) * kept);
    if (!dd) {
      err = hipErrorOutOfMemory;
    } else if (dtype == 1) {
      hipLaunchKernelGGL(gather_kernel<float>, dim3((unsigned)rows), dim3(NT), 0, s,
                         static_cast<const float*>(A), lda, static_cast<const DevGather*>(dd), kept);
      err = hipGetLastError();
    } else {
      hipLaunchKernelGGL(gather_kernel<double>, dim3((unsigned)rows), dim3(NT), 0, s,
                         static_cast<const double*>(A), lda, static_cast<const DevGather*>(dd), kept);
      err = hipGetLastError();
    }
  }
  delete[] h;
  return err;
}

hipError_t launch_index_compose(const IndexDesc* descs, int nprob, Staging& st, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  void* dd = st.push(descs, sizeof(IndexDesc) * nprob);
  if (!dd) return hipErrorOutOfMemory;
  hipLaunchKernelGGL(index_kernel, dim3(nprob), dim3(NT), 0, s, static_cast<const IndexDesc*>(dd));
  return hipGetLastError();
}

void launch_leaf_of(int n_leaves, const int* lo_dev, const int* hi_dev, int* leaf_of, hipStream_t s) {
  if (n_leaves <= 0) return;
  hipLaunchKernelGGL(leaf_of_kernel, dim3(n_leaves), dim3(NT), 0, s, lo_dev, hi_dev, leaf_of);
}

}  // namespace hss
