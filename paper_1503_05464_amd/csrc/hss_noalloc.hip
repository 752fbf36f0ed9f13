// Allocation-free variant of the sampling products (hss_sample_noalloc).
//
// hss_sample takes its workspace (split-K partial sums and, in the reduced
// modes, the copies of R in the products' precision) from the device pool.
// This variant takes it from one fixed array of device memory that the
// library holds for the life of the process, so a call allocates nothing:
// no hipMalloc, no hipFree, no pool, no pinned staging.  The kernels and
// their launch plans are those of hss_sample, so both give the same bits.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "hss_handle.h"

namespace {

// 2^24 doubles (128 MiB): enough for the sampling workspace of n = 65536 with
// 64 columns in every precision (FP64 needs 64 MiB there, FP32 / BF16x3 128).
constexpr long long kScratchDoubles = 1LL << 24;

// The array itself.  Its name is a host-side stand-in for the symbol: host
// code passes only the device address obtained below, never the name.
static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mu;
std::vector<double*> g_scratch_ptr;  // per device, null until looked up

// The device address of `scratch` on the current device: looked up once per
// device, with that device current, and kept.  Null on failure (error set).
double* scratch_of_current_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) {
    (void)hipGetLastError();
    hss::set_error(HSS_ERR_HIP, "hipGetDevice failed");
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      hss::set_error(HSS_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return nullptr;
    }
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

hss_status hss_sample_noalloc(const void* A, int dtype, int sample_prec, long long n, long long lda,
                              const int* leaf_of, int ncols, const double* Rr, const double* Rc,
                              long long ldr, double* Sr, double* Sc, long long lds, void* stream) {
  hss::set_error(HSS_OK, "");
  long long wd = 0;
  const hss_status st = hss::sample_args(A, dtype, sample_prec, n, lda, ncols, Rr, Rc, ldr, Sr, Sc, lds, &wd);
  if (st != HSS_OK) return st;
  if (wd > kScratchDoubles)
    return hss::set_error(HSS_ERR_ARG, "hss_sample_noalloc: these sizes need " + std::to_string(wd) +
                                           " doubles of workspace; its fixed scratch holds " +
                                           std::to_string(kScratchDoubles));
  double* work = nullptr;
  if (wd > 0) {
    work = scratch_of_current_device();
    if (!work) return HSS_ERR_HIP;
  }
  // every word of scratch a call reads is written earlier in the same call
  // (partial sums are stored, not accumulated; the R copies are written whole,
  // padding included), so nothing is cleared
  const hipError_t e = hss::sample_queue(A, dtype, sample_prec, n, lda, leaf_of, ncols, Rr, Rc, ldr, Sr, Sc,
                                         lds, work, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hss::set_error(HSS_ERR_HIP, std::string("sampling launch: ") + hipGetErrorString(e));
  return HSS_OK;
}

}  // extern "C"
