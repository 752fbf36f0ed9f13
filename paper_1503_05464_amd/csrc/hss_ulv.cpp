// ULV-like factorization (Alg. 3) and solve (Alg. 4) of an HSS handle.
#include <hip/hip_runtime.h>

#include "hss_handle.h"

extern "C" {

hss_status hss_factor(hss_handle h, void* stream) {
  (void)stream;
  if (!h) return HSS_ERR_ARG;
  return HSS_ERR_STATE;
}

hss_status hss_solve(hss_handle h, int nrhs, const double* b, long long ldb, double* x,
                     long long ldx, void* stream) {
  (void)nrhs;
  (void)b;
  (void)ldb;
  (void)x;
  (void)ldx;
  (void)stream;
  if (!h) return HSS_ERR_ARG;
  return HSS_ERR_STATE;
}

}  // extern "C"
