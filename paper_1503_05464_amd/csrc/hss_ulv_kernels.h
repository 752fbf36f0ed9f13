// Descriptors and launchers of the ULV kernels (kernels_ulv.hip).
#pragma once

#include "hss_internal.h"

namespace hss {

struct VtLeafDesc {  // V^T of a leaf written as k rows of Z (m columns)
  double* Z;
  long long ldz;
  int m, k;
  const int* perm;   // J then rest
  const double* E;   // (m-k) x k
};

struct TriDesc {     // X <- T^{-1} X on one diagonal block (nb <= 64)
  const double* T;
  long long ldt;
  double* X;
  long long ldx;
  int nb, nrhs;
  int lower, unit;
};

struct ReflDesc {    // V <- H_0 ... H_{r-1} V (transpose = 1), reflectors in rows of Z
  const double* Z;
  long long ldz;
  const double* tau;
  int r, m;
  double* V;
  long long ldv;
  int nrhs;
  int transpose;
  const double* Y = nullptr;  // precomputed dense Y and block factors T (both or
  const double* T = nullptr;  // neither): then Z is not read
};

// Blocked application of reflectors (compact WY form): the reflector
// vectors as columns of a dense Y, and the triangular factor of each block
// of 64 of them.
struct ReflYDesc {   // Y[q][i] = u_i[q] (m x r, ld r) from the rows of Z
  const double* Z;
  long long ldz;
  double* Y;
  int r, m;
};
struct SumDesc {     // out (rows x cols, ld ldo) = sum of parts partials (ld cols, stride apart)
  const double* part;
  long long stride;
  int parts, rows, cols;
  double* out;
  long long ldo;
};
hipError_t launch_sum_partials(const SumDesc* d, int nd, Staging& st, hipStream_t s);
struct LarftDesc {   // T (kb x kb, ld 64) of reflectors i0..i0+kb-1 from G = Y_b^T Y_b (ld 64)
  const double* G;
  const double* tau;  // tau of the block's first reflector
  double* T;
  int kb;
};
hipError_t launch_refl_y(const ReflYDesc* d, int nd, int rmax, int mmax, Staging& st, hipStream_t s);
hipError_t launch_larft(const LarftDesc* d, int nd, Staging& st, hipStream_t s);

hipError_t launch_vt_leaf(const VtLeafDesc* d, int nd, int kmax, Staging& st, hipStream_t s);
hipError_t launch_tri_block(const TriDesc* d, int nd, Staging& st, hipStream_t s);
hipError_t launch_lu_panel(double* A, long long ld, int n, int j0, int nb, int* piv, int* info,
                           hipStream_t s);
hipError_t launch_lu_swap(double* A, long long ld, int ncols, const int* piv, int j0, int nb,
                          int skip0, int skip1, hipStream_t s);

}  // namespace hss
