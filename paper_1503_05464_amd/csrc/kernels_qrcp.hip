// Batched interpolative decomposition [X, J] = ID(Y, eps) by Householder QR
// with column pivoting, stopped at the first pivot with |R_ii| <= eps |R_11|
// (Sec. 2.2; the modified xGEQP3 of Sec. 3.2).
//
// Problem q holds Y_q (d x m) as the m rows of a row-major matrix (the rows
// of a node's local sample), so "column j of Y" is a contiguous vector.
// Pivot rule: largest remaining 2-norm, lowest column index on ties; the
// remaining norms are recomputed exactly after every reflection (no
// downdating), so small tolerances keep their accuracy.  Columns are never
// swapped: a per-column step number marks the pivots and R(i, j) stays in
// row i of column j's storage.
//
// Two factorization kernels, chosen per problem by size:
//  * small problems (m <= 256, d <= 192): one workgroup of RW wavefronts holds
//    the whole matrix in registers (wavefront w owns columns w, w+RW, ...;
//    lane l owns rows l, l+64, ...) and runs every pivot step without
//    touching global memory;
//  * large problems: one launch per pivot step for the whole batch; a problem
//    is split over ceil(m/8) workgroups of 8 wavefronts, one column per
//    wavefront; every workgroup of a problem selects the same pivot from the
//    same per-workgroup candidates (double-buffered between steps so no
//    workgroup waits on another), builds the same reflector from the pivot
//    column, and updates its own columns.  Kernel boundaries order the steps.
// A finishing pass forms J (pivot order) and the other columns in increasing
// order, and E = (R1^{-1} R2)^T by a blocked triangular solve whose
// off-diagonal updates run on the batched GEMM.  It is skipped for IDs the
// caller rejects.
//
// Early exit: when the caller's fail rule (rank above d - p_margin and below
// m) is certain -- more than kfail pivots accepted and m > d, so the rank can
// not reach m -- the factorization stops; the reported rank is then a lower
// bound that still trips the rule.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "hss_internal.h"

namespace hss {
namespace {

struct DevProb {
  IdProblem p;
  long long off;    // into the per-column arrays (sum of m)
  long long aoff;   // into the per-step arrays (sum of kmax)
  int kmax;         // min(m, d)
  int g0;           // first workgroup of this problem (large path)
  int G;            // workgroups of this problem (large path)
};

constexpr int NT = 256;      // threads of the finishing kernels
constexpr int SW = 8;        // wavefronts (= columns) per step workgroup
constexpr int ST = SW * 64;  // threads per step workgroup

struct Work {
  double* nrm;   // 2 * sum(m): double-buffered norms
  int* step;     // sum(m): pivot step of each column, -1 if not selected
  double* alpha; // sum(kmax): R_ii
  int* piv;      // sum(kmax): pivot column of step i
  int* k;        // nprob
  int* done;     // nprob
  double* nu0;   // nprob
  int* ndone;    // 1
  double* cand_v;  // 2 * tg: per-workgroup pivot candidates (step parity)
  int* cand_i;     // 2 * tg
  unsigned long long* cbuf;  // 2 * min(tg, kCandSlots) * 2 * ldcb: candidate columns as
                             // tagged words (persistent path), zeroed before each launch
  long long ldcb;  // max d rounded up to a multiple of 512 (a whole column of registers)
  long long nslots;  // min(tg, kCandSlots): workgroups a persistent launch may have
  long long krec;    // max kmax: steps a persistent launch may publish
  unsigned long long* rec;  // 2 * nslots * kmax: one published candidate record per
                            // workgroup and step, zeroed before each persistent launch
  long long rstride = 0;    // records per workgroup in a launch (its largest kmax): the
                            // records of workgroup g are rec[2 (g rstride + step) ...]
  int rmask = 1;   // column slots per workgroup in a persistent launch, minus one (a power of two)
  int xmask = 0;   // steps between full record exchanges, minus one: (rmask + 1) / 2 - 1
  int* err;        // 1: a wait for a candidate timed out (persistent path)
  int give_up = 0; // nonzero: every wait gives up at once (tests of the rerun)
  double* W;     // sum(m * d)
  double* W2;    // sum(m * d) of the problems factored in place without pivoting:
                 // their persistent launches write here, then copy back
};

size_t al(size_t b) { return (b + 255) / 256 * 256; }

// persistent path: at most this many workgroups per launch (candidate
// column slots per step parity), and the stride of a published column
constexpr long long kCandSlots = 1024;
long long ldcb_of(long long dmax) { return (dmax + 511) / 512 * 512; }

// pivot steps a problem can take
int kmax_of(const IdProblem& p) {
  const int k = std::min(p.m, p.d);
  return p.nfac > 0 ? std::min(p.nfac, k) : k;
}

// a problem factored without pivoting in place (W == Y, the ULV's LQ)
static bool is_inplace_nopiv(const IdProblem& p) { return p.nfac > 0 && p.W != nullptr && p.W == p.Y; }
static long long inplace_nopiv_doubles(const IdProblem* probs, int nprob) {
  long long t = 0;
  for (int q = 0; q < nprob; ++q)
    if (is_inplace_nopiv(probs[q])) t += (long long)probs[q].m * probs[q].d;
  return t;
}

void carve(const IdProblem* probs, int nprob, void* base, Work& w, long long& tm, long long& tk,
           long long& tw) {
  tm = tk = tw = 0;
  long long tg = 0, dm = 1, km = 1;
  for (int q = 0; q < nprob; ++q) {
    tg += (probs[q].m + SW - 1) / SW;
    tm += probs[q].m;
    tk += kmax_of(probs[q]);
    km = std::max<long long>(km, kmax_of(probs[q]));
    dm = std::max<long long>(dm, probs[q].d);
    if (!probs[q].W) tw += (long long)probs[q].m * probs[q].d;
  }
  char* c = static_cast<char*>(base);
  auto take = [&](size_t b) {
    char* r = c;
    c += al(b ? b : 1);
    return r;
  };
  w.nrm = reinterpret_cast<double*>(take(2 * tm * 8));
  w.step = reinterpret_cast<int*>(take(tm * 4));
  w.alpha = reinterpret_cast<double*>(take(tk * 8));
  w.piv = reinterpret_cast<int*>(take(tk * 4));
  w.k = reinterpret_cast<int*>(take((size_t)nprob * 4));
  w.done = reinterpret_cast<int*>(take((size_t)nprob * 4));
  w.nu0 = reinterpret_cast<double*>(take((size_t)nprob * 8));
  w.ndone = reinterpret_cast<int*>(take(4));
  w.cand_v = reinterpret_cast<double*>(take(2 * tg * 8));
  w.cand_i = reinterpret_cast<int*>(take(2 * tg * 4));
  w.ldcb = ldcb_of(dm);
  w.nslots = std::min(tg, kCandSlots);
  w.cbuf = reinterpret_cast<unsigned long long*>(take(2 * w.nslots * 2 * w.ldcb * 8));
  w.krec = km;
  w.rec = reinterpret_cast<unsigned long long*>(take(2 * w.nslots * km * 8));
  w.err = reinterpret_cast<int*>(take(4));
  w.W = reinterpret_cast<double*>(take(tw * 8));
  w.W2 = reinterpret_cast<double*>(take(inplace_nopiv_doubles(probs, nprob) * 8));
}

// wavefront sums of N values at once: butterfly over lanes, the first four
// levels by DPP (quad permutes, then half-row and row mirrors), the last two
// across rows by gfx950's v_permlane16_swap / v_permlane32_swap (register
// swaps between the rows of two registers, no LDS crossbar).  Every lane
// ends with the same sums.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
// A lane's own value and that of its partner across 16 lanes (W = 16: rows
// 0 <-> 1, 2 <-> 3) or 32 lanes (W = 32: the two halves), in an order that
// depends on the lane: swapping the rows of two copies of v leaves one copy
// with the even rows (lower half) twice and the other with the odd rows
// (upper half) twice.
template <int W>
__device__ __forceinline__ void cross_pair(double v, double& a, double& b) {
  unsigned alo = (unsigned)__double2loint(v), ahi = (unsigned)__double2hiint(v);
  unsigned blo = alo, bhi = ahi;
  if (W == 16) {
    const auto l = __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
    alo = l[0], blo = l[1], ahi = h[0], bhi = h[1];
  } else {
    const auto l = __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
    alo = l[0], blo = l[1], ahi = h[0], bhi = h[1];
  }
  a = __hiloint2double((int)ahi, (int)alo);
  b = __hiloint2double((int)bhi, (int)blo);
}
template <int W>
__device__ __forceinline__ void cross_pair_i(int v, int& a, int& b) {
  unsigned x = (unsigned)v, y = x;
  const auto r = W == 16 ? __builtin_amdgcn_permlane16_swap(x, y, false, false)
                         : __builtin_amdgcn_permlane32_swap(x, y, false, false);
  a = (int)r[0];
  b = (int)r[1];
}
// The last two levels either by cross-row shuffles (ds_bpermute, through the
// LDS crossbar) or by the permlane swaps (VALU).  The swaps serve the
// persistent kernel (IDs 484 -> 471 ms per gauss65536 compression); the
// reduction-heavy small-problem kernel runs 40 % slower with them and keeps
// the shuffles.
template <int N>
__device__ __forceinline__ void wave_sum_n(double (&v)[N]) {
#pragma unroll
  for (int c = 0; c < N; ++c) v[c] += dpp_d<0xB1>(v[c]);  // quad_perm [1,0,3,2]
#pragma unroll
  for (int c = 0; c < N; ++c) v[c] += dpp_d<0x4E>(v[c]);  // quad_perm [2,3,0,1]
#pragma unroll
  for (int c = 0; c < N; ++c) v[c] += dpp_d<0x141>(v[c]);  // row_half_mirror
#pragma unroll
  for (int c = 0; c < N; ++c) v[c] += dpp_d<0x140>(v[c]);  // row_mirror
#pragma unroll
  for (int c = 0; c < N; ++c) v[c] += __shfl_xor(v[c], 16, 64);
#pragma unroll
  for (int c = 0; c < N; ++c) v[c] += __shfl_xor(v[c], 32, 64);
}
template <int N>
__device__ __forceinline__ void wave_sum_n_pl(double (&v)[N]) {
#pragma unroll
  for (int c = 0; c < N; ++c) v[c] += dpp_d<0xB1>(v[c]);
#pragma unroll
  for (int c = 0; c < N; ++c) v[c] += dpp_d<0x4E>(v[c]);
#pragma unroll
  for (int c = 0; c < N; ++c) v[c] += dpp_d<0x141>(v[c]);
#pragma unroll
  for (int c = 0; c < N; ++c) v[c] += dpp_d<0x140>(v[c]);
  // own + partner in either order: the same sum (addition commutes)
#pragma unroll
  for (int c = 0; c < N; ++c) {
    double a, b;
    cross_pair<16>(v[c], a, b);
    v[c] = a + b;
  }
#pragma unroll
  for (int c = 0; c < N; ++c) {
    double a, b;
    cross_pair<32>(v[c], a, b);
    v[c] = a + b;
  }
}

// wavefront sum of one value, by the same butterfly (four DPP levels, two
// cross-row shuffles); every lane ends with the sum
__device__ __forceinline__ double wave_sum(double v) {
  double a[1] = {v};
  wave_sum_n<1>(a);
  return a[0];
}

__device__ __forceinline__ void better(double& bv, int& bi, double ov, int oi) {
  if (ov > bv || (ov == bv && oi < bi)) {
    bv = ov;
    bi = oi;
  }
}

// wavefront argmax of (value, index) under `better`, by the same butterfly
// as wave_sum_n: the order is total, so every lane ends with the same pair
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ void wave_argmax(double& bv, int& bi) {
  better(bv, bi, dpp_d<0xB1>(bv), dpp_i<0xB1>(bi));
  better(bv, bi, dpp_d<0x4E>(bv), dpp_i<0x4E>(bi));
  better(bv, bi, dpp_d<0x141>(bv), dpp_i<0x141>(bi));
  better(bv, bi, dpp_d<0x140>(bv), dpp_i<0x140>(bi));
  better(bv, bi, __shfl_xor(bv, 16, 64), __shfl_xor(bi, 16, 64));
  better(bv, bi, __shfl_xor(bv, 32, 64), __shfl_xor(bi, 32, 64));
}
__device__ __forceinline__ void wave_argmax_pl(double& bv, int& bi) {
  better(bv, bi, dpp_d<0xB1>(bv), dpp_i<0xB1>(bi));
  better(bv, bi, dpp_d<0x4E>(bv), dpp_i<0x4E>(bi));
  better(bv, bi, dpp_d<0x141>(bv), dpp_i<0x141>(bi));
  better(bv, bi, dpp_d<0x140>(bv), dpp_i<0x140>(bi));
  // across rows: the better of {own, partner} in either order (a total order)
  double av, cv;
  int ai, ci;
  cross_pair<16>(bv, av, cv);
  cross_pair_i<16>(bi, ai, ci);
  bv = av, bi = ai;
  better(bv, bi, cv, ci);
  cross_pair<32>(bv, av, cv);
  cross_pair_i<32>(bi, ai, ci);
  bv = av, bi = ai;
  better(bv, bi, cv, ci);
}

// ---------------------------------------------------------------------------
// small problems: one workgroup, matrix in registers
// ---------------------------------------------------------------------------
// NOPIV: every problem of the launch factors without pivoting (step i's
// pivot is column i).  Then no candidate is searched and no norm kept but
// the pivot column's own, which its wavefront forms from its registers (in
// the order the pivoted path forms it); the reflector goes through LDS
// buffers alternating by step, so a step needs one barrier.
template <int RW, int CPW, int RPL, bool NOPIV = false>
__global__ __launch_bounds__(RW * 64) void qrcp_reg_kernel(const DevProb* __restrict__ probs,
                                                          const int* __restrict__ list, double rtol,
                                                          Work w) {
  __shared__ double xcol[NOPIV ? 2 : 1][RPL * 64];
  __shared__ double pn_s[2];
  __shared__ double nrm_s[RW * CPW];  // squared norms: compared as they are, the winner's root taken
  __shared__ int step_s[RW * CPW];
  __shared__ double red_v[RW];
  __shared__ int red_i[RW];

  const int q = list[blockIdx.x];
  const DevProb dp = probs[q];
  const IdProblem& P = dp.p;
  const int m = P.m, d = P.d;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  double y[CPW][RPL];
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int j = wave + RW * c;
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int r = lane + 64 * t;
      const double v = (j < m && r < d) ? P.Y[(long long)j * P.ldy + r] : 0.0;
      y[c][t] = v;
      s = fma(v, v, s);
    }
    if constexpr (!NOPIV) s = wave_sum(s);
    if (lane == 0 && j < m) {
      if constexpr (!NOPIV) nrm_s[j] = s;
      step_s[j] = -1;
    }
  }
  __syncthreads();
  const int kmax = dp.kmax;
  double nu0 = 0.0;
  int k = 0;
  if constexpr (NOPIV) {
    for (int i = 0; i < kmax; ++i) {
      const int wp = i % RW, cp = i / RW, b = i & 1;
      if (wave == wp) {  // the pivot column: reflector source and its norm below row i
        double sn = 0.0;
#pragma unroll
        for (int c = 0; c < CPW; ++c)
          if (c == cp) {
#pragma unroll
            for (int t = 0; t < RPL; ++t) {
              const int r = lane + 64 * t;
              xcol[b][r] = y[c][t];
              if (r >= i && r < d) sn = fma(y[c][t], y[c][t], sn);
            }
          }
        sn = wave_sum(sn);
        if (lane == 0) {
          pn_s[b] = sqrt(sn);
          step_s[i] = i;
        }
      }
      __syncthreads();
      const double best = pn_s[b];
      const double x0 = xcol[b][i];
      const bool zero = !(best > 0.0);
      const double alpha = zero ? 0.0 : -copysign(best, x0);
      const double v0 = x0 - alpha;
      const double tau = zero ? 0.0 : -v0 / alpha;
      const double inv_v0 = zero ? 0.0 : 1.0 / v0;
      double uu[RPL];
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int r = lane + 64 * t;
        uu[t] = (r < d && r > i) ? xcol[b][r] * inv_v0 : (r == i ? 1.0 : 0.0);
      }
      if (tid == 0) {
        w.alpha[dp.aoff + i] = alpha;
        w.piv[dp.aoff + i] = i;
      }
      // the columns after the pivot (the earlier ones are finished)
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const int j = wave + RW * c;
        if (j >= m || j <= i) continue;
        double dot = 0.0;
#pragma unroll
        for (int t = 0; t < RPL; ++t) dot = fma(uu[t], y[c][t], dot);
        const double f = tau * wave_sum(dot);
#pragma unroll
        for (int t = 0; t < RPL; ++t) y[c][t] = fma(-f, uu[t], y[c][t]);
      }
      k = i + 1;
      // no closing barrier: the next step writes the other buffer, and the
      // one after it this buffer only once every wavefront has passed the
      // next step's barrier, i.e. finished reading here
    }
  } else {
  for (int i = 0; i < kmax; ++i) {
    double bv = -1.0;
    int bi = INT_MAX;
    for (int j = tid; j < m; j += RW * 64)
      if (step_s[j] < 0) better(bv, bi, nrm_s[j], j);
    wave_argmax(bv, bi);
    if (lane == 0) {
      red_v[wave] = bv;
      red_i[wave] = bi;
    }
    __syncthreads();
    // every thread reduces the RW wavefront results (no second barrier);
    // red_v / red_i are written again only after this step's later barriers
    double sb = red_v[0];
    int sp = red_i[0];
#pragma unroll
    for (int q2 = 1; q2 < RW; ++q2) better(sb, sp, red_v[q2], red_i[q2]);
    const bool nopiv = P.nfac > 0;
    const double best = sqrt(fmax(nopiv ? nrm_s[i] : sb, 0.0));  // -1 (no candidate) stops as 0 would
    const int p = nopiv ? i : sp;
    if (i == 0) nu0 = best;
    if (!nopiv && (best <= 0.0 || best <= rtol * nu0)) break;
    if (!nopiv && P.kfail >= 0 && i > P.kfail && m > d) break;
    const int wp = p % RW, cp = p / RW;
    if (wave == wp) {
#pragma unroll
      for (int c = 0; c < CPW; ++c)
        if (c == cp) {
#pragma unroll
          for (int t = 0; t < RPL; ++t) xcol[0][lane + 64 * t] = y[c][t];
        }
    }
    if (tid == 0) step_s[p] = i;
    __syncthreads();
    const double x0 = xcol[0][i];
    const bool zero = !(best > 0.0);
    const double alpha = zero ? 0.0 : -copysign(best, x0);
    const double v0 = x0 - alpha;
    const double tau = zero ? 0.0 : -v0 / alpha;
    const double inv_v0 = zero ? 0.0 : 1.0 / v0;
    double uu[RPL];
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int r = lane + 64 * t;
      uu[t] = (r < d && r > i) ? xcol[0][r] * inv_v0 : (r == i ? 1.0 : 0.0);
    }
    if (wave == wp && !nopiv) {
#pragma unroll
      for (int c = 0; c < CPW; ++c)
        if (c == cp) {
#pragma unroll
          for (int t = 0; t < RPL; ++t)
            if (lane + 64 * t == i) y[c][t] = alpha;
        }
    }
    if (tid == 0) {
      w.alpha[dp.aoff + i] = alpha;
      w.piv[dp.aoff + i] = p;
    }
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const int j = wave + RW * c;
      if (j >= m || step_s[j] >= 0) continue;
      double dot = 0.0;
#pragma unroll
      for (int t = 0; t < RPL; ++t) dot = fma(uu[t], y[c][t], dot);
      const double f = tau * wave_sum(dot);
      double s = 0.0;
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int r = lane + 64 * t;
        const double v = fma(-f, uu[t], y[c][t]);
        y[c][t] = v;
        if (r > i && r < d) s = fma(v, v, s);
      }
      s = wave_sum(s);
      if (lane == 0) nrm_s[j] = s;
    }
    k = i + 1;
    __syncthreads();
  }
  }
  __syncthreads();  // step_s complete before the write-back
  // write back the R data and the pivot steps
  int* step = w.step + dp.off;
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int j = wave + RW * c;
    if (j >= m) continue;
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int r = lane + 64 * t;
      if (r < d) P.W[(long long)j * P.ldw + r] = y[c][t];
    }
    if (lane == 0) step[j] = step_s[j];
  }
  if (tid == 0) w.k[q] = k;
}

// ---------------------------------------------------------------------------
// small problems, 16 lanes per column: one workgroup of eight wavefronts per
// problem.  Each 16-lane row of a wavefront holds one column (lane l16 of
// the row has rows l16, l16 + 16, ..., R16 per column), so a wavefront holds
// four columns per group and CG groups.  A column's dot products and norms
// are sums over its 16 lanes -- four DPP levels that serve the four columns
// of a group at once -- instead of over 64 lanes per column (the reductions
// were the bulk of the instructions of a step).  Column j of group g is
// 4 (g RW + wave) + row.  Two barriers per step: the pivot candidates come
// from the norms in registers, and the reflector goes through LDS.
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ void row16_sum_n(double (&v)[N]) {
#pragma unroll
  for (int c = 0; c < N; ++c) v[c] += dpp_d<0xB1>(v[c]);  // quad_perm [1,0,3,2]
#pragma unroll
  for (int c = 0; c < N; ++c) v[c] += dpp_d<0x4E>(v[c]);  // quad_perm [2,3,0,1]
#pragma unroll
  for (int c = 0; c < N; ++c) v[c] += dpp_d<0x141>(v[c]);  // row_half_mirror
#pragma unroll
  for (int c = 0; c < N; ++c) v[c] += dpp_d<0x140>(v[c]);  // row_mirror
}

// NOPIV: as for the 64-lane kernel, a launch of factorizations without
// pivoting only: no candidates, the pivot column's norm formed by its row of
// lanes, reflector buffers alternating by step, one barrier per step.
template <int CG, int R16, bool NOPIV = false>
__global__ __launch_bounds__(512) void qrcp_reg16_kernel(const DevProb* __restrict__ probs,
                                                        const int* __restrict__ list, double rtol, Work w) {
  constexpr int RW = 8, NC = 4 * RW * CG;  // wavefronts, columns held
  constexpr int SB = CG < 4 ? CG : 4;      // groups whose sums are taken together
  static_assert(CG % SB == 0, "whole sub-batches");
  __shared__ double xcol[NOPIV ? 2 : 1][R16 * 16];
  __shared__ double pn_s[2];
  __shared__ double nrm_s[NC];
  __shared__ int step_s[NC];
  __shared__ double red_v[RW];
  __shared__ int red_i[RW];

  const int q = list[blockIdx.x];
  const DevProb dp = probs[q];
  const IdProblem& P = dp.p;
  const int m = P.m, d = P.d;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, rq = lane >> 4;
  const bool nopiv = P.nfac > 0;

  // this lane's best candidate of the step to come: the norms are folded in
  // as soon as they are known, not kept per column
  double bv = -1.0;
  int bi = INT_MAX;
  double y[CG][R16];
#pragma unroll
  for (int g0 = 0; g0 < CG; g0 += SB) {
    double s[SB];
#pragma unroll
    for (int gg = 0; gg < SB; ++gg) {
      const int g = g0 + gg, j = 4 * (g * RW + wave) + rq;
      s[gg] = 0.0;
#pragma unroll
      for (int t = 0; t < R16; ++t) {
        const int r = l16 + 16 * t;
        const double v = (j < m && r < d) ? P.Y[(long long)j * P.ldy + r] : 0.0;
        y[g][t] = v;
        s[gg] = fma(v, v, s[gg]);
      }
    }
    if constexpr (!NOPIV) row16_sum_n<SB>(s);
#pragma unroll
    for (int gg = 0; gg < SB; ++gg) {
      const int j = 4 * ((g0 + gg) * RW + wave) + rq;
      if (j < m) {
        if constexpr (!NOPIV) {
          better(bv, bi, s[gg], j);  // squared norms: the winner's root is taken
          if (l16 == 0) nrm_s[j] = s[gg];
        }
        if (l16 == 0) step_s[j] = -1;
      }
    }
  }
  unsigned sel = 0;  // groups whose column (of this lane's row) is a pivot
  const int kmax = dp.kmax;
  double nu0 = 0.0;
  int k = 0;
  if constexpr (NOPIV) {
    for (int i = 0; i < kmax; ++i) {
      const int wp = (i >> 2) % RW, gp = (i >> 2) / RW, rp = i & 3, b = i & 1;
      if (wave == wp && rq == rp) {  // the pivot column's row of lanes
        double sn[1] = {0.0};
#pragma unroll
        for (int g = 0; g < CG; ++g)
          if (g == gp) {
#pragma unroll
            for (int t = 0; t < R16; ++t) {
              const int r = l16 + 16 * t;
              xcol[b][r] = y[g][t];
              if (r >= i && r < d) sn[0] = fma(y[g][t], y[g][t], sn[0]);
            }
          }
        row16_sum_n<1>(sn);
        if (l16 == 0) {
          pn_s[b] = sqrt(sn[0]);
          step_s[i] = i;
        }
      }
      __syncthreads();
      const double best = pn_s[b];
      const double x0 = xcol[b][i];
      const bool zero = !(best > 0.0);
      const double alpha = zero ? 0.0 : -copysign(best, x0);
      const double v0 = x0 - alpha;
      const double tau = zero ? 0.0 : -v0 / alpha;
      const double inv_v0 = zero ? 0.0 : 1.0 / v0;
      double uu[R16];
#pragma unroll
      for (int t = 0; t < R16; ++t) {
        const int r = l16 + 16 * t;
        uu[t] = (r < d && r > i) ? xcol[b][r] * inv_v0 : (r == i ? 1.0 : 0.0);
      }
      if (tid == 0) {
        w.alpha[dp.aoff + i] = alpha;
        w.piv[dp.aoff + i] = i;
      }
      // the columns after the pivot, SB groups' sums at a time
#pragma unroll
      for (int g0 = 0; g0 < CG; g0 += SB) {
        double f[SB];
#pragma unroll
        for (int gg = 0; gg < SB; ++gg) {
          f[gg] = 0.0;
#pragma unroll
          for (int t = 0; t < R16; ++t) f[gg] = fma(uu[t], y[g0 + gg][t], f[gg]);
        }
        row16_sum_n<SB>(f);
#pragma unroll
        for (int gg = 0; gg < SB; ++gg) {
          const int g = g0 + gg, j = 4 * (g * RW + wave) + rq;
          const double fg = (j < m && j > i) ? tau * f[gg] : 0.0;
#pragma unroll
          for (int t = 0; t < R16; ++t) y[g][t] = fma(-fg, uu[t], y[g][t]);
        }
      }
      k = i + 1;
      // no closing barrier: the next step writes the other buffers, and the
      // one after it these only once every wavefront has passed the next
      // step's barrier
    }
  } else {
  for (int i = 0; i < kmax; ++i) {
    // candidates across the four rows of the wavefront, then across wavefronts
    better(bv, bi, __shfl_xor(bv, 16, 64), __shfl_xor(bi, 16, 64));
    better(bv, bi, __shfl_xor(bv, 32, 64), __shfl_xor(bi, 32, 64));
    if (lane == 0) {
      red_v[wave] = bv;
      red_i[wave] = bi;
    }
    __syncthreads();
    double sb = red_v[0];
    int sp = red_i[0];
#pragma unroll
    for (int w2 = 1; w2 < RW; ++w2) better(sb, sp, red_v[w2], red_i[w2]);
    const double best = sqrt(fmax(nopiv ? nrm_s[i] : sb, 0.0));  // -1 (no candidate) stops as 0 would
    const int p = nopiv ? i : sp;
    if (i == 0) nu0 = best;
    if (!nopiv && (best <= 0.0 || best <= rtol * nu0)) break;
    if (!nopiv && P.kfail >= 0 && i > P.kfail && m > d) break;
    // the pivot column's owner: wavefront (p / 4) % RW, group (p / 4) / RW, row p % 4
    const int wp = (p >> 2) % RW, gp = (p >> 2) / RW, rp = p & 3;
    if (wave == wp && rq == rp) {
#pragma unroll
      for (int g = 0; g < CG; ++g)
        if (g == gp) {
#pragma unroll
          for (int t = 0; t < R16; ++t) xcol[0][l16 + 16 * t] = y[g][t];
          sel |= 1u << g;
        }
      if (l16 == 0) step_s[p] = i;
    }
    __syncthreads();
    const double x0 = xcol[0][i];
    const bool zero = !(best > 0.0);
    const double alpha = zero ? 0.0 : -copysign(best, x0);
    const double v0 = x0 - alpha;
    const double tau = zero ? 0.0 : -v0 / alpha;
    const double inv_v0 = zero ? 0.0 : 1.0 / v0;
    double uu[R16];
#pragma unroll
    for (int t = 0; t < R16; ++t) {
      const int r = l16 + 16 * t;
      uu[t] = (r < d && r > i) ? xcol[0][r] * inv_v0 : (r == i ? 1.0 : 0.0);
    }
    if (tid == 0) {
      w.alpha[dp.aoff + i] = alpha;
      w.piv[dp.aoff + i] = p;
    }
    // H applied to the live columns, SB groups' sums at a time; their new
    // norms become the next step's candidates
    bv = -1.0;
    bi = INT_MAX;
#pragma unroll
    for (int g0 = 0; g0 < CG; g0 += SB) {
      double f[SB];
#pragma unroll
      for (int gg = 0; gg < SB; ++gg) {
        f[gg] = 0.0;
#pragma unroll
        for (int t = 0; t < R16; ++t) f[gg] = fma(uu[t], y[g0 + gg][t], f[gg]);
      }
      row16_sum_n<SB>(f);
      double s2[SB];
#pragma unroll
      for (int gg = 0; gg < SB; ++gg) {
        const int g = g0 + gg, j = 4 * (g * RW + wave) + rq;
        const bool live = j < m && !((sel >> g) & 1u);
        const double fg = live ? tau * f[gg] : 0.0;
        s2[gg] = 0.0;
#pragma unroll
        for (int t = 0; t < R16; ++t) {
          const int r = l16 + 16 * t;
          const double v = fma(-fg, uu[t], y[g][t]);
          y[g][t] = v;
          if (r > i && r < d) s2[gg] = fma(v, v, s2[gg]);
        }
      }
      row16_sum_n<SB>(s2);
#pragma unroll
      for (int gg = 0; gg < SB; ++gg) {
        const int g = g0 + gg, j = 4 * (g * RW + wave) + rq;
        if (j < m && !((sel >> g) & 1u)) {
          better(bv, bi, s2[gg], j);
          if (l16 == 0) nrm_s[j] = s2[gg];
        }
      }
    }
    k = i + 1;
    // no closing barrier: xcol, red_v and nrm_s are written next only after
    // the next step's first barrier, which every thread reaches only once
    // done with this step
  }
  }
  // write back the R data and the pivot steps; a pivot's own row (its
  // step) gets R_ii = alpha, which the step loop leaves out of the registers
  __syncthreads();
  int* step = w.step + dp.off;
#pragma unroll
  for (int g = 0; g < CG; ++g) {
    const int j = 4 * (g * RW + wave) + rq;
    if (j >= m) continue;
    const int sj = step_s[j];
    const double aj = (!nopiv && sj >= 0 && sj < k) ? w.alpha[dp.aoff + sj] : 0.0;
#pragma unroll
    for (int t = 0; t < R16; ++t) {
      const int r = l16 + 16 * t;
      if (r < d) P.W[(long long)j * P.ldw + r] = (!nopiv && sj >= 0 && sj < k && r == sj) ? aj : y[g][t];
    }
    if (l16 == 0) step[j] = sj;
  }
  if (tid == 0) w.k[q] = k;
}

// ---------------------------------------------------------------------------
// large problems: one launch per pivot step
//
// Workgroup g of a problem owns columns g*SW .. g*SW+SW-1, one per
// wavefront.  After its update every workgroup publishes its best remaining
// column (norm, index) for the next step (double-buffered by step parity);
// the next step's workgroups all reduce the same candidates the same way.
// The workgroup stages the reflector in LDS; each wavefront keeps its own
// column (rows i..d-1, T per lane) in registers, so every element is read
// once and written once per step.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wg_candidate(double v, int j, double* rv, int* ri, double* cv,
                                             int* ci) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    rv[wave] = v;
    ri[wave] = j;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double bv = rv[0];
    int bi = ri[0];
    for (int t = 1; t < SW; ++t) better(bv, bi, rv[t], ri[t]);
    *cv = bv;
    *ci = bi;
  }
}

__global__ __launch_bounds__(ST) void id_init_kernel(const DevProb* __restrict__ probs,
                                                    const int* __restrict__ wg_prob, long long tg,
                                                    Work w) {
  __shared__ double rv[SW];
  __shared__ int ri[SW];
  const int q = wg_prob[blockIdx.x];
  const DevProb dp = probs[q];
  const IdProblem& P = dp.p;
  const int g = blockIdx.x - dp.g0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = g * SW + wave;
  double nv = -1.0;
  if (j < P.m) {
    const double* src = P.Y + (long long)j * P.ldy;
    double* dst = P.W + (long long)j * P.ldw;
    const bool copy = src != dst;
    double s = 0.0;
    for (int r = lane; r < P.d; r += 64) {
      const double v = src[r];
      if (copy) dst[r] = v;
      s = fma(v, v, s);
    }
    nv = sqrt(wave_sum(s));
    if (lane == 0) {
      w.nrm[dp.off + j] = nv;
      w.step[dp.off + j] = -1;
    }
  }
  wg_candidate(nv, j < P.m ? j : INT_MAX, rv, ri, w.cand_v + blockIdx.x, w.cand_i + blockIdx.x);
  if (g == 0 && threadIdx.x == 0) {
    w.done[q] = 0;
    w.k[q] = 0;
  }
}

template <int T>
__global__ __launch_bounds__(ST) void id_step_kernel(const DevProb* __restrict__ probs,
                                                    const int* __restrict__ wg_prob, int i,
                                                    double rtol, long long tm, long long tg,
                                                    Work w) {
  extern __shared__ double u[];  // T > 0: rows i..d-1 of the reflector
  __shared__ double rv[SW];
  __shared__ int ri[SW];
  __shared__ double s_best;
  __shared__ int s_p;

  const int q = wg_prob[blockIdx.x];
  if (w.done[q]) return;
  const DevProb dp = probs[q];
  const IdProblem& P = dp.p;
  const int m = P.m, d = P.d;
  const int g = blockIdx.x - dp.g0;
  const bool leader = (g == 0 && threadIdx.x == 0);
  if (i >= dp.kmax) {
    if (leader) {
      w.done[q] = 1;
      atomicAdd(w.ndone, 1);
    }
    return;
  }
  const double* __restrict__ nrm = w.nrm + (i & 1) * tm + dp.off;
  double* __restrict__ nrm_next = w.nrm + ((i + 1) & 1) * tm + dp.off;
  int* __restrict__ step = w.step + dp.off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool nopiv = P.nfac > 0;
  double best;
  int p;
  if (nopiv) {  // columns in order
    best = nrm[i];
    p = i;
  } else {  // all workgroups of the problem reduce the same candidates the same way
    const double* cv = w.cand_v + (i & 1) * tg + dp.g0;
    const int* ci = w.cand_i + (i & 1) * tg + dp.g0;
    double bv = -1.0;
    int bi = INT_MAX;
    for (int t = tid; t < dp.G; t += ST) better(bv, bi, cv[t], ci[t]);
    wave_argmax(bv, bi);
    if (lane == 0) {
      rv[wave] = bv;
      ri[wave] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      double v = rv[0];
      int ix = ri[0];
      for (int t = 1; t < SW; ++t) better(v, ix, rv[t], ri[t]);
      s_best = v;
      s_p = ix;
    }
    __syncthreads();
    best = s_best;
    p = s_p;
  }
  const double nu0 = (i == 0) ? best : w.nu0[q];
  if (i == 0 && leader) w.nu0[q] = best;
  const bool stop =
      !nopiv && ((best <= 0.0 || best <= rtol * nu0) || (P.kfail >= 0 && i > P.kfail && m > d));
  if (stop) {
    if (leader) {
      w.done[q] = 1;
      atomicAdd(w.ndone, 1);
    }
    return;
  }
  const double* __restrict__ wp = P.W + (long long)p * P.ldw;
  const double x0 = wp[i];
  const bool zero = !(best > 0.0);
  const double alpha = zero ? 0.0 : -copysign(best, x0);
  const double v0 = x0 - alpha;
  const double tau = zero ? 0.0 : -v0 / alpha;
  const double inv_v0 = zero ? 0.0 : 1.0 / v0;
  if (leader) {
    w.alpha[dp.aoff + i] = alpha;
    w.piv[dp.aoff + i] = p;
    step[p] = i;
    w.k[q] = i + 1;
  }
  // the reflector u = (1, W[p][i+1..d-1] / v0), staged once per workgroup
  if (T > 0) {
    for (int r = i + tid; r < d; r += ST) u[r - i] = (r == i) ? 1.0 : wp[r] * inv_v0;
    __syncthreads();
  }
  const int j = g * SW + wave;
  bool act = j < m && j != p;
  if (act) {
    const int sj = step[j];
    act = !(sj >= 0 && sj < i);
  }
  double nv = -1.0;
  if (act) {
    double* __restrict__ wj = P.W + (long long)j * P.ldw;
    double s = 0.0;
    if (T > 0) {
      double y[T > 0 ? T : 1];
      double dot = 0.0;
      // lane's rows i + lane + 64 t, addressed from one base pointer
      double* col = wj + i + lane;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const int r = i + lane + 64 * t;
        y[t] = (r < d) ? col[64 * t] : 0.0;
      }
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const int r = i + lane + 64 * t;
        if (r < d) dot = fma(u[r - i], y[t], dot);
      }
      const double f = tau * wave_sum(dot);
      // the stores form their addresses afresh instead of keeping the
      // loads' T addresses live: 2T registers per lane, not 4T
      asm volatile("" : "+v"(col) : : "memory");
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const int r = i + lane + 64 * t;
        if (r < d) {
          const double nvv = fma(-f, u[r - i], y[t]);
          col[64 * t] = nvv;
          if (r > i) s = fma(nvv, nvv, s);
        }
      }
    } else {
      double dot = 0.0;
      for (int r = i + lane; r < d; r += 64) dot = fma(r == i ? 1.0 : wp[r] * inv_v0, wj[r], dot);
      const double f = tau * wave_sum(dot);
      for (int r = i + lane; r < d; r += 64) {
        const double v = fma(-f, r == i ? 1.0 : wp[r] * inv_v0, wj[r]);
        wj[r] = v;
        if (r > i) s = fma(v, v, s);
      }
    }
    nv = sqrt(wave_sum(s));
    if (lane == 0) nrm_next[j] = nv;
  }
  if (!nopiv) {
    const long long slot = ((i + 1) & 1) * tg + blockIdx.x;
    wg_candidate(act ? nv : -1.0, act ? j : INT_MAX, rv, ri, w.cand_v + slot, w.cand_i + slot);
  }
}

// ---------------------------------------------------------------------------
// large problems, persistent: one launch runs every pivot step.
//
// Workgroup g of a problem owns columns g*PW*C .. (g+1)*PW*C-1, C per
// wavefront, and keeps them in registers for the whole factorization (lane l
// holds rows l, l+64, ..., T per column; rows d..64T-1 are zero and stay
// zero, so no row needs a bounds test inside the step loop).  Two
// wavefronts share each SIMD and every value lives in architectural
// registers.  After each step the workgroup publishes its best remaining
// column: norm and index go to a 16-byte record of its own for that step,
// the values to a column slot of its own (a ring of 2, 4 or 8 slots by step).
// Every workgroup of the problem waits for the G records of the step,
// reduces the same candidates the same way, reads the winner's published
// values as the reflector and updates its own columns.  Per step, global
// memory carries only the candidates and one column per workgroup.
//
// Every word that crosses workgroups carries the step it belongs to, so a
// reader can tell a current word from a stale one by looking at the word
// alone; no ordering between different words is needed, hence no fences
// and no wait for stores to complete.  All such accesses are relaxed
// agent-scope atomics on aligned 64-bit words in memory zeroed before the
// launch (single-copy atomic, and coherent per location), and no
// read-modify-write atomics are used.
// - A record is two words written once per launch: the norm with its sign
//   bit flipped (never zero: norms are +0 or more, or -1 for no candidate)
//   and (step + 1) << 32 | index.  A reader takes a record once both words
//   are non-zero and the step matches.
// - A column value is written as two words, (step + 1) << 32 | low 32 bits
//   and (step + 1) << 32 | high 32 bits, so a slot still holding an earlier
//   step's column shows a different tag; a reader loads every row again
//   until both tags match the step.
// Every wait is bounded: a workgroup that waits too long raises the error
// flag and leaves, and so does every workgroup that sees the flag; the
// factorization is then reported as failed and nothing is written back.
// ---------------------------------------------------------------------------
constexpr int PW = 8;        // wavefronts per persistent workgroup (two per SIMD)
constexpr int PT = PW * 64;  // threads per persistent workgroup
constexpr int kSpinLimit = 1 << 22;
constexpr unsigned long long kSignBit = 1ull << 63;

template <typename V>
__device__ __forceinline__ void st_dev(V* p, V v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename V>
__device__ __forceinline__ V ld_dev(const V* p) {
  return __hip_atomic_load(const_cast<V*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The step loop is written for the register allocator: slices are skipped
// in groups of PG (a handful of uniform branches per step, the finished
// rows of a processed group see u = 0), at most PG reflector values are
// read from LDS ahead of their use, and the published column's addresses are
// formed inside the loop.  Each wavefront keeps only its best remaining
// column's norm, not one per column.
constexpr int PG = 4;

template <int T, int C>
__global__ __launch_bounds__(PT) void qrcp_persist_kernel(const DevProb* __restrict__ probs,
                                                         const int* __restrict__ wg_prob,
                                                         double rtol, Work w) {
  static_assert(T % PG == 0, "slices are skipped PG at a time");
  constexpr int SU = (T * 64 + PT - 1) / PT;  // reflector rows staged per thread
  __shared__ double u[T * 64];
  __shared__ double rv[PW];
  __shared__ int ri[PW];
  __shared__ double gv_s[PW];
  __shared__ int gi_s[PW];
  __shared__ int s_ok;

  const int q = wg_prob[blockIdx.x];
  const DevProb dp = probs[q];
  const int m = dp.p.m, d = dp.p.d;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool leader = ((int)blockIdx.x == dp.g0 && tid == 0);
  // no pivoting (Householder QR of the first nfac columns, the others only
  // transformed): step i's pivot is column i, the only candidate published.
  // Every workgroup still publishes a record every step.  With pivoting, or
  // with two column slots per workgroup, every workgroup waits for all the
  // records of every step: that exchange keeps the workgroups within one
  // step of each other, which the double-buffered slots need (an owner of
  // consecutive columns would otherwise run ahead and overwrite a slot that
  // a slower workgroup has yet to read).  A launch of problems without
  // pivoting may have R = 4 or 8 slots per workgroup (slot i mod R for step
  // i); its workgroups then wait for all records only at steps that are
  // multiples of R / 2, and at the other steps for the record of column i's
  // owner alone.  A slot is written again R steps later, by a workgroup
  // that has by then passed such a full exchange at a step between the
  // two, so every workgroup has finished reading it.
  const bool nopiv = dp.p.nfac > 0;
  constexpr int CPG = PW * C;  // columns per workgroup
  const int jb = (blockIdx.x - dp.g0) * CPG + wave * C;
  int* __restrict__ step = w.step + dp.off;
  const long long ldcb = w.ldcb;
  const long long nslot = gridDim.x;

  double y[C][T];
  double bv = -1.0;  // this wavefront's best remaining column: norm, index
  int bi = INT_MAX;
  unsigned sel = 0;  // columns of this wavefront already chosen as pivots
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int j = jb + c;
    // a lane's base address and constant strides: no per-row offsets to keep
    const double* __restrict__ src = dp.p.Y + (long long)min(j, m - 1) * dp.p.ldy + lane;
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const double v = (j < m && lane < d - 64 * t) ? src[64 * t] : 0.0;
      y[c][t] = v;
      s = fma(v, v, s);
    }
    if (nopiv ? j == 0 : j < m) better(bv, bi, wave_sum(s), j);  // squared norms throughout
    if (j < m && lane == 0) step[j] = -1;
    asm volatile("" ::: "memory");  // one column's loads in flight at a time
  }
  if (tid == 0) s_ok = 1;

  // publish this workgroup's best column for step i: norm and index in a
  // record, and the row slices from i / 64 on (the reader masks rows below
  // i).  The owning wavefront writes the record and then the column (the
  // first wavefront writes the record when the workgroup has no candidate
  // left): the record does not queue behind the column's stores, and the
  // readers need the column only after they have reduced all records (7.8
  // against 8.7 us per step on two 1664 x 2686 problems).  Writing only the
  // winner's column, after the exchange, took longer (9.3 us per step): the
  // records arrived 1 us sooner, the column 2 us later.
  auto publish = [&](int i) __attribute__((always_inline)) {  // y must stay in registers
    if (lane == 0) {
      rv[wave] = bv;
      ri[wave] = bi;
    }
    __syncthreads();
    double v = rv[0];
    int ix = ri[0];
#pragma unroll
    for (int t = 1; t < PW; ++t) better(v, ix, rv[t], ri[t]);
    const bool own = ix >= jb && ix < jb + C;  // uniform within a wavefront
    if (lane == 0 && (own || (ix == INT_MAX && wave == 0))) {
      unsigned long long* r = w.rec + 2 * ((long long)blockIdx.x * w.rstride + i);
      st_dev(r, (unsigned long long)__double_as_longlong(v) ^ kSignBit);
      st_dev(r + 1, ((unsigned long long)(i + 1) << 32) | (unsigned)ix);
    }
    if (own) {
      // uniform bases and one 32-bit lane offset, formed here (not hoisted
      // out of the step loop as T live addresses)
      const long long slot = (long long)(i & w.rmask) * nslot + blockIdx.x;
      char* blo = reinterpret_cast<char*>(w.cbuf + slot * 2 * ldcb);
      char* bhi = reinterpret_cast<char*>(w.cbuf + slot * 2 * ldcb + ldcb);
      unsigned vo = (unsigned)lane * 8u;
      asm volatile("" : "+v"(vo));
      const unsigned long long tag = (unsigned long long)(i + 1) << 32;
      const int ti = i >> 6;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        if (ix != jb + c) continue;
#pragma unroll
        for (int g = 0; g < T / PG; ++g) {
          if (PG * g + PG <= ti) continue;
#pragma unroll
          for (int tt = 0; tt < PG; ++tt) {
            const unsigned off = vo + 512u * (unsigned)(PG * g + tt);
            const unsigned long long b = (unsigned long long)__double_as_longlong(y[c][PG * g + tt]);
            st_dev(reinterpret_cast<unsigned long long*>(blo + off), tag | (b & 0xffffffffull));
            st_dev(reinterpret_cast<unsigned long long*>(bhi + off), tag | (b >> 32));
          }
        }
      }
    }
  };

  // wait for the problem's G candidates of step i; false on a timeout
  auto gather = [&](int i, double& best, int& p) __attribute__((always_inline)) -> bool {
    // workgroup-major records: the G records of one step lie in G different
    // cache lines (and memory channels), not packed into a few lines that
    // every poller of the problem would hit (2.5 us from the last record to
    // its readers with packed records, against a 0.5 us one-way latency)
    const unsigned long long* recs = w.rec + 2 * ((long long)dp.g0 * w.rstride + i);
    const long long rs2 = 2 * w.rstride;
    const unsigned long long want = (unsigned long long)(i + 1);
    double gv = -1.0;
    int gi = INT_MAX;
    bool ok = true;
    if (w.give_up) {  // host switch: leave at once, as after a timeout
      if (tid == 0) st_dev(w.err, 1);
      ok = false;
    }
    // without pivoting only the owner of column i has a candidate (every
    // other record says none), so between full exchanges one thread waits
    // for the owner's record alone; the reduction below gives the same pair
    const bool full = !nopiv || (i & w.xmask) == 0;
    const int t0 = full ? tid : (tid == 0 ? i / CPG : dp.G);
    const int tstride = full ? PT : dp.G;
    for (int t = t0; t < dp.G && ok; t += tstride) {
      int spins = 0;
      unsigned long long a, b;
      const unsigned long long* rt = recs + (long long)t * rs2;
      while (true) {
        a = ld_dev(rt);
        b = ld_dev(rt + 1);
        if (a != 0 && (b >> 32) == want) break;
        if ((++spins & 63) == 0) {
          if (ld_dev(w.err)) {
            ok = false;
            break;
          }
          if (spins >= kSpinLimit) {
            st_dev(w.err, 1);
            ok = false;
            break;
          }
        }
        __builtin_amdgcn_s_sleep(1);
      }
      if (ok) better(gv, gi, __longlong_as_double((long long)(a ^ kSignBit)), (int)(unsigned)b);
    }
    if (!ok) s_ok = 0;
    wave_argmax_pl(gv, gi);
    // gv_s / gi_s, not rv / ri: publish has no closing barrier, so another
    // wavefront may still be reading rv / ri
    if (lane == 0) {
      gv_s[wave] = gv;
      gi_s[wave] = gi;
    }
    __syncthreads();
    // every thread reduces the PW wavefront results itself (no second barrier)
    double v = gv_s[0];
    int ix = gi_s[0];
#pragma unroll
    for (int t = 1; t < PW; ++t) better(v, ix, gv_s[t], gi_s[t]);
    best = sqrt(fmax(v, 0.0));  // squared norms in the records: the winner's root only
    p = ix;
    return s_ok != 0;
  };

  publish(0);
  double nu0 = 0.0;
  int k = 0;
  for (int i = 0; i < dp.kmax; ++i) {
    double best;
    int p;
    if (!gather(i, best, p)) return;
    // uniform: a scalar base address for the winner's slot below
    p = __builtin_amdgcn_readfirstlane(p);
    if (i == 0) nu0 = best;
    if (!nopiv && (best <= 0.0 || best <= rtol * nu0)) break;
    if (!nopiv && dp.p.kfail >= 0 && i > dp.p.kfail && m > d) break;
    const int gp = p / CPG;  // the workgroup that published column p
    const unsigned long long* xp = w.cbuf + ((long long)(i & w.rmask) * nslot + dp.g0 + gp) * 2 * ldcb;
    // the winner's rows i..d-1 into LDS (zero elsewhere), loads in flight
    // together; a row whose words do not both carry this step's tag yet is
    // loaded again (bounded).  LDS receives the Householder vector
    // v = x - alpha e_i unscaled: row i holds v0 = x0 - alpha, formed by the
    // thread that loads it (alpha = -sign(x0) ||x||, so sign(v0) = sign(x0)
    // and every thread recovers alpha from v0).
    {
      const unsigned want = (unsigned)(i + 1);
      unsigned long long wl[SU], wh[SU];
      const char* xb = reinterpret_cast<const char*>(xp);
      const char* xc = reinterpret_cast<const char*>(xp + ldcb);
      // 32-bit byte offsets from the uniform bases: a scalar base plus one
      // offset register per load, not a 64-bit address per load
      auto at = [](const char* base, unsigned row) {
        return reinterpret_cast<const unsigned long long*>(base + row * 8u);
      };
#pragma unroll
      for (int t = 0; t < SU; ++t) {
        const int r = tid + PT * t;
        const unsigned rr = (r >= i && r < d) ? (unsigned)r : (unsigned)i;
        wl[t] = ld_dev(at(xb, rr));
        wh[t] = ld_dev(at(xc, rr));
      }
#pragma unroll
      for (int t = 0; t < SU; ++t) {
        const int r = tid + PT * t;
        if (r >= T * 64) break;
        const bool in = r >= i && r < d;
        int spins = 0;
        while (in && ((unsigned)(wl[t] >> 32) != want || (unsigned)(wh[t] >> 32) != want)) {
          if ((++spins & 63) == 0 && (ld_dev(w.err) || spins >= kSpinLimit)) {
            st_dev(w.err, 1);
            s_ok = 0;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          wl[t] = ld_dev(at(xb, (unsigned)r));
          wh[t] = ld_dev(at(xc, (unsigned)r));
        }
        const double x = __longlong_as_double((long long)((wh[t] << 32) | (wl[t] & 0xffffffffull)));
        u[r] = in ? (r == i ? x + copysign(best, x) : x) : 0.0;
      }
    }
    __syncthreads();
    if (!s_ok) return;  // a wait timed out (flag raised for the whole problem)
    // u is only read from here until the next step's loads, which come after
    // the barriers of publish and gather
    const double v0 = u[i];
    const double alpha = -copysign(best, v0);
    // H = I - beta v v^T (a zero column, only without pivoting: H = I)
    const double beta = best > 0.0 ? -1.0 / (alpha * v0) : 0.0;
    if (p >= jb && p < jb + C) {
      sel |= 1u << (p - jb);
      // the owner marks its column: the same wavefront wrote its -1, and
      // plain stores from different workgroups may sit in different caches
      if (lane == 0) step[p] = i;
    }
    if (leader) {
      w.alpha[dp.aoff + i] = alpha;
      w.piv[dp.aoff + i] = p;
    }
    // rows below i are finished: groups of slices below i/64 are skipped,
    // and u is zero on the finished rows of the groups that run.  The C
    // columns go through each phase together, so their dependency chains
    // and reductions overlap.
    const int ti = i >> 6;
    double f[C];
#pragma unroll
    for (int c = 0; c < C; ++c) f[c] = 0.0;
#pragma unroll
    for (int g = 0; g < T / PG; ++g) {
      if (PG * g + PG <= ti) continue;
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int tt = 0; tt < PG; ++tt) {
        const int t = PG * g + tt;
        const double ut = u[lane + 64 * t];
#pragma unroll
        for (int c = 0; c < C; ++c) f[c] = fma(ut, y[c][t], f[c]);
      }
    }
    wave_sum_n_pl<C>(f);
    asm volatile("" ::: "memory");  // u is read again below rather than kept in registers
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const bool live = !((sel >> c) & 1u) && jb + c < m;  // pivots stay as they are
      f[c] = live ? beta * f[c] : 0.0;
    }
    // norms of the rows below i: slice i/64 counts the lanes past i only
    double s2[C];
#pragma unroll
    for (int c = 0; c < C; ++c) s2[c] = 0.0;
    const double keep = lane > (i & 63) ? 1.0 : 0.0;
#pragma unroll
    for (int g = 0; g < T / PG; ++g) {
      if (PG * g + PG <= ti) continue;
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int tt = 0; tt < PG; ++tt) {
        const int t = PG * g + tt;
        const double ut = u[lane + 64 * t];
        const double wt = t > ti ? 1.0 : (t == ti ? keep : 0.0);
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const double v = fma(-f[c], ut, y[c][t]);
          y[c][t] = v;
          s2[c] = fma(v * wt, v, s2[c]);
        }
      }
    }
    wave_sum_n_pl<C>(s2);
    bv = -1.0;
    bi = INT_MAX;
#pragma unroll
    for (int c = 0; c < C; ++c)
      if (nopiv ? jb + c == i + 1 : (!((sel >> c) & 1u) && jb + c < m)) better(bv, bi, s2[c], jb + c);
    k = i + 1;
    if (i + 1 < dp.kmax) publish(i + 1);
  }
  if (leader) w.k[q] = k;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int j = jb + c;
    if (j >= m) continue;
    double* __restrict__ out = dp.p.W + (long long)j * dp.p.ldw + lane;
#pragma unroll
    for (int t = 0; t < T; ++t)
      if (lane < d - 64 * t) out[64 * t] = y[c][t];
    asm volatile("" ::: "memory");
  }
}

// ---------------------------------------------------------------------------
// finishing: permutation, diagonal of R1, blocked E = (R1^{-1} R2)^T
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void id_perm_kernel(const DevProb* __restrict__ probs,
                                                    const int* __restrict__ sel, Work w) {
  __shared__ int cnt[NT];
  const int q = sel[blockIdx.x];
  const DevProb dp = probs[q];
  const IdProblem& P = dp.p;
  const int m = P.m, k = w.k[q];
  const int* step = w.step + dp.off;
  const int tid = threadIdx.x;
  for (int a = tid; a < k; a += NT) {
    const int j = w.piv[dp.aoff + a];
    P.perm[a] = j;
    P.W[(long long)j * P.ldw + a] = w.alpha[dp.aoff + a];
  }
  const int per = (m + NT - 1) / NT;
  const int j0 = tid * per, j1 = min(m, j0 + per);
  int c = 0;
  for (int j = j0; j < j1; ++j) c += (step[j] < 0 || step[j] >= k) ? 1 : 0;
  cnt[tid] = c;
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int t = 0; t < NT; ++t) {
      const int v = cnt[t];
      cnt[t] = acc;
      acc += v;
    }
  }
  __syncthreads();
  int pos = k + cnt[tid];
  for (int j = j0; j < j1; ++j)
    if (step[j] < 0 || step[j] >= k) P.perm[pos++] = j;
}

// Diagonal block of the solve E * Rt = R2^T with Rt = R1^T lower
// triangular: for every unselected column c (one thread each),
// x[a] = (y[a] - sum_{b > a} x[b] Rt[b][a]) / Rt[a][a] on [b0, b1).
struct DiagDesc {
  const double* W;
  long long ldw;
  const int* perm;
  double* E;
  int k, nrest, b0, b1;
  long long wg0;
};

// NB: 64, or 32 / 16 when every block of the launch has at most that many
// rows (low ranks): the padded steps add signed zeros only, so the result is
// the same with fewer steps and registers.
template <int NB>
__global__ __launch_bounds__(NT) void trsm_diag_kernel(const DiagDesc* __restrict__ descs, int nd) {
  __shared__ double Rt[NB][NB + 1];
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].wg0 <= (long long)blockIdx.x) lo = mid;
    else hi = mid - 1;
  }
  const DiagDesc g = descs[lo];
  const int nb = g.b1 - g.b0;
  // padded to NB x NB with the identity: the padded entries solve to zero
  // and the unrolled loops below need no test against nb
  for (int e = threadIdx.x; e < NB * NB; e += NT) {
    const int bb = e / NB, aa = e % NB;
    Rt[bb][aa] = (bb < nb && aa <= bb)
                     ? g.W[(long long)g.perm[g.b0 + bb] * g.ldw + g.b0 + aa]
                     : (aa == bb ? 1.0 : 0.0);
  }
  __syncthreads();
  const int c = (int)(blockIdx.x - g.wg0) * NT + threadIdx.x;
  if (c >= g.nrest) return;
  double* x = g.E + (long long)c * g.k + g.b0;
  double xv[NB];
#pragma unroll
  for (int a = 0; a < NB; ++a) {  // entries past nb read entry 0 and are zeroed
    const double v = x[a < nb ? a : 0];
    xv[a] = a < nb ? v : 0.0;
  }
  // column by column, from the last: once x[b] is final, the updates of the
  // entries above it are independent of each other
#pragma unroll
  for (int b = NB - 1; b >= 0; --b) {
    xv[b] = xv[b] / Rt[b][b];
#pragma unroll
    for (int a = 0; a < b; ++a) xv[a] = fma(-xv[b], Rt[b][a], xv[a]);
  }
#pragma unroll
  for (int a = 0; a < NB; ++a)
    if (a < nb) x[a] = xv[a];
}

}  // namespace

size_t id_workspace_bytes(const IdProblem* probs, int nprob) {
  long long tm = 0, tk = 0, tw = 0, tg = 0, dm = 1, km = 1;
  for (int q = 0; q < nprob; ++q) {
    tg += (probs[q].m + SW - 1) / SW;
    tm += probs[q].m;
    tk += kmax_of(probs[q]);
    km = std::max<long long>(km, kmax_of(probs[q]));
    dm = std::max<long long>(dm, probs[q].d);
    if (!probs[q].W) tw += (long long)probs[q].m * probs[q].d;
  }
  const long long ns = std::min(tg, kCandSlots);
  return al(2 * tm * 8) + al(tm * 4) + al(tk * 8) + al(tk * 4) + 3 * al((size_t)nprob * 8) +
         al(4) + al(2 * tg * 8) + al(2 * tg * 4) + al(2 * ns * 2 * ldcb_of(dm) * 8) + al(2 * ns * km * 8) +
         al(4) + al(tw * 8) + al(inplace_nopiv_doubles(probs, nprob) * 8) + 4096;
}

// Register-resident classes (wavefronts, columns per wavefront, rows per
// lane) chosen so that no instance spills: -1 = use the step kernels.
constexpr int kSmallClasses = 10;
static int small_class(const IdProblem& p) {
  const int m = p.m, d = p.d;
  if (m > 256 || d > 192 || m == 0 || d == 0) return -1;
  if (d <= 64) return m <= 32 ? 0 : m <= 64 ? 1 : m <= 128 ? 2 : 3;
  if (d <= 128) return m <= 64 ? 4 : m <= 128 ? 5 : 6;
  return m <= 64 ? 7 : m <= 128 ? 8 : 9;
}

// Persistent-path variants: T rows per lane (d <= 64 T), C columns per
// wavefront, sized so that the columns fit in the register file.
struct PVariant {
  int T, C;
  const void* fn;
};
static const PVariant kPVariants[] = {
    {8, 8, reinterpret_cast<const void*>(&qrcp_persist_kernel<8, 8>)},
    {12, 7, reinterpret_cast<const void*>(&qrcp_persist_kernel<12, 7>)},
    {16, 6, reinterpret_cast<const void*>(&qrcp_persist_kernel<16, 6>)},
    {24, 4, reinterpret_cast<const void*>(&qrcp_persist_kernel<24, 4>)},
    {32, 3, reinterpret_cast<const void*>(&qrcp_persist_kernel<32, 3>)},
    {36, 3, reinterpret_cast<const void*>(&qrcp_persist_kernel<36, 3>)},
    {40, 2, reinterpret_cast<const void*>(&qrcp_persist_kernel<40, 2>)},
};

// cost model constants (measured on gfx950): time per pivot step of a
// persistent launch, a base plus a term that grows with the workgroups of its
// widest problem (each one publishes a candidate every step: 7.5 us at 4,
// 10.7 us at 167); the floor of one step-path launch, and the rate at which
// the step path moves the active rows
constexpr double kPersistStepUs = 7.3;
constexpr double kPersistStepUsPerWg = 0.02;
constexpr double kStepFloorUs = 25.0;
constexpr double kStepBytesPerS = 3.0e12;

static int resident_workgroups(const void* fn) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, PT, 0) != hipSuccess) return 0;
  return per * cus;
}

// Runs the pivoted problems of `large` whose columns fit in registers as
// persistent launches (problems grouped while their workgroups fit on the
// device at once: the grid never exceeds the resident capacity); the others
// are returned in `rest`.
// A problem fails the rule: rank above its kfail and below its row count.
static bool fails_rule(const IdProblem& p, int k) { return p.kfail >= 0 && k > p.kfail && k < p.m; }

static hipError_t run_persistent(std::vector<DevProb>& h, const std::vector<int>& large, double rtol,
                                 const Work& w, Staging& st, hipStream_t s, std::vector<int>& rest,
                                 std::vector<char>& skipped, int& npersist, int& nlaunch) {
  int dmax = 0;
  std::vector<int> cand, second;
  // problems factored in place without pivoting write to W2 (a rerun after
  // a timed-out wait needs the input untouched) and are copied back after
  std::vector<long long> off2(h.size(), -1);
  std::vector<double*> w_orig(h.size(), nullptr);
  std::vector<long long> ld_orig(h.size(), 0);
  {
    long long o = 0;
    for (size_t q = 0; q < h.size(); ++q)
      if (is_inplace_nopiv(h[q].p)) {
        off2[q] = o;
        o += (long long)h[q].p.m * h[q].p.d;
      }
  }
  for (int q : large) {
    const IdProblem& p = h[q].p;
    if (h[q].kmax == 0 || p.d > 64 * 40) rest.push_back(q);
    else {
      // the first side of each node ahead of every second side: when the
      // batch needs several launches, a node whose first side fails skips
      // the launch of its second side
      if (p.partner >= 0 && p.partner < q) second.push_back(q);
      else cand.push_back(q);
      dmax = std::max(dmax, p.d);
    }
  }
  cand.insert(cand.end(), second.begin(), second.end());
  if (cand.empty()) return hipSuccess;
  // HSS_QRCP_PATH = step | persistent forces a path; otherwise a cost model
  // picks one for the whole batch
  const char* env = std::getenv("HSS_QRCP_PATH");
  const bool force_step = env && std::strcmp(env, "step") == 0;
  const bool force_pers = env && std::strcmp(env, "persistent") == 0;
  if (force_step) {
    rest.insert(rest.end(), cand.begin(), cand.end());
    return hipSuccess;
  }
  int v = 0;
  while (kPVariants[v].T * 64 < dmax) ++v;
  const PVariant& pv = kPVariants[v];
  const int cpg = PW * pv.C;
  int maxwg = (int)std::min<long long>(resident_workgroups(pv.fn), w.nslots);
  if (const char* cap = std::getenv("HSS_QRCP_PERSIST_WG")) {  // tests: fewer workgroups per launch
    const int c = std::atoi(cap);
    if (c > 0) maxwg = std::min(maxwg, c);
  }
  if (!force_pers) {
    // persistent: launches run one after another, each ~kPersistStepUs per
    // step; step path: one launch per step for the whole batch, bound by
    // the larger of the launch floor and the traffic (read + write of the
    // active rows)
    double t_pers = 0.0, bytes = 0.0;
    int smax = 0, nwg = 0, lsteps = 0, lg = 0;
    for (int q : cand) {
      const IdProblem& p = h[q].p;
      int steps = h[q].kmax;
      if (p.kfail >= 0 && p.m > p.d) steps = std::min(steps, p.kfail + 2);
      smax = std::max(smax, steps);
      bytes += 16.0 * p.m * std::max(1.0, p.d - 0.5 * steps);  // per step, averaged
      const int G = (p.m + cpg - 1) / cpg;
      if (G > maxwg) continue;
      if (nwg + G > maxwg) {
        t_pers += lsteps * (kPersistStepUs + kPersistStepUsPerWg * lg);
        nwg = 0;
        lsteps = 0;
        lg = 0;
      }
      nwg += G;
      lsteps = std::max(lsteps, steps);
      lg = std::max(lg, G);
    }
    t_pers += lsteps * (kPersistStepUs + kPersistStepUsPerWg * lg);
    const double t_step = smax * std::max(kStepFloorUs, bytes * 1e6 / kStepBytesPerS);
    const char* vb = std::getenv("HSS_VERBOSE");
    if (vb && vb[0] >= '2') {
      long long sm = 0;
      for (int q : cand) sm += h[q].p.m;
      std::fprintf(stderr, "[hss-id] cost: %zu problems, sum m %lld, max d %d, <= %d steps, %d x %d columns resident: "
                   "persistent %.0f us, step %.0f us\n", cand.size(), sm, dmax, smax, maxwg, cpg, t_pers, t_step);
    }
    if (maxwg <= 0 || t_pers >= t_step) {
      rest.insert(rest.end(), cand.begin(), cand.end());
      return hipSuccess;
    }
  }
  // one persistent grid on the device at a time: two of them started from
  // different streams could each hold part of the device and wait for the
  // rest (until the bounded wait gives up), so launch and completion happen
  // under a process-wide lock
  static std::mutex persist_mu;
  std::lock_guard<std::mutex> lock(persist_mu);
  std::vector<int> done;
  std::vector<char> launched(h.size(), 0);
  std::vector<int> kchk(h.size(), 0);
  bool checked_all = true;  // every launched problem's rank is known on the host
  size_t i0 = 0;
  while (i0 < cand.size()) {
    // before a second side whose first side ran in an earlier launch: wait,
    // read the ranks, and skip the second sides of the nodes that failed
    // (unless a wait of those launches timed out: then nothing is known)
    if (!checked_all) {
      bool need = false;
      for (size_t i = i0; i < cand.size() && !need; ++i) {
        const int pq = h[cand[i]].p.partner;
        need = pq >= 0 && launched[pq];
      }
      if (need) {
        int herr = 0;
        hipError_t e = hipMemcpyAsync(&herr, w.err, 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(kchk.data(), w.k, h.size() * 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        checked_all = true;
        if (!herr) {
          std::vector<int> keep(cand.begin(), cand.begin() + i0);
          for (size_t i = i0; i < cand.size(); ++i) {
            const int q = cand[i], pq = h[q].p.partner;
            if (pq >= 0 && launched[pq] && fails_rule(h[pq].p, kchk[pq])) skipped[q] = 1;
            else keep.push_back(q);
          }
          const char* vb = std::getenv("HSS_VERBOSE");
          if (vb && vb[0] >= '2' && keep.size() < cand.size()) {
            std::fprintf(stderr, "[hss-id] %zu second sides skipped: their node's first side failed\n",
                         cand.size() - keep.size());
            std::fflush(stderr);
          }
          cand.swap(keep);
          if (i0 >= cand.size()) break;
        }
      }
    }
    std::vector<int> batch, wgp;
    int nwg = 0;
    size_t i1 = i0;
    for (; i1 < cand.size(); ++i1) {
      const int q = cand[i1];
      const int G = (h[q].p.m + cpg - 1) / cpg;
      if (G > maxwg) {  // never fits: step path
        rest.push_back(q);
        continue;
      }
      if (nwg + G > maxwg) break;
      h[q].g0 = nwg;
      h[q].G = G;
      for (int t = 0; t < G; ++t) wgp.push_back(q);
      nwg += G;
      batch.push_back(q);
      if (off2[q] >= 0 && !w_orig[q]) {  // in place without pivoting: write to W2
        w_orig[q] = h[q].p.W;
        ld_orig[q] = h[q].p.ldw;
        h[q].p.W = w.W2 + off2[q];
        h[q].p.ldw = h[q].p.d;
      }
    }
    i0 = i1;
    if (batch.empty()) continue;
    if (!st.reserve({sizeof(DevProb) * h.size(), wgp.size() * 4})) return hipErrorOutOfMemory;
    const DevProb* dprobs = static_cast<const DevProb*>(st.push(h.data(), sizeof(DevProb) * h.size()));
    const int* dwg = static_cast<const int*>(st.push(wgp.data(), wgp.size() * 4));
    if (!dprobs || !dwg) return hipErrorOutOfMemory;
    int kb = 1;  // the launch's records: steps 0..kb-1 of nwg workgroups (kb apart), zeroed
    for (int q : batch) kb = std::max(kb, h[q].kmax);
    hipError_t e = hipMemsetAsync(w.rec, 0, (size_t)kb * nwg * 16, s);
    // column slots per workgroup: 2, or for problems without pivoting as
    // many as the workspace's 2 x nslots slots allow, up to 8
    int rs = 2;
    bool allnp = true;
    for (int q : batch) allnp = allnp && h[q].p.nfac > 0;
    if (const char* r2 = std::getenv("HSS_QRCP_RING2"))  // tests: the exchange at every step
      if (r2[0] && r2[0] != '0') allnp = false;
    while (allnp && rs < 8 && 2LL * rs * nwg <= 2 * w.nslots) rs *= 2;
    // the launch's column slots (rs x nwg, two words per row): zero tags, so
    // that nothing left by an earlier launch passes for this one's
    if (e == hipSuccess) e = hipMemsetAsync(w.cbuf, 0, (size_t)rs * nwg * 2 * w.ldcb * 8, s);
    if (e == hipSuccess && done.empty()) e = hipMemsetAsync(w.err, 0, 4, s);
    if (e != hipSuccess) return e;
    Work wa = w;
    wa.rstride = kb;
    wa.rmask = rs - 1;
    wa.xmask = rs / 2 - 1;
    {
      const char* gu = std::getenv("HSS_QRCP_GIVE_UP");
      wa.give_up = (gu && gu[0] && gu[0] != '0') ? 1 : 0;
    }
    if (const char* vb = std::getenv("HSS_VERBOSE"); vb && vb[0] >= '2') {
      std::fprintf(stderr, "[hss-id] persistent launch: %zu problems, %d workgroups, %d column slots each\n",
                   batch.size(), nwg, rs);
      std::fflush(stderr);
    }
    void* args[] = {(void*)&dprobs, (void*)&dwg, (void*)&rtol, (void*)&wa};
    e = hipLaunchKernel(pv.fn, dim3(nwg), dim3(PT), args, 0, s);
    if (e == hipSuccess) {
      npersist += (int)batch.size();
      ++nlaunch;
      done.insert(done.end(), batch.begin(), batch.end());
      for (int q : batch) launched[q] = 1;
      checked_all = false;
    } else {
      (void)hipGetLastError();
      rest.insert(rest.end(), batch.begin(), batch.end());
    }
    for (int q : batch) {
      h[q].g0 = -1;
      h[q].G = 0;
    }
  }
  // the in-place problems back to their own W: those launched and finished
  // are copied there (on a timeout their untouched inputs are factored
  // again in place, as are problems whose launch failed)
  auto restore = [&](bool copy) -> hipError_t {
    for (size_t q = 0; q < h.size(); ++q) {
      if (!w_orig[q]) continue;
      if (copy && launched[q]) {
        const hipError_t ce =
            hipMemcpy2DAsync(w_orig[q], (size_t)ld_orig[q] * 8, h[q].p.W, (size_t)h[q].p.ldw * 8,
                             (size_t)h[q].p.d * 8, (size_t)h[q].p.m, hipMemcpyDeviceToDevice, s);
        if (ce != hipSuccess) return ce;
      }
      h[q].p.W = w_orig[q];
      h[q].p.ldw = ld_orig[q];
      w_orig[q] = nullptr;
    }
    return hipSuccess;
  };
  if (done.empty()) return restore(false);
  // a wait that timed out (workgroups not all resident at once): the inputs
  // are untouched, so the per-step path factors those problems again
  int herr = 0;
  hipError_t e = hipMemcpyAsync(&herr, w.err, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  if (herr) {  // (a skip decided above saw no timeout: those nodes fail either way)
    const char* vb = std::getenv("HSS_VERBOSE");
    if (vb && vb[0] && vb[0] != '0') {
      std::fprintf(stderr, "[hss-id] persistent wait gave up: %zu problems factored again on the step path\n",
                   done.size());
      std::fflush(stderr);
    }
    rest.insert(rest.end(), done.begin(), done.end());
    for (size_t q = 0; q < skipped.size(); ++q)  // their partners are factored again: so are they
      if (skipped[q]) {
        skipped[q] = 0;
        rest.push_back((int)q);
      }
    npersist = 0;
    nlaunch = 0;
  }
  return restore(herr == 0);
}

static size_t round_up_256(size_t b) { return (b + 255) / 256 * 256; }

// Workgroups of small-problem class c resident on the device at once.
static int small_resident(int c) {
  static int cache[kSmallClasses] = {0};
  static std::once_flag once;
  std::call_once(once, [] {
    const void* fns[kSmallClasses] = {
        reinterpret_cast<const void*>(&qrcp_reg16_kernel<1, 4>),
        reinterpret_cast<const void*>(&qrcp_reg16_kernel<2, 4>),
        reinterpret_cast<const void*>(&qrcp_reg16_kernel<4, 4>),
        reinterpret_cast<const void*>(&qrcp_reg16_kernel<8, 4>),
        reinterpret_cast<const void*>(&qrcp_reg16_kernel<2, 8>),
        reinterpret_cast<const void*>(&qrcp_reg16_kernel<4, 8>),
        reinterpret_cast<const void*>(&qrcp_reg_kernel<16, 16, 2>),
        reinterpret_cast<const void*>(&qrcp_reg16_kernel<2, 12>),
        reinterpret_cast<const void*>(&qrcp_reg16_kernel<4, 12>),
        reinterpret_cast<const void*>(&qrcp_reg_kernel<16, 16, 3>)};
    const int waves[kSmallClasses] = {8, 8, 8, 8, 8, 8, 16, 8, 8, 16};
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 256;
    for (int c = 0; c < kSmallClasses; ++c) {
      int per = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fns[c], waves[c] * 64, 0) != hipSuccess) per = 1;
      cache[c] = std::max(1, per) * cus;
    }
  });
  return cache[c];
}

hipError_t launch_id_factor(IdProblem* probs, int nprob, double rtol, void* work, size_t work_bytes,
                            int* k_host, Staging& st, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  if (work_bytes < id_workspace_bytes(probs, nprob)) return hipErrorInvalidValue;
  Work w;
  long long tm, tk, tw;
  carve(probs, nprob, work, w, tm, tk, tw);
  std::vector<DevProb> h(nprob);
  long long off = 0, aoff = 0, woff = 0;
  int g = 0, dmax = 1, smax = 0;
  std::vector<int> wg_prob, small[kSmallClasses], large;
  for (int q = 0; q < nprob; ++q) {
    IdProblem& p = probs[q];
    if (!p.W) {
      p.ldw = p.d > 0 ? p.d : 1;
      p.W = w.W + woff;
      woff += (long long)p.m * p.d;
    }
    DevProb& dp = h[q];
    dp.p = p;
    dp.off = off;
    dp.aoff = aoff;
    dp.kmax = kmax_of(p);
    off += p.m;
    aoff += dp.kmax;
    dp.g0 = -1;
    dp.G = 0;
    if (p.m == 0 || p.d == 0) {
      dp.kmax = 0;
    }
    const int sc = small_class(p);
    if (sc >= 0) small[sc].push_back(q);
    else large.push_back(q);
  }
  // large pivoted problems: persistent launches where they fit, the rest
  // one launch per step
  int npersist = 0, nplaunch = 0;
  std::vector<char> skipped(nprob, 0);
  {
    std::vector<int> rest;
    hipError_t e = run_persistent(h, large, rtol, w, st, s, rest, skipped, npersist, nplaunch);
    if (e != hipSuccess) return e;
    large.swap(rest);
  }
  for (int q : large) {
    DevProb& dp = h[q];
    const IdProblem& p = probs[q];
    dp.g0 = g;
    dp.G = (p.m + SW - 1) / SW;
    for (int t = 0; t < dp.G; ++t) wg_prob.push_back(q);
    g += dp.G;
    dmax = std::max(dmax, p.d);
    int steps = dp.kmax;
    if (p.kfail >= 0 && p.m > p.d) steps = std::min(steps, p.kfail + 2);
    smax = std::max(smax, steps);
  }
  // Small problems: when they fill the device for two rounds or more, the
  // first side of every node runs first and the second side only where the
  // first passed the rule (a node with a failing side fails either way), at
  // the cost of one wait; a single round is latency-bound and runs at once.
  std::vector<int> small_b[kSmallClasses];
  bool split = false;
  {
    double rounds = 0.0;
    bool pairs = false;
    for (int c = 0; c < kSmallClasses; ++c) {
      if (small[c].empty()) continue;
      rounds += (double)small[c].size() / std::max(1, small_resident(c));
      for (int q : small[c]) pairs = pairs || (probs[q].partner >= 0 && probs[q].kfail >= 0);
    }
    const char* ss = std::getenv("HSS_QRCP_SMALL_SPLIT");  // tests: 1 always, 0 never
    split = pairs && (ss && ss[0] ? ss[0] == '1' : rounds >= 2.0);
    if (split)
      for (int c = 0; c < kSmallClasses; ++c) {
        std::vector<int> a;
        for (int q : small[c]) {
          const int pq = probs[q].partner;
          if (pq >= 0 && pq < q && small_class(probs[pq]) >= 0) small_b[c].push_back(q);
          else a.push_back(q);
        }
        small[c].swap(a);
      }
  }
  // every table of the launches below stays valid until the last of them
  {
    size_t tot = round_up_256(sizeof(DevProb) * nprob) + round_up_256(wg_prob.size() * 4);
    for (int c = 0; c < kSmallClasses; ++c)
      tot += round_up_256(small[c].size() * 4) + round_up_256(small_b[c].size() * 4);
    if (!st.reserve({tot})) return hipErrorOutOfMemory;
  }
  const DevProb* dprobs = static_cast<const DevProb*>(st.push(h.data(), sizeof(DevProb) * nprob));
  if (!dprobs) return hipErrorOutOfMemory;
  hipError_t e = hipMemsetAsync(w.ndone, 0, 4, s);
  if (e != hipSuccess) return e;
  // small problems: one register-resident workgroup each
  auto launch_small = [&](std::vector<int>* lists) -> hipError_t {
    for (int c = 0; c < kSmallClasses; ++c) {
      std::vector<int>& L = lists[c];
      if (L.empty()) continue;
      const int* dl = static_cast<const int*>(st.push(L.data(), L.size() * 4));
      if (!dl) return hipErrorOutOfMemory;
      const dim3 grid((unsigned)L.size());
      // a list of factorizations without pivoting only (the ULV factor's);
      // HSS_REG_NOPIV=0 keeps them on the pivoting kernel (tests compare)
      const char* nv = std::getenv("HSS_REG_NOPIV");
      bool nopiv_list = !(nv && nv[0] == '0');
      for (int q : L) nopiv_list = nopiv_list && probs[q].nfac > 0;
#define QR_LAUNCH(G_, R_)                                                                           \
  if (nopiv_list)                                                                                   \
    hipLaunchKernelGGL((qrcp_reg16_kernel<G_, R_, true>), grid, dim3(512), 0, s, dprobs, dl, rtol, w); \
  else                                                                                              \
    hipLaunchKernelGGL((qrcp_reg16_kernel<G_, R_>), grid, dim3(512), 0, s, dprobs, dl, rtol, w)
#define QR_LAUNCH64(W_, C_, R_)                                                                        \
  if (nopiv_list)                                                                                      \
    hipLaunchKernelGGL((qrcp_reg_kernel<W_, C_, R_, true>), grid, dim3(W_ * 64), 0, s, dprobs, dl, rtol, w); \
  else                                                                                                 \
    hipLaunchKernelGGL((qrcp_reg_kernel<W_, C_, R_>), grid, dim3(W_ * 64), 0, s, dprobs, dl, rtol, w)
      // 16 lanes per column: (column groups, rows per lane) = 32 G columns,
      // 16 R rows; the two largest classes, whose 16-lane form would spill
      // registers inside the step loop, keep 64 lanes per column (W
      // wavefronts, C columns per wavefront, R rows per lane), on 16
      // wavefronts: each runs half as many columns' sum chains per step
      switch (c) {
        case 0: QR_LAUNCH(1, 4); break;
        case 1: QR_LAUNCH(2, 4); break;
        case 2: QR_LAUNCH(4, 4); break;
        case 3: QR_LAUNCH(8, 4); break;
        case 4: QR_LAUNCH(2, 8); break;
        case 5: QR_LAUNCH(4, 8); break;
        case 6: QR_LAUNCH64(16, 16, 2); break;
        case 7: QR_LAUNCH(2, 12); break;
        case 8: QR_LAUNCH(4, 12); break;
        default: QR_LAUNCH64(16, 16, 3); break;
      }
#undef QR_LAUNCH
#undef QR_LAUNCH64
      const hipError_t le = hipGetLastError();
      if (le != hipSuccess) return le;
    }
    return hipSuccess;
  };
  e = launch_small(small);
  if (e != hipSuccess) return e;
  if (split) {
    // the first sides' ranks, then the second sides of the nodes still alive
    std::vector<int> kk(nprob, 0);
    e = hipMemcpyAsync(kk.data(), w.k, (size_t)nprob * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    int nskip = 0;
    for (int c = 0; c < kSmallClasses; ++c) {
      std::vector<int> b;
      for (int q : small_b[c]) {
        const int pq = probs[q].partner;
        if (fails_rule(probs[pq], kk[pq])) {
          skipped[q] = 1;
          ++nskip;
        } else {
          b.push_back(q);
        }
      }
      small_b[c].swap(b);
    }
    const char* vb = std::getenv("HSS_VERBOSE");
    if (vb && vb[0] >= '2') {
      std::fprintf(stderr, "[hss-id] small problems in two phases: %d second sides skipped\n", nskip);
      std::fflush(stderr);
    }
    e = launch_small(small_b);
    if (e != hipSuccess) return e;
  }
  {
    const char* v = std::getenv("HSS_VERBOSE");
    if (v && v[0] && v[0] != '0' && (npersist > 0 || g > 0)) {
      std::fprintf(stderr,
                   "[hss-id] %d problems, %d persistent (%d launches), %d step-path workgroups "
                   "(<= %d steps)\n",
                   nprob, npersist, nplaunch, g, smax);
      std::fflush(stderr);
    }
  }
  // large problems: a launch per pivot step
  if (g > 0) {
    const int* dwg = static_cast<const int*>(st.push(wg_prob.data(), wg_prob.size() * 4));
    if (!dwg) return hipErrorOutOfMemory;
    long long tg = 0;
    for (int q = 0; q < nprob; ++q) tg += (probs[q].m + SW - 1) / SW;
    hipLaunchKernelGGL(id_init_kernel, dim3(g), dim3(ST), 0, s, dprobs, dwg, tg, w);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    int nlarge = 0;
    for (int q = 0; q < nprob; ++q) nlarge += h[q].g0 >= 0 ? 1 : 0;
    // The register variants stage rows i..d-1 of the reflector in LDS: at
    // most 64 * kStepTMax values.  Steps with more active rows than that
    // take the general loop, which streams the pivot column from memory.
    constexpr int kStepTMax = 64;
    const size_t lds = (size_t)std::min(dmax, 64 * kStepTMax) * 8;
    for (int i = 0; i < smax; ++i) {
      // rows i..d-1 are active: registers per lane follow the largest d - i
      const int tb = (dmax - i + 63) / 64;
#define STEP(T_) hipLaunchKernelGGL(id_step_kernel<T_>, dim3(g), dim3(ST), lds, s, dprobs, dwg, i, rtol, tm, tg, w)
      if (tb > kStepTMax) STEP(0);
      else if (tb <= 2) STEP(2);
      else if (tb <= 4) STEP(4);
      else if (tb <= 8) STEP(8);
      else if (tb <= 12) STEP(12);
      else if (tb <= 16) STEP(16);
      else if (tb <= 20) STEP(20);
      else if (tb <= 24) STEP(24);
      else if (tb <= 28) STEP(28);
      else if (tb <= 32) STEP(32);
      else if (tb <= 36) STEP(36);
      else if (tb <= 40) STEP(40);
      else if (tb <= 48) STEP(48);
      else if (tb <= 56) STEP(56);
      else STEP(64);
#undef STEP
      if ((i & 63) == 63 && i + 1 < smax) {  // stop early once every problem is done
        int nd = 0;
        e = hipMemcpyAsync(k_host, w.ndone, 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        nd = k_host[0];
        if (nd >= nlarge) break;
      }
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  e = hipMemcpyAsync(k_host, w.k, (size_t)nprob * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  for (int q = 0; q < nprob; ++q)  // not factored: the other side of the node failed
    if (skipped[q]) k_host[q] = 0;
  return e;
}

hipError_t launch_id_finish(const IdProblem* probs, int nprob, const int* k_host, const int* sel,
                            int nsel, void* work, Staging& st, hipStream_t s) {
  if (nsel <= 0) return hipSuccess;
  Work w;
  long long tm, tk, tw;
  carve(probs, nprob, work, w, tm, tk, tw);
  std::vector<DevProb> h(nprob);
  long long off = 0, aoff = 0;
  for (int q = 0; q < nprob; ++q) {
    h[q].p = probs[q];
    h[q].off = off;
    h[q].aoff = aoff;
    h[q].kmax = kmax_of(probs[q]);
    off += probs[q].m;
    aoff += h[q].kmax;
  }
  if (!st.reserve({sizeof(DevProb) * nprob, (size_t)nsel * 4})) return hipErrorOutOfMemory;
  const DevProb* dprobs = static_cast<const DevProb*>(st.push(h.data(), sizeof(DevProb) * nprob));
  const int* dsel = static_cast<const int*>(st.push(sel, (size_t)nsel * 4));
  if (!dprobs || !dsel) return hipErrorOutOfMemory;
  hipLaunchKernelGGL(id_perm_kernel, dim3(nsel), dim3(NT), 0, s, dprobs, dsel, w);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // blocked back substitution, last block first
  int maxblk = 0;
  for (int t = 0; t < nsel; ++t) {
    const int q = sel[t], k = k_host[q];
    if (k > 0 && probs[q].m > k) maxblk = std::max(maxblk, (k + 63) / 64);
  }
  std::vector<GemmDesc> gd;
  std::vector<DiagDesc> dd;
  for (int b = maxblk - 1; b >= 0; --b) {
    gd.clear();
    dd.clear();
    long long wg = 0;
    for (int t = 0; t < nsel; ++t) {
      const int q = sel[t], k = k_host[q];
      const IdProblem& p = probs[q];
      const int nrest = p.m - k;
      if (k <= 0 || nrest <= 0 || b * 64 >= k) continue;
      const int b0 = b * 64, b1 = std::min(k, b0 + 64);
      GemmDesc g{};
      g.M = nrest;
      g.N = b1 - b0;
      g.K = k - b1;
      g.A = p.E + b1;
      g.lda = k;
      g.B = Seg{p.W + b0, nullptr, p.ldw, INT_MAX, p.perm + b1};
      g.C = Seg{p.W + b0, nullptr, p.ldw, INT_MAX, p.perm + k};
      g.D = SegOut{p.E + b0, nullptr, k, INT_MAX, nullptr};
      g.alpha = -1.0;
      g.beta = 1.0;
      gd.push_back(g);
      DiagDesc x;
      x.W = p.W;
      x.ldw = p.ldw;
      x.perm = p.perm;
      x.E = p.E;
      x.k = k;
      x.nrest = nrest;
      x.b0 = b0;
      x.b1 = b1;
      x.wg0 = wg;
      wg += (nrest + NT - 1) / NT;
      dd.push_back(x);
    }
    if (dd.empty()) continue;
    e = launch_gemm_batched(gd.data(), (int)gd.size(), st, s);
    if (e != hipSuccess) return e;
    const DiagDesc* ddev = static_cast<const DiagDesc*>(st.push(dd.data(), dd.size() * sizeof(DiagDesc)));
    if (!ddev) return hipErrorOutOfMemory;
    int nbmax = 1;
    for (const DiagDesc& x : dd) nbmax = std::max(nbmax, x.b1 - x.b0);
    if (nbmax <= 16)
      hipLaunchKernelGGL(trsm_diag_kernel<16>, dim3((unsigned)wg), dim3(NT), 0, s, ddev, (int)dd.size());
    else if (nbmax <= 32)
      hipLaunchKernelGGL(trsm_diag_kernel<32>, dim3((unsigned)wg), dim3(NT), 0, s, ddev, (int)dd.size());
    else
      hipLaunchKernelGGL(trsm_diag_kernel<64>, dim3((unsigned)wg), dim3(NT), 0, s, ddev, (int)dd.size());
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

namespace {
// one workgroup per factored column i of a no-pivot problem
struct RefRow {
  int q;
  int i;
};
__global__ __launch_bounds__(NT) void qr_reflector_kernel(const DevProb* __restrict__ probs,
                                                         const RefRow* __restrict__ rows, Work w) {
  const RefRow rr = rows[blockIdx.x];
  const DevProb dp = probs[rr.q];
  const IdProblem& P = dp.p;
  const int i = rr.i;
  double* wi = P.W + (long long)i * P.ldw;
  const double alpha = w.alpha[dp.aoff + i];
  const double x0 = wi[i];
  const double v0 = x0 - alpha;
  const bool zero = alpha == 0.0;
  const double inv_v0 = zero ? 0.0 : 1.0 / v0;
  __syncthreads();  // every thread has read x0 before it is replaced
  for (int r = i + 1 + threadIdx.x; r < P.d; r += NT) wi[r] = zero ? 0.0 : wi[r] * inv_v0;
  if (threadIdx.x == 0) {
    wi[i] = alpha;
    P.tau[i] = zero ? 0.0 : -v0 / alpha;
  }
}
}  // namespace

hipError_t launch_qr_reflectors(const IdProblem* probs, int nprob, void* work, Staging& st,
                                hipStream_t s) {
  Work w;
  long long tm, tk, tw;
  carve(probs, nprob, work, w, tm, tk, tw);
  std::vector<DevProb> h(nprob);
  std::vector<RefRow> rows;
  long long off = 0, aoff = 0;
  for (int q = 0; q < nprob; ++q) {
    h[q].p = probs[q];
    h[q].off = off;
    h[q].aoff = aoff;
    h[q].kmax = kmax_of(probs[q]);
    off += probs[q].m;
    aoff += h[q].kmax;
    if (probs[q].nfac > 0)
      for (int i = 0; i < h[q].kmax; ++i) rows.push_back(RefRow{q, i});
  }
  if (rows.empty()) return hipSuccess;
  if (!st.reserve({sizeof(DevProb) * nprob, rows.size() * sizeof(RefRow)})) return hipErrorOutOfMemory;
  const DevProb* dprobs = static_cast<const DevProb*>(st.push(h.data(), sizeof(DevProb) * nprob));
  const RefRow* drows = static_cast<const RefRow*>(st.push(rows.data(), rows.size() * sizeof(RefRow)));
  if (!dprobs || !drows) return hipErrorOutOfMemory;
  hipLaunchKernelGGL(qr_reflector_kernel, dim3((unsigned)rows.size()), dim3(NT), 0, s, dprobs, drows, w);
  return hipGetLastError();
}

}  // namespace hss
