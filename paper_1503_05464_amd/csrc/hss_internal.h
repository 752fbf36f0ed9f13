// Internal declarations shared by the host orchestration and the HIP
// kernels of the randomized HSS library (gfx950).
#pragma once

#include <initializer_list>
#include <vector>

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hss {

// ---------------------------------------------------------------------------
// Staging of per-launch descriptor tables: a pinned host buffer and its
// device mirror, bump-allocated.  push() writes into the pinned buffer and
// queues the copy on the stream.  A block is rewritten only once the work
// that reads it has run: either the caller synchronised the stream (reset),
// or the block was retired behind an event (retire) and is taken again only
// after that event completed, so no queued copy or kernel ever reads a
// rewritten region.
// ---------------------------------------------------------------------------
struct Staging {
  char* host = nullptr;
  char* dev = nullptr;
  size_t cap = 0;
  size_t used = 0;
  hipStream_t stream = nullptr;
  bool stream_used = false;  // copies were queued on `stream`
  struct Spare {             // a retired block and the event its readers end before
    char* host;
    char* dev;
    size_t cap;
    hipEvent_t ev;
  };
  std::vector<Spare> spares;
  // Takes a block of at least `bytes` (a retired one whose readers have run,
  // or a new one).
  hipError_t init(size_t bytes, hipStream_t s);
  // Waits for the readers of every block, then frees them all.
  void release();
  // Returns the device address of the copied table, or nullptr on failure.
  // A push that does not fit retires the current block and continues in
  // another one, so tables pushed earlier are only safe if their kernels
  // were launched before that push; tables that must stay valid together
  // are reserved first.
  void* push(const void* src, size_t bytes);
  // Room for pushes of these sizes that stay valid together: any change of
  // block happens here, before the first of them.  False on failure.
  bool reserve(std::initializer_list<size_t> sizes);
  // The caller has synchronised the stream: the block is free again.
  void reset() { used = 0; }
  // Ends a stream-ordered call without waiting: the tables pushed so far stay
  // valid until the work queued on `stream` up to now has run; the next push
  // goes to another block.
  hipError_t retire();
};

// ---------------------------------------------------------------------------
// Random matrices: Philox4x64-10 + Box-Muller (kernels_rng.hip)
// ---------------------------------------------------------------------------
void launch_random_normal(unsigned long long seed, int which, long long n, int col0, int col1,
                          double* R, long long ld, hipStream_t s);
// Columns col0..col0+ncol-1 of the random matrix `which` of one matrix, rows
// 0..n-1, written from R (column col0 at R[0], leading dimension ld).
struct RngJob {
  unsigned long long seed;
  int which;
  long long n;
  int col0, ncol;
  double* R;
  long long ld;
};
// Every job in one launch, each entry rounded to the sampling precision
// `mode` (0 FP64, 1 FP32, 2 BF16) as launch_round_r rounds it.
hipError_t launch_random_normal_batched(const RngJob* jobs, int njob, int mode, Staging& st,
                                        hipStream_t s);

// v rounded to nearest even to FP32 (mode 1) or to 8 significant bits, the
// precision of BF16 (mode 2: the low 45 bits of the FP64 fraction rounded
// away, a carry may bump the exponent); unchanged for mode 0.
__device__ __forceinline__ double round_sample_prec(double v, int mode) {
  if (mode == 1) return (double)(float)v;
  if (mode != 2) return v;
  unsigned long long u = (unsigned long long)__double_as_longlong(v);
  u += 0x00000FFFFFFFFFFFull + ((u >> 45) & 1ull);
  u &= ~0x00001FFFFFFFFFFFull;
  return __longlong_as_double((long long)u);
}

// ---------------------------------------------------------------------------
// Sampling products on FP64 MFMA (kernels_sample.hip)
//   Sr = (A - M) Rr, Sc = (A - M)^T Rc, M = leaf diagonal blocks if leaf_of
// `work` must hold sample_workspace_doubles(n, ncols) doubles (split-K
// partial sums); it may be null when that size is 0.
// ---------------------------------------------------------------------------
long long sample_workspace_doubles(long long n, int ncols);

// Reduced-precision sampling for FP32 A (kernels_sample_mixed.hip): mode 1 =
// FP32 MFMA, mode 2 = A split into three BF16 terms on BF16 MFMA; R must be
// representable in the mode's precision.  FP32 accumulation over chunks of
// 256 k, FP64 across chunks.
long long sample_mixed_workspace_doubles(long long n, int ncols);
hipError_t launch_sample_mixed(const float* A, long long n, long long lda, const int* leaf_of,
                               int ncols, int mode, const double* Rr, const double* Rc,
                               long long ldr, double* Sr, double* Sc, long long lds, double* work,
                               hipStream_t s);
// The sampling products of many matrices (one FP32 A each) in one launch per
// side; all of one mode.  Rr/Rc/Sr/Sc point at the first column to form.
struct SampleJob {
  const float* A;
  long long lda, n;
  const int* leaf_of;
  int ncols;
  const double* Rr;
  const double* Rc;
  long long ldr;
  double* Sr;
  double* Sc;
  long long lds;
};
long long sample_mixed_grouped_workspace_doubles(const SampleJob* jobs, int njob);
hipError_t launch_sample_mixed_grouped(const SampleJob* jobs, int njob, int mode, double* work,
                                       Staging& st, hipStream_t s);
// R columns col0..col1-1 (rows 0..n-1, leading dimension ld, R points at row
// 0 column 0) rounded to nearest even in place: mode 1 to FP32, mode 2 to
// BF16; mode 0 leaves R unchanged.
void launch_round_r(double* R, long long ld, long long n, int col0, int col1, int mode,
                    hipStream_t s);
void launch_sample(const void* A, int dtype, long long n, long long lda, const int* leaf_of,
                   int ncols, const double* Rr, const double* Rc, long long ldr, double* Sr,
                   double* Sc, long long lds, double* work, hipStream_t s);

// ---------------------------------------------------------------------------
// Batched FP64 GEMM with row gathers / scatters (kernels_gemm.hip)
//   D[rowD(r), c] = beta * C[rowC(r), c] + alpha * sum_k Aop(r, k) B[rowB(k), c]
// for r < M, c < N.  Aop(r, k) = A[r*lda + k] or, if transA, A[k*lda + r].
// A "segmented" source X with rows split at `split`: row q < split lives at
// X0 + q*ld, row q >= split at X1 + (q - split)*ld.  Maps are optional.
// ---------------------------------------------------------------------------
struct Seg {
  const double* p0;
  const double* p1;
  long long ld;
  int split;   // rows >= split come from p1 (split = INT_MAX: single segment)
  const int* map;  // optional logical-row -> segmented-row map
};
struct SegOut {
  double* p0;
  double* p1;
  long long ld;
  int split;
  const int* map;
};
struct GemmDesc {
  int M, N, K;
  const double* A;
  long long lda;
  int transA;
  Seg B;
  Seg C;
  SegOut D;
  double alpha, beta;
};
// Runs all problems of `descs` (host array) in one launch, with the tile
// shape `variant` (0 .. gemm_variants()-1) or, for variant < 0, the one the
// tuning table gives the batch's size class.
hipError_t launch_gemm_batched(const GemmDesc* descs, int nprob, Staging& st, hipStream_t s,
                               int variant = -1);
int gemm_variants();

// ---------------------------------------------------------------------------
// Batched interpolative decomposition (kernels_qrcp.hip)
// ---------------------------------------------------------------------------
struct IdProblem {
  const double* Y;   // rows of Y^T: m rows, d columns, leading dimension ldy
  long long ldy;
  int m, d;
  double* W;         // null: launch_id_factor uses a workspace copy of Y;
                     // set by the caller: factor in place in W (ld ldw, W == Y)
  long long ldw;
  int* perm;         // m entries out: J (pivot order) then rest (increasing)
  double* E;         // (m-k) x k out (row-major, ld = k)
  int kfail;         // early exit once k > kfail and k < m is certain (-1: never)
  int nfac;          // 0: pivoted ID; > 0: Householder QR without pivoting of
                     // columns 0..nfac-1, the other columns only transformed
  double* tau;       // no-pivot mode: nfac Householder scalars out
  int partner = -1;  // the problem of the same node's other side, or -1: when
                     // one side fails the rule (k > kfail, k < m) the node
                     // fails, so the other side may be skipped (k = 0)
};
// Device workspace for a batch (carved by the launcher).
size_t id_workspace_bytes(const IdProblem* probs, int nprob);
// Column-pivoted QR to tolerance of every problem; synchronises the stream
// and returns the ranks in k_host (pinned or pageable host array).
hipError_t launch_id_factor(IdProblem* probs, int nprob, double rtol, void* work, size_t work_bytes,
                            int* k_host, Staging& st, hipStream_t s);
// J / rest permutation and E for the problems listed in `sel` (after
// launch_id_factor on the same batch and workspace).
hipError_t launch_id_finish(const IdProblem* probs, int nprob, const int* k_host, const int* sel,
                            int nsel, void* work, Staging& st, hipStream_t s);
// No-pivot mode: stores reflector i (LAPACK style, unit leading entry
// implied) in row i of W beyond the diagonal, R_ii on the diagonal, and tau.
hipError_t launch_qr_reflectors(const IdProblem* probs, int nprob, void* work, Staging& st,
                                hipStream_t s);

// ---------------------------------------------------------------------------
// Small helpers (kernels_misc.hip)
// ---------------------------------------------------------------------------
struct GatherDesc {   // out[r*ldo + c] = A[rows[r]*lda + cols[c]] (widened)
  const int* rows;
  const int* cols;
  int nr, nc;
  double* out;
  long long ldo;
  int row_off, col_off;  // added to rows/cols (for contiguous ranges: rows = null)
  const void* A;         // this problem's matrix (same dtype as the launch), or null:
  long long lda;         // the launch's A and lda
};
hipError_t launch_gather(const void* A, int dtype, long long lda, const GatherDesc* descs,
                         int nprob, Staging& st, hipStream_t s);

struct IndexDesc {    // out[a] = base(perm[a]) for a < k; base(q) = q < split ? b0[q] (or q+off0) : b1[q-split]
  const int* perm;
  int k;
  const int* b0;
  const int* b1;
  int split;
  int off0;           // used when b0 == null: base(q) = off0 + q
  int* out;
};
hipError_t launch_index_compose(const IndexDesc* descs, int nprob, Staging& st, hipStream_t s);

void launch_leaf_of(int n_leaves, const int* lo_dev, const int* hi_dev, int* leaf_of, hipStream_t s);

}  // namespace hss
