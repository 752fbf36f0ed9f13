// Host-side state of an HSS handle: tree, per-node generators (device
// pointers into the handle's arena), compression bookkeeping and workspaces.
#pragma once

#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hss.h"
#include "hss_internal.h"

namespace hss {

// Device memory owned by a handle: large chunks, bump-allocated, 256-byte
// aligned, released together.
// Device memory below comes from the device's stream-ordered pool
// (hipMallocAsync / hipFreeAsync on the stream given), so allocating and
// freeing never synchronizes the device or blocks other host threads.
void* pool_alloc(size_t bytes, hipStream_t s);
void pool_free(void* p, hipStream_t s);
// orders stream s after event ev (device-side wait; host-side if that fails)
void order_after(hipStream_t s, hipEvent_t ev);

struct Arena {
  hipStream_t stream = nullptr;  // stream of the allocations and of the release
  std::vector<void*> chunks;
  char* cur = nullptr;
  size_t left = 0;
  size_t total = 0;
  size_t chunk = (size_t)64 << 20;  // minimum chunk size
  std::mutex mu;                     // handles of one batch may allocate from several threads
  void* alloc(size_t bytes);
  void release();
  Arena() = default;
  Arena(const Arena&) = delete;
  Arena& operator=(const Arena&) = delete;
  ~Arena() { release(); }
};

// A growable device buffer reused between launches (freed and reallocated
// larger when needed).
struct Scratch {
  void* p = nullptr;
  size_t cap = 0;
  hipStream_t last = nullptr;  // stream of the latest use: the free is ordered after it
  void* ensure(size_t bytes, hipStream_t s);
  void release();
};

struct Node {
  int lo = 0, hi = 0, left = -1, right = -1, parent = -1, height = 0;
  bool leaf() const { return left < 0; }
  int size() const { return hi - lo; }
  // compression state
  int state = HSS_UNTOUCHED;
  int cdone = 0;        // columns of the local samples / R_tau computed
  bool set_up = false;  // sizes fixed, D or B gathered, buffers allocated
  int mr = 0, mc = 0;   // rows of S^r_loc, S^c_loc (and of U, V)
  int kr = 0, kc = 0;   // ranks of U, V
  double* Sr = nullptr;  // local samples, mr x ldg (leaf: rows of the global S)
  double* Sc = nullptr;
  double* Rr = nullptr;  // R^r_tau = V^T R^r_in, kc x ldg
  double* Rc = nullptr;  // R^c_tau = U^T R^c_in, kr x ldg
  int* perm_r = nullptr;  // mr: J^r (pivot order) then the rest (increasing)
  int* perm_c = nullptr;
  double* Er = nullptr;   // (mr-kr) x kr
  double* Ec = nullptr;   // (mc-kc) x kc
  int* Ir = nullptr;      // global row skeleton (kr)
  int* Ic = nullptr;      // global column skeleton (kc)
  double* D = nullptr;    // leaf: size x size
  double* B12 = nullptr;  // inner: kr_a x kc_b
  double* B21 = nullptr;  // inner: kr_b x kc_a
  // ULV factors (Alg. 3).  Z (zrows x md, row-major, md = node dimension
  // mr, r = md - kr) holds, after the LQ factorization of W_t:
  //   rows 0..r-1        L (lower, row j entries 0..j) and the reflectors
  //                      (row i entries i+1..md-1, unit leading entry);
  //   rows r..r+kc-1     (Q Vh)^T, so columns 0..r-1 are Vt_t^T, r.. Vt_b^T;
  //   rows r+kc..        W_b Q^T: columns 0..r-1 are W_b Q_t^T, r.. Dt.
  double* Z = nullptr;
  double* tau = nullptr;  // r Householder scalars
  double* Yq = nullptr;   // the r reflectors as a dense Y (md x r, ld r), made once by the factor
  double* Tq = nullptr;   // triangular factors of Y's blocks of 64 reflectors (64 x 64 each)
};

struct Handle {
  long long n = 0;
  int dtype = HSS_F64;
  hss_opts opts{};
  std::vector<Node> nodes;
  int height = 0;                        // height of the root
  std::vector<std::vector<int>> levels;  // non-root nodes by height
  std::vector<int> leaves;               // leaves in index order
  // generators and factors (kept until the handle is destroyed; the handles
  // of one batch share one arena, freed with the last of them)
  std::shared_ptr<Arena> gen = std::make_shared<Arena>();
  Scratch work_id, work_sample, work_mv, work_misc;
  Staging staging;
  hipStream_t stream = nullptr;
  // global random matrices and samples, n x ldg
  double* Rr = nullptr;
  double* Rc = nullptr;
  double* Sr = nullptr;
  double* Sc = nullptr;
  long long ldg = 0;
  int* leaf_of = nullptr;
  int* k_host = nullptr;  // pinned readback of ranks
  // recorded after the work of the latest stream-ordered call (matvec,
  // solve): hss_destroy waits for it before the generators are freed
  hipEvent_t queued = nullptr;
  int k_host_cap = 0;
  // results
  int d = 0;
  int passes = 0;
  bool converged = true;
  bool compressed = false;
  bool factored = false;
  int verbose = 0;  // HSS_VERBOSE: 1 = one line per pass on stderr, 2 = also one per level
  double t_total = 0, t_sample = 0, t_levels = 0, t_id = 0, t_sgemm = 0;
  int n_sgemm = 0;
  double sgemm_flops = 0, sgemm_bytes = 0;
  // level kernels: ID flops (4 d m k per attempt and side), local-sample and
  // R_tau GEMM bytes and time, D / B gather bytes and time
  double id_flops = 0, lgemm_bytes = 0, t_lgemm = 0, gather_bytes = 0, t_gather = 0;
  // ULV root LU with partial pivoting (device data)
  double* root_lu = nullptr;
  int* root_piv = nullptr;
  int* root_info = nullptr;
  int root_m = 0;
  long long generator_bytes() const;
};

// Records the thread-local error message returned by hss_last_error().
hss_status set_error(hss_status st, const std::string& msg);
hss_status matvec_impl(Handle& H, int nrhs, const double* x, long long ldx, double* b,
                       long long ldb, hipStream_t s);
// hss_compress_batched; share_arena = false gives every handle its own
// generator arena (for handles that outlive the others of their batch).
hss_status compress_batched(int nmat, const void* const* A, int dtype, const long long* n,
                            const long long* lda, const hss_tree* trees, const hss_opts* opts,
                            void* stream, hss_handle* out, int* status, bool share_arena);
// Device bytes a handle holds (generators, factors, workspaces, staging).
long long resident_bytes(const Handle& H);
// Records H.queued on s (after the work of a stream-ordered call).
hipError_t mark_queued(Handle& H, hipStream_t s);
// Checks the arguments of the sampling products (as hss_sample documents
// them); on success *work_doubles is the workspace the products need.
hss_status sample_args(const void* A, int dtype, int sample_prec, long long n, long long lda, int ncols,
                       const double* Rr, const double* Rc, long long ldr, double* Sr, double* Sc,
                       long long lds, long long* work_doubles);
// Queues the sampling products on s with the given workspace (no allocation).
hipError_t sample_queue(const void* A, int dtype, int sample_prec, long long n, long long lda,
                        const int* leaf_of, int ncols, const double* Rr, const double* Rc, long long ldr,
                        double* Sr, double* Sc, long long lds, double* work, hipStream_t s);

}  // namespace hss

struct hss_handle_s {
  hss::Handle h;
};
