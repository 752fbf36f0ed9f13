/*
 * hss.h -- C ABI of the MI355X (gfx950) randomized HSS library.
 *
 * Randomized compression of a dense n x n matrix into Hierarchically
 * Semi-Separable form, HSS matrix-vector products and the ULV-like
 * factorization and solve, following Rouet, Li, Ghysels, Napov,
 * "A distributed-memory package for dense Hierarchically Semi-Separable
 * matrix computations using randomization" (arXiv 1503.05464).
 *
 * Conventions shared by every entry point
 *  - Matrices are row-major: element (i, j) of a matrix with leading
 *    dimension ld is at p[i*ld + j].
 *  - Pointers named A, x, b, R, S, Y, ... are DEVICE pointers unless the
 *    comment says "host".  Caller-owned buffers are only read or written
 *    during the call (stream-ordered calls: until the work on `stream`
 *    completes) and never retained.
 *  - `stream` is a hipStream_t passed as void*; NULL is the default stream.
 *  - No C++ exception crosses the ABI.  Every call returns an hss_status;
 *    on an error, hss_last_error() returns a thread-local message.
 *  - A handle owns all of its device memory until hss_destroy().  Calls on
 *    one handle must not overlap; different handles are independent.
 */
#ifndef HSS_H
#define HSS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hss_handle_s* hss_handle;

typedef enum {
  HSS_OK = 0,
  HSS_NOT_CONVERGED = 1,  /* d reached d_max: the handle is complete and usable,
                             but some ID was accepted above the fail rule */
  HSS_ERR_ARG = -1,       /* invalid argument (sizes, pointers, tree) */
  HSS_ERR_ALLOC = -2,     /* device allocation failed */
  HSS_ERR_HIP = -3,       /* a HIP runtime call or kernel launch failed */
  HSS_ERR_STATE = -4,     /* call out of order (e.g. solve before factor) */
  HSS_ERR_SINGULAR = -5   /* a zero pivot in the ULV factors or the root LU */
} hss_status;

typedef enum { HSS_F64 = 0, HSS_F32 = 1 } hss_dtype; /* storage type of A */

/*
 * Precision of the sampling products S^r = A R^r, S^c = A^T R^c.  In the
 * reduced modes R is rounded once, when drawn (round to nearest even from the
 * FP64 value), and that rounded R is what every later step of the compression
 * uses, so the sampled products differ from FP64 products of the same A and R
 * only by accumulation: FP32 over chunks of 256 values of k, FP64 across
 * chunks.  The IDs, the B and D blocks and everything after them stay FP64.
 */
typedef enum {
  HSS_SAMPLE_F64 = 0,    /* FP64 MFMA; an FP32 A is widened exactly */
  HSS_SAMPLE_F32 = 1,    /* FP32 MFMA; A must be stored in FP32; R rounded to FP32 */
  HSS_SAMPLE_BF16X3 = 2  /* A must be stored in FP32 and is split exactly into three
                            BF16 terms; BF16 MFMA; R rounded to BF16 */
} hss_sample_prec;

/* Node states of the adaptive sampling (Sec. 3.3). */
enum { HSS_UNTOUCHED = 0, HSS_PARTIALLY_COMPRESSED = 1, HSS_COMPRESSED = 2 };

/*
 * Compression parameters (Sec. 2.2, Sec. 3.3).
 *  rtol      relative ID threshold eps: the pivoted QR of a node stops at
 *            the first pivot with |R_ii| <= rtol * |R_11|.
 *  d0, dd    initial number of random vectors and the growth step.
 *  d_max     cap on d; if a pass still fails at d_max, one more pass accepts
 *            every ID and hss_compress returns HSS_NOT_CONVERGED.
 *  p_margin  an ID of rank k fails when k > d - p_margin and k < m (m = rows
 *            of the node's local sample); default 10, the oversampling of
 *            Alg. 1 (d = r + 10).
 *  seed      Philox4x64-10 key; R^r and R^c entry (i, j) is a function of
 *            (seed, stream, i, j) only, so appended columns never depend on
 *            the growth history.
 *  leaf_size tree built by bisection when no tree is given.
 *  R_user_r, R_user_c  optional DEVICE n x d_max row-major random matrices
 *            (leading dimension ld_R_user) used instead of Philox; for tests.
 */
typedef struct {
  double rtol;
  int d0;
  int dd;
  int d_max;
  int p_margin;
  unsigned long long seed;
  int leaf_size;
  int sample_prec;            /* hss_sample_prec */
  const double* R_user_r;
  const double* R_user_c;
  long long ld_R_user;
} hss_opts;

/* Fills *o with rtol 1e-6, d0 64, dd 32, d_max 4096, p_margin 10, seed 0,
 * leaf_size 64, FP64 sampling, no user R. */
void hss_default_opts(hss_opts* o);

/*
 * Binary cluster tree (Sec. 2.1): host arrays of n_nodes entries; node 0 is
 * the root with interval [0, n); node t owns [lo[t], hi[t]); left/right are
 * child numbers or -1 for a leaf; the children split the parent interval
 * into two adjacent parts (left first).  Copied by the callee.
 */
typedef struct {
  int n_nodes;
  const int* lo;
  const int* hi;
  const int* left;
  const int* right;
} hss_tree;

/*
 * Randomized compression of the dense matrix A (Alg. 1) with adaptive
 * sampling (Alg. 5, late notification, run level by level over heights).
 *  A       DEVICE, n x n row-major, leading dimension lda >= n, storage type
 *          dtype (hss_dtype).  Read only; may be freed when the call returns
 *          (D and B are copied into the handle).
 *  tree    NULL: bisection tree of [0, n) with opts->leaf_size (intervals of
 *          m > leaf_size split into floor(m/2), ceil(m/2)).
 *  opts    NULL: hss_default_opts.
 *  *out    receives a new handle (also on HSS_NOT_CONVERGED).
 * Host-synchronous: returns when the handle is complete.  All device work is
 * issued on `stream`.  The random matrices, samples and other buffers of the
 * compression (about 4 n d_max doubles and more) are released before the
 * call returns, to the library's cache of device blocks (see
 * hss_release_cached_memory) or to the allocator set by hss_set_allocator;
 * the handle keeps only the generators.
 */
hss_status hss_compress(const void* A, int dtype, long long n, long long lda,
                        const hss_tree* tree, const hss_opts* opts, void* stream,
                        hss_handle* out);

/*
 * Compression of nmat independent matrices in one call, for callers with
 * many small problems (e.g. the frontal matrices of a sparse solver).  Each
 * matrix is compressed exactly as hss_compress would (Alg. 1 with the
 * adaptive sampling of Sec. 3.3 / Alg. 5): its own random matrices, its own
 * d, its own fail/retry decisions.  What is shared is the schedule: the
 * passes of all matrices run together, and each height of every unfinished
 * matrix is one batched launch of each phase (gathers, local-sample
 * products, IDs, index sets, R_tau), so small matrices fill the device
 * together.
 *  A[i]     DEVICE n[i] x n[i] row-major, leading dimension lda[i], all of
 *           one dtype; read during the call only.
 *  trees    NULL (bisection with opts->leaf_size) or nmat trees (as in
 *           hss_compress).
 *  opts     shared by all matrices; no user random matrices.
 *  out      nmat handles (each owned by the caller, hss_destroy each);
 *  status   optional host array: HSS_OK or HSS_NOT_CONVERGED per matrix.
 * Returns HSS_OK if every matrix converged, HSS_NOT_CONVERGED if any did
 * not (all handles valid), or an error, in which case no handle is
 * returned.  Host-synchronous; all work on `stream`.  The handles of one
 * call keep their generators in one shared device pool, freed when the last
 * of them is destroyed.
 */
hss_status hss_compress_batched(int nmat, const void* const* A, int dtype, const long long* n,
                                const long long* lda, const hss_tree* trees, const hss_opts* opts,
                                void* stream, hss_handle* out, int* status);

/*
 * b = A_HSS x (Alg. 2) for nrhs columns.  x: DEVICE n x nrhs (ldx >= nrhs),
 * b: DEVICE n x nrhs (ldb >= nrhs), must not overlap x.  Stream-ordered: all
 * device work is queued on `stream` and the call may return before it has
 * run; b is written once that work completes (synchronise `stream`, or order
 * later work after it).  x must stay unchanged until then.  A later call on
 * the handle may use another stream: it is ordered after this one.
 */
hss_status hss_matvec(hss_handle h, int nrhs, const double* x, long long ldx,
                      double* b, long long ldb, void* stream);

/*
 * b[i] = A_HSS[i] x[i] (Alg. 2) for nmat compressed handles at once, each
 * as hss_matvec computes it: every phase of Alg. 2 (the upward sweep of one
 * height, the downward sweep of one height, the leaves) is one batched
 * launch over all matrices, heights counted from the leaves.
 *  h        nmat distinct compressed handles (matrices of any sizes).
 *  x[i]     DEVICE n_i x nrhs, leading dimension ldx[i] >= nrhs.
 *  b[i]     DEVICE n_i x nrhs, leading dimension ldb[i] >= nrhs; must not
 *           overlap x[i].
 *  h, x, b, ldx, ldb are host arrays of nmat entries.
 * Uses h[0]'s workspace: not concurrently with another call on h[0].
 * Returns HSS_OK, HSS_ERR_STATE (a handle not compressed) or HSS_ERR_ARG;
 * nothing is computed on an error.  Stream-ordered, like hss_matvec.
 */
hss_status hss_matvec_batched(int nmat, const hss_handle* h, int nrhs, const double* const* x,
                              const long long* ldx, double* const* b, const long long* ldb,
                              void* stream);

/* ULV-like factorization of the HSS form (Alg. 3); root LU with partial
 * pivoting.  The handle keeps the factors, and each node's reflectors also
 * in compact WY form (a dense Y and the triangular T of each block of 64)
 * for the solves: together a few n x leaf_size blocks of device memory.
 * Host-synchronous.  A second call on a factored handle does nothing.
 * Returns HSS_OK, HSS_ERR_ARG (NULL handle), HSS_ERR_STATE (not
 * compressed), HSS_ERR_ALLOC, HSS_ERR_HIP or HSS_ERR_SINGULAR (a zero pivot
 * in the root LU). */
hss_status hss_factor(hss_handle h, void* stream);

/* Solve A_HSS x = b after hss_factor (Alg. 4).  b, x: DEVICE n x nrhs
 * (ldb, ldx >= nrhs); HSS_ERR_STATE before hss_factor.  Stream-ordered, like
 * hss_matvec: the work is queued on `stream`, x is written once it has run,
 * and b must stay unchanged until then. */
hss_status hss_solve(hss_handle h, int nrhs, const double* b, long long ldb,
                     double* x, long long ldx, void* stream);

/* Summary of a compression.  Times are wall-clock milliseconds measured
 * with HIP events on the compression stream. */
typedef struct {
  long long n;
  int n_nodes;
  int height;
  int d_final;
  int passes;
  int converged;
  int max_rank;
  long long generator_bytes;   /* D + B + E + index arrays */
  double sample_flops;         /* 4 n^2 d_final */
  double t_total_ms;
  double t_sample_ms;          /* random matrices + sampling products */
  double t_levels_ms;          /* local samples, IDs, updates */
  double t_id_ms;              /* pivoted QR + triangular solves */
  int n_sample_launches;       /* launches of the sampling GEMM kernel */
  double t_sample_gemm_ms;     /* their summed duration (HIP events on the stream) */
  double sample_gemm_flops;    /* their algorithmic flops, 2 n^2 per column per side */
  double sample_gemm_bytes;    /* their algorithmic bytes: A once per launch + R in + S out */
  double id_flops;             /* pivoted QRs: 4 d m k per ID attempt and side (k: steps taken) */
  double t_level_gemm_ms;      /* local-sample and R_tau products (HIP events) */
  double level_gemm_bytes;     /* their algorithmic bytes: operands once, C when read */
  double t_gather_ms;          /* D and B gathers from A (HIP events) */
  double gather_bytes;         /* their algorithmic bytes: entries read from A + written */
} hss_stats_t;

hss_status hss_stats(hss_handle h, hss_stats_t* st);

/* Per-node ranks and local-sample row counts (host arrays of n_nodes
 * entries; any may be NULL).  Root entries are 0. */
hss_status hss_ranks(hss_handle h, int* kr, int* kc, int* mr, int* mc);

/*
 * Generators of one node, host memory (hss_export fills caller buffers of
 * the sizes hss_ranks reports; hss_import reads them).  m = mr (U side) or
 * mc (V side) rows, k = kr or kc.
 *  Jr, Jc    k entries, pivot order, local row numbers in [0, m).
 *  Er, Ec    (m-k) x k row-major; row i belongs to the i-th smallest local
 *            row number not in J (U = Pi [I; E], Sec. 2.2).
 *  Ir, Ic    k global indices of the row / column skeleton (Alg. 1).
 *  D         leaves: |I| x |I| row-major diagonal block.
 *  B12, B21  inner nodes with children a, b: kr_a x kc_b and kr_b x kc_a.
 * Pointers that are NULL are skipped.
 */
typedef struct {
  int* Jr;
  int* Jc;
  double* Er;
  double* Ec;
  int* Ir;
  int* Ic;
  double* D;
  double* B12;
  double* B21;
} hss_node_generators;

hss_status hss_export_node(hss_handle h, int node, hss_node_generators* g);

/*
 * Builds a handle from host generators (for example from another
 * implementation): n, the tree (as in hss_compress), per-node ranks
 * kr[], kc[] (host, n_nodes entries, 0 at the root) and one
 * hss_node_generators per node (Ir, Ic unused).  Validates the index sets.
 */
hss_status hss_import(long long n, const hss_tree* tree, const int* kr, const int* kc,
                      const hss_node_generators* nodes, hss_handle* out);

/* Frees the handle's device memory, after the work of its stream-ordered
 * calls (matvec, solve) has run: waits for it on the host. */
void hss_destroy(hss_handle h);

/*
 * Device memory allocator for everything the library allocates on the device
 * (handles, compression buffers, workspaces), for callers that want one pool
 * for their framework and the library (e.g. PyTorch's caching allocator).
 *  alloc(bytes, device, stream, ctx)  returns at least `bytes` bytes of device
 *      memory on `device` (the current device of the call), 256-byte
 *      aligned, that work queued on `stream` after the call may use; NULL
 *      on failure (the library call then returns HSS_ERR_ALLOC).
 *  free(p, bytes, device, stream, ctx)  gives back a block: `stream` and
 *      `bytes` are those of the matching alloc; the library no longer uses p
 *      in work queued on `stream` after this call (it waited on the host for
 *      uses on other streams), so the allocator may reuse p for work queued
 *      later on that stream, as stream-ordered pools do.
 * Both NULL: the default (the runtime's stream-ordered pool plus the
 * library's cache of freed blocks, see hss_release_cached_memory).  Every
 * block goes back to the allocator that made it, so the allocator may be
 * changed while handles are live.  Process-wide; the callbacks may be called
 * from any thread (also the server's workers).  HSS_ERR_ARG if exactly one of
 * alloc, free is NULL.
 */
typedef void* (*hss_alloc_fn)(size_t bytes, int device, void* stream, void* ctx);
typedef void (*hss_free_fn)(void* p, size_t bytes, int device, void* stream, void* ctx);
hss_status hss_set_allocator(hss_alloc_fn alloc, hss_free_fn free, void* ctx);

/* Gives back to the runtime the memory that the library keeps for reuse:
   freed device blocks of 1 MB and more (up to a quarter of each device's
   memory is kept; a compression frees and allocates the same sizes from
   one call to the next) and pinned host staging blocks (up to 1 GiB).
   Memory of live handles, servers and calls in flight is not touched.
   Waits on the host until each cached block's last use has finished.
   Callable from any thread, at any time.  Returns HSS_OK, or HSS_ERR_HIP
   when a runtime call failed (the other blocks are still released). */
hss_status hss_release_cached_memory(void);

/* Thread-local message of the last error (empty string if none). */
const char* hss_last_error(void);

/* ---------------------------------------------------------------------
 * Serving: requests of compress (Alg. 1, adaptive sampling of Sec. 3.3) +
 * ULV factorization (Alg. 3) + solve (Alg. 4) that arrive over time, and
 * solve-only requests (Alg. 4) against handles the server keeps resident.
 *
 * Requests wait in arrival order.  Each worker thread of the server owns a
 * HIP stream; a free worker admits the oldest waiting request it can run
 * and, behind it, the waiting requests of the same kind:
 *  - compress requests with the same storage type and options, compressed
 *    together by one batched compression (hss_compress_batched), then
 *    factored and solved one by one;
 *  - solve-only requests on distinct resident handles, queued back to back
 *    on the worker's stream;
 * while their device footprint fits the budget and the batch holds at most
 * max_batch requests.  A compress request's footprint counts A, b and x,
 * the compression buffers (about 8 n d_max doubles) and the generators and
 * ULV factors; a solve-only request's counts b, x and the solve workspace.
 * Handles kept resident count with their actual device bytes until
 * hss_server_release.  Requests that arrive meanwhile are admitted by the
 * next free worker as memory frees up, so their work overlaps on the device
 * with the batches already running.  A request whose footprint alone
 * exceeds the budget runs when nothing else is admitted.  Each result is
 * computed exactly as the same calls made alone would compute it, up to the
 * rounding of a batch's QRCP path choice.
 * ------------------------------------------------------------------- */
typedef struct hss_server_s* hss_server;

typedef struct {
  long long hbm_budget; /* bytes of device memory admitted requests and resident
                           handles may hold; 0: 80 % of the device's memory */
  int max_batch;        /* requests admitted together (default 32) */
  int workers;          /* worker threads / streams, 1..16 (default 2) */
} hss_server_opts;

typedef struct {
  int status;       /* HSS_OK, HSS_NOT_CONVERGED, or the error of the request */
  int batch_size;   /* requests admitted in the same batch */
  int d_final;      /* random vectors used (compress requests) */
  int max_rank;     /* largest generator rank */
  double t_submit;  /* seconds since the server started: submitted, */
  double t_start;   /* admitted, */
  double t_done;    /* solved (results in x) */
  hss_handle handle; /* compress requests with keep = 1: the compressed and
                        factored handle, resident in the server until
                        hss_server_release; NULL otherwise */
} hss_request_info;

/* Fills *o with hbm_budget 0 (80 % of device memory), max_batch 32,
 * workers 2. */
void hss_server_default_opts(hss_server_opts* o);

/* Starts the worker threads.  opts NULL: defaults. */
hss_status hss_server_create(const hss_server_opts* opts, hss_server* out);

/*
 * One request.
 *  Compress request (handle NULL): compress A (DEVICE n x n row-major,
 *    leading dimension lda, storage dtype; opts as in hss_compress, NULL:
 *    defaults, no user random matrices), factor, and solve A_HSS x = b for
 *    nrhs columns (nrhs may be 0).  keep = 1 keeps the compressed and
 *    factored handle resident: it is returned in hss_request_info.handle and
 *    serves later solve-only requests; it belongs to the server (do not
 *    hss_destroy it) until hss_server_release.
 *  Solve-only request (handle = a resident handle, A NULL): solve
 *    A_HSS x = b with the handle's factors (nrhs >= 1); n is taken from the
 *    handle.  Requests on one handle run one at a time, in arrival order.
 *  b, x: DEVICE n x nrhs with leading dimensions ldb, ldx.
 */
typedef struct {
  const void* A;
  int dtype;
  long long n;
  long long lda;
  const hss_opts* opts;
  hss_handle handle;
  int nrhs;
  const double* b;
  long long ldb;
  double* x;
  long long ldx;
  int keep;
} hss_server_request;

/*
 * Queues request *r (copied).  The server reads A and b after the work queued
 * so far on `stream` (the stream that wrote them).  A and b must stay valid
 * and unchanged, and x untouched, until hss_server_wait on *ticket returns.
 * Returns at once.  HSS_ERR_ARG for invalid sizes or pointers or a handle
 * that is not resident in this server (or is being released).
 */
hss_status hss_server_submit_request(hss_server s, const hss_server_request* r, void* stream,
                                     long long* ticket);

/* A compress request with keep = 0 (the arguments of hss_server_request). */
hss_status hss_server_submit(hss_server s, const void* A, int dtype, long long n, long long lda,
                             const hss_opts* opts, int nrhs, const double* b, long long ldb,
                             double* x, long long ldx, void* stream, long long* ticket);

/*
 * Blocks until the request is done, fills *info (may be NULL) and forgets
 * the ticket.  Returns the request's status.
 */
hss_status hss_server_wait(hss_server s, long long ticket, hss_request_info* info);

/*
 * Destroys a resident handle (from a keep = 1 request) once the requests on
 * it that are queued or running have finished (waits for them), and gives
 * its bytes back to the budget.  HSS_ERR_ARG if h is not resident here.
 */
hss_status hss_server_release(hss_server s, hss_handle h);

/* Finishes every queued request, stops the workers, destroys the handles
 * still resident and frees the server. */
void hss_server_destroy(hss_server s);

/* ---------------------------------------------------------------------
 * Building blocks of hss_compress, exported for parity tests.
 * ------------------------------------------------------------------- */

/*
 * Columns col0..col1-1 of the Gaussian random matrix of `which` (0 = R^r,
 * 1 = R^c) for rows 0..n-1 into R (DEVICE, ld >= col1 - col0, column col0
 * at R[0]).  Entry (i, j): Philox4x64-10 with key (seed, 0) and counter
 * (i/4, j, which, 0) gives four words; word w maps to
 * u = ((w >> 12) + 1/2) 2^-52; rows 4q, 4q+1 are the Box-Muller pair of
 * (u0, u1), rows 4q+2, 4q+3 that of (u2, u3): sqrt(-2 ln ua) cos(2 pi ub),
 * sqrt(-2 ln ua) sin(2 pi ub).  With sample_prec HSS_SAMPLE_F32 or
 * HSS_SAMPLE_BF16X3 every entry is then rounded to nearest even to FP32 or
 * to BF16 (8 significant bits), as hss_compress does in that mode.
 * Stream-ordered.
 */
hss_status hss_random_normal(unsigned long long seed, int which, long long n, int col0,
                             int col1, int sample_prec, double* R, long long ld, void* stream);

/*
 * Sampling products (Sec. 2.2): Sr = (A - M) Rr and Sc = (A - M)^T Rc for
 * ncols columns, where M is zero (leaf_of == NULL) or the block-diagonal part
 * of A made of the leaf diagonal blocks (leaf_of: DEVICE int array of n
 * entries, the leaf number of each index; indices of one leaf are
 * contiguous), which yields the leaves' local samples directly:
 * S^(l) = (A - D^(l)) R (Sec. 2.2).  A: DEVICE n x n (dtype), Rr, Rc: DEVICE
 * n x ncols (ldr); Sr, Sc: DEVICE n x ncols (lds).  Either of Sr/Rr or
 * Sc/Rc may be NULL.  sample_prec as in hss_sample_prec: the reduced modes
 * need dtype HSS_F32 and R already representable in their precision
 * (hss_random_normal with the same sample_prec); HSS_ERR_ARG otherwise.
 * Stream-ordered in every mode.  The split-K partial sums (and, in the
 * reduced modes, the copies of R in the products' precision) go to a
 * workspace the call allocates and frees stream-ordered.
 */
hss_status hss_sample(const void* A, int dtype, int sample_prec, long long n, long long lda,
                      const int* leaf_of, int ncols, const double* Rr, const double* Rc,
                      long long ldr, double* Sr, double* Sc, long long lds, void* stream);

/*
 * hss_sample for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.  Same
 * arguments, same kernels and the same bits as hss_sample; the caller passes
 * the inputs and outputs, and the workspace comes from one fixed array of
 * 2^24 doubles (128 MiB) of device memory that the library holds on each
 * device it runs on until the process ends.  The call allocates nothing (no
 * hipMalloc, hipFree, pool or pinned staging).  Sizes whose workspace exceeds
 * the array (FP64: split-K partials of n x ncols per split; reduced modes:
 * also two n x ncols copies of R) return HSS_ERR_ARG with the needed size;
 * n = 65536 with 64 columns fits in every precision.  Stream-ordered.  Every
 * call on one device shares that array: calls that overlap on one device
 * (on different streams, or from different threads) race and give wrong
 * results; calls ordered on one stream are safe.
 */
hss_status hss_sample_noalloc(const void* A, int dtype, int sample_prec, long long n, long long lda,
                              const int* leaf_of, int ncols, const double* Rr, const double* Rc,
                              long long ldr, double* Sr, double* Sc, long long lds, void* stream);

/*
 * Batched FP64 GEMMs C_p = alpha op(A_p) B_p + beta C_p, op(A) = A or A^T, in
 * one launch of the kernel that runs the library's per-node products (local
 * samples and R_tau of Alg. 1, the sweeps of Alg. 2, the ULV updates of Alg.
 * 3/4).  For parity tests and for the tile autotuner.
 *  M, N, K, lda, transA, ldb, ldc: host arrays of nprob entries.
 *  A, B, C: host arrays of nprob DEVICE pointers, row-major: op(A_p) is
 *           M x K (A_p is M x K with lda >= K, or K x M with lda >= M if
 *           transA), B_p is K x N (ldb >= N), C_p is M x N (ldc >= N).  C_p
 *           must not overlap A_p or B_p.
 *  variant  tile shape 0 .. hss_gemm_variants()-1, or < 0 for the shape the
 *           tuning table gives the batch's size class (what the library uses).
 * Stream-ordered.  HSS_ERR_ARG for invalid sizes or a variant out of range.
 */
hss_status hss_gemm_batched(int nprob, const int* M, const int* N, const int* K, const double* const* A,
                            const long long* lda, const int* transA, const double* const* B,
                            const long long* ldb, double* const* C, const long long* ldc, double alpha,
                            double beta, int variant, void* stream);

/* Number of tile shapes of hss_gemm_batched. */
int hss_gemm_variants(void);

/*
 * Batched interpolative decompositions (Sec. 2.2, Sec. 3.2).  Problem p
 * takes the rows of a DEVICE matrix Y_p^T (m[p] rows, d[p] columns, leading
 * dimension ldy[p], pointer ys[p]) -- i.e. Y_p is d x m and its columns are
 * the rows given -- and returns its eps-rank k[p] (host), the selected
 * columns J (pivot order) followed by the rest in increasing order in
 * perm[p] (DEVICE, m entries), and E (DEVICE, (m-k) x k row-major) in
 * es[p] (capacity m*m/4+m doubles).  Host arrays ys, m, d, ldy, perms, es
 * of nprob entries.  Host-synchronous.
 */
hss_status hss_id_batched(int nprob, const double* const* ys, const int* m, const int* d,
                          const long long* ldy, double rtol, int* const* perms,
                          double* const* es, int* k, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HSS_H */
