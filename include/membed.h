/*
 * membed.h -- C ABI of the MI355X (gfx950) manifold-graph embedding library.
 *
 * Method: F. Chen, G. Cheung, X. Zhang, "Fast computation of generalized
 * eigenvectors for manifold graph embedding".  Given a symmetric positive
 * graph W (Section 3.1) the library builds
 *   - the disconnected two-hop sets T_i and Q = sum_i Theta_i   (Section 4.1.1, eq. (Q)),
 *   - eps = lambda_2(Q)                                        (Section 4.2),
 *   - mu = min_i mu_i                                          (Section 4.2, eq. (mu)),
 *   - A = L - mu Q + eps I                                     (eq. (obj2)),
 *   - b_i from the Gershgorin radii r_i of A, prod b_i = 1     (Section 4.3),
 * and returns the first K generalized eigenvectors of (A, B = diag(b)),
 * B-orthonormal (P^T B P = I), by LOBPCG (Section 4.3).
 *
 * Conventions for every entry point:
 *   - Pointers documented "device" point to GPU memory of the current HIP
 *     device; "host" pointers to CPU memory.  `stream` is a hipStream_t
 *     (NULL = the legacy default stream); all GPU work of a call is ordered
 *     on it.  Calls return after their results are complete on the device
 *     unless stated otherwise.
 *   - Status codes: 0 = success, > 0 = warning (outputs valid), < 0 = error
 *     (outputs untouched).  No entry point prints or aborts.
 *   - Dense N x K blocks are row-major (row i holds node i's K coordinates).
 *   - Threading: a handle may be used by one host thread at a time.
 *   - Device memory: every entry point that computes takes a caller-owned
 *     workspace (device memory, e.g. a uint8 tensor) with a query of its
 *     size; given one, the call carves every device array it needs from it
 *     and makes no device allocation (no hipMalloc, no pinned host memory).
 *     Passing NULL instead lets the library allocate stream-ordered device
 *     memory itself.  me_apply (a diagnostic hook) always allocates.
 */
#ifndef MEMBED_H
#define MEMBED_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ME_OK = 0,
  ME_WARN_NOT_CONVERGED = 1, /* max_iter reached; X, lambda are the last iterate      */
  ME_WARN_EPS_ZERO = 2,      /* two-hop graph disconnected: eps = mu = 0, A = L         */
  ME_ERR_INVALID_ARG = -1,   /* null pointer, bad sizes, unsorted/duplicate/out-of-range columns */
  ME_ERR_NOT_SYMMETRIC = -2, /* W_ij != W_ji (Section 3.1)                              */
  ME_ERR_SELF_LOOP = -3,     /* W_ii present                                            */
  ME_ERR_BAD_WEIGHT = -4,    /* weight not finite or <= 0 (Section 3.1: W_ij > 0); in
                                ME_MIXED also a weight beyond FP32's range              */
  ME_ERR_ISOLATED_NODE = -5, /* node with no edge: r_i = 0, b undefined (Section 4.3)   */
  ME_ERR_K_RANGE = -6,       /* K outside 1..16, or the LOBPCG block does not fit N     */
  ME_ERR_WORKSPACE = -7,     /* workspace missing or smaller than the query returned    */
  ME_ERR_HIP = -8,           /* a HIP runtime call failed                               */
  ME_ERR_BREAKDOWN = -9,     /* non-finite values appeared in the iteration             */
  ME_ERR_TOO_LARGE = -10     /* nnz(W) + nnz(T) exceeds 2^31 - 1                        */
} me_status;

/* Precision of the bulk N-length work (SpMM, Gram products, block updates).
 * The small dense solves (Cholesky, Rayleigh-Ritz) and the final residual
 * certificate are always FP64.  ME_MIXED keeps a copy of the weights in FP32
 * for the preconditioner: a graph with a weight above FP32's largest value
 * (3.4e38) is refused with ME_ERR_BAD_WEIGHT (ME_FP64 has no such limit), and one with
 * a weight past FP16's largest finite value (65504) runs its preconditioner
 * on FP32 weights instead of the packed 16-bit entries. */
enum { ME_FP64 = 0, ME_MIXED = 1 };
/* Preconditioner T of the LOBPCG residual (the paper names LOBPCG and leaves
 * T open): none; Jacobi diag(A)^-1; or `cheb_degree` steps of Chebyshev
 * iteration for A y = r with Jacobi scaling, i.e. a polynomial in
 * diag(A)^-1 A that approximates A^-1 on [a, b] (b: Gershgorin bound,
 * a: half the diag(A)-Rayleigh quotient of the leading Ritz vector). */
enum { ME_PRECOND_NONE = 0, ME_PRECOND_JACOBI = 1, ME_PRECOND_CHEBYSHEV = 2 };
/* The Chebyshev preconditioner of the embedding solve approximates the
 * inverse of L + eps I (one-hop entries only; spectrally within about mu |Q|
 * of A, and a third of the entries) or of A itself.  Any symmetric positive
 * definite preconditioner leaves the converged pairs unchanged; it only
 * changes the iteration count.  The eps solve's preconditioner always
 * inverts Q. */
enum { ME_CHEB_LAPLACIAN = 0, ME_CHEB_FULL = 1 };
/* Addressing of the operator-product kernels.  ME_ADDR_AUTO (default) uses
 * 32-bit buffer offsets whenever every array of a solve is below 2 GiB and
 * 64-bit global addresses otherwise; ME_ADDR_GLOBAL always uses the 64-bit
 * form.  Both visit the entries in the same order, so the results are the
 * same; the option exists to exercise the large-graph form on small graphs. */
enum { ME_ADDR_AUTO = 0, ME_ADDR_GLOBAL = 1 };
/* Storage of the Chebyshev iterates in ME_MIXED (arithmetic stays FP32).
 * ME_ITER_FP32 is the default.  ME_ITER_FP16 stores them in FP16, the
 * residual block scaled per column to unit norm first.  It applies to the
 * embedding solve of a call that is given exactly one input graph (me_embed,
 * me_embed_batch with G = 1) with one-hop entries (ME_CHEB_LAPLACIAN), block
 * width 8 or 16, packed entries and buffer addressing, and falls back to FP32
 * everywhere else: in a batch of two or more graphs (whatever happens to the
 * others: failed, solved densely) and in every server request.  The choice
 * depends only on the call, so a graph's result never depends on the rest of
 * its batch or on the server's load.  It halves the bytes of the iterates but rounds the
 * preconditioner more coarsely, so LOBPCG takes more iterations, how many
 * more depending on the graph: on uniform spheres a few (net gain where the
 * step is bound by HBM bandwidth), on Swiss rolls up to 40% (net loss).  The
 * converged pairs meet the same FP64 residual test either way. */
enum { ME_ITER_FP32 = 0, ME_ITER_FP16 = 1 };
/* How a round of LOBPCG iterations is enqueued: kernel by kernel on the
 * stream (ME_LAUNCH_STREAM), or as a HIP graph of one iteration, captured
 * once per set of active solves on a private stream and replayed
 * (ME_LAUNCH_GRAPH).  ME_LAUNCH_AUTO (default) replays graphs for a solve
 * of one graph of at most 16384 nodes, whose kernels are short enough for
 * launch costs to matter (2000 nodes: 11% faster), and launches kernel by
 * kernel otherwise (a batch re-captures whenever a graph finishes: 5%
 * slower with graphs).  The same kernels with the same arguments run in
 * the same order either way, so results are bitwise identical.  Calls given
 * a caller workspace, and rounds whose kernels are being timed, always
 * launch kernel by kernel. */
enum { ME_LAUNCH_AUTO = 0, ME_LAUNCH_STREAM = 1, ME_LAUNCH_GRAPH = 2 };

/* Precision of the product A W inside each LOBPCG iteration (Section 4.3
 * names the method only).  ME_PRODUCT_FP64 (default): the difference-form
 * product in FP64.  ME_PRODUCT_FP32 (ME_MIXED only): W is rounded to FP32 and
 * multiplied in FP32 (FP32 weights), the result widened to FP64; AX and AP
 * follow from it through the block updates.  X, the Grams, the Rayleigh-Ritz
 * step and the certificate stay FP64, and a result is returned as converged
 * only once the FP64 certificate accepts it.  Kept for measurement, not
 * recommended: the 2000-node square converges (15 iterations against 14),
 * but on the 3000-node Swiss roll the implicitly updated A X drifts away
 * from A X and the solve never converges.  Applies to the embedding solve of
 * me_embed and me_embed_batch; the eps solve keeps FP64 products, and a
 * server rejects the option (ME_ERR_INVALID_ARG). */
enum { ME_PRODUCT_FP64 = 0, ME_PRODUCT_FP32 = 1 };

/* Input graph W (Section 3.1), CSR, device memory, owned by the caller and
 * only read during the call.  rowptr int64[n+1] (rowptr[0] = 0), col int32[nnz]
 * strictly increasing inside each row, val float64[nnz].  Must be symmetric
 * (exactly), with no self loops, all weights finite and > 0, every node with
 * at least one edge. */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int64_t* rowptr;
  const int32_t* col;
  const double* val;
} me_csr;

typedef struct {
  int precision;      /* ME_FP64 (default) or ME_MIXED                              */
  int precond;        /* ME_PRECOND_CHEBYSHEV (default), _JACOBI or _NONE           */
  int max_iter;       /* LOBPCG iteration cap for the embedding solve (default 20000) */
  int eps_max_iter;   /* iteration cap for the eps = lambda_2(Q) solve (default 20000) */
  double eps_tol;     /* relative residual target of the eps solve (default 1e-6;
                         the Rayleigh quotient's error is of order eps_tol^2 times
                         lambda_2 over the gap to the eigenvalues past the block) */
  int check_every;    /* iterations enqueued between host convergence reads (default 16) */
  uint64_t seed;      /* seed of the library's starting blocks (default 0)          */
  int cheb_degree;    /* Chebyshev preconditioner degree, 2..256 (default 128)      */
  int cheb_op;        /* operator the Chebyshev preconditioner inverts in the
                         embedding solve: ME_CHEB_LAPLACIAN (default) or ME_CHEB_FULL */
  int addressing;     /* ME_ADDR_AUTO (default) or ME_ADDR_GLOBAL                     */
  int cheb_iterates;  /* ME_ITER_FP32 (default) or ME_ITER_FP16                        */
  int launch;         /* ME_LAUNCH_AUTO (default), ME_LAUNCH_STREAM or ME_LAUNCH_GRAPH */
  int cholqr_passes;  /* B-orthonormalisations of the preconditioned block per
                         iteration (projection off X, then CholQR): 1 (default)
                         or 2 (CholQR2)                                            */
  int product;        /* ME_PRODUCT_FP64 (default) or ME_PRODUCT_FP32             */
} me_opts;

/* Per-solve report.  Times are host wall-clock milliseconds of the phases. */
typedef struct {
  int status;          /* me_status of the call                                    */
  int iterations;      /* LOBPCG iterations of the embedding solve                 */
  int eps_iterations;  /* LOBPCG iterations of the eps solve (0 if not needed)     */
  int block;           /* internal LOBPCG block width (>= K)                       */
  double eps;          /* lambda_2(Q)                                              */
  double mu;           /* Gershgorin weight of eq. (mu)                            */
  double max_residual; /* max_j |A x_j - l_j B x_j| / (|l_j| |B x_j|), FP64, at exit */
  double orth_error;   /* max |X^T B X - I| at exit, FP64                           */
  double ms_build;     /* graph-operator build incl. eps (0 in me_embed)           */
  double ms_solve;     /* embedding LOBPCG incl. final FP64 pass                   */
} me_info;

/* Opaque graph-operator handle (device-resident T, Q, eps, mu, b, packed A). */
typedef struct me_graph_ops me_graph_ops;

/* Fills `opts` with the defaults listed above.  `opts` host, not null. */
void me_opts_default(me_opts* opts);

/* Text of a status code (static storage). */
const char* me_status_string(int status);

/* Upper bound of the device workspace me_build_graph_ops needs for W
 * (Sections 3.1, 4.1.1, 4.2): W's copy and per-node arrays, the two-hop
 * pattern T and the packed operator, the locality order's scratch and the
 * eps = lambda_2(Q) solve.  nnz(T) is only known after the build, so T is
 * sized by the bound W's degrees give: T_i lies in the union of the
 * neighbourhoods of i's neighbours, so nnz(T) <= sum_k d_k (d_k - 1).
 *   W      host struct of device pointers (see me_csr); only its row
 *          pointers are read (copied to the host).
 *   opts   host, may be NULL.
 *   bytes  host output.
 * Errors: ME_ERR_INVALID_ARG (null arguments, row pointers not starting at 0,
 * not ending at nnz or decreasing).  Synchronises `stream`. */
int me_build_workspace_bytes(const me_csr* W, const me_opts* opts, void* stream, size_t* bytes);

/* Validates W and builds every operator of the generalized problem
 * (Sections 3.1, 4.1.1, 4.2, 4.3): degrees, the two-hop pattern T with
 * counts T_i, Q (with the (i,i) entry of Theta_i equal to 1 so that Q is the
 * Laplacian of the two-hop graph; the printed 1/T_i makes Q indefinite),
 * eps = lambda_2(Q) by LOBPCG on Q with the constant vector deflated (exactly
 * 0 when the two-hop graph is disconnected: ME_WARN_EPS_ZERO), mu, b and the
 * packed difference-form operator A.
 *   W         host struct holding device pointers (see me_csr); read only
 *             during the call (the handle keeps a copy of W).
 *   opts      host, may be NULL (defaults).
 *   ws        device workspace of at least me_build_workspace_bytes bytes, or
 *             NULL.  Given one, the handle's arrays live in it (it must
 *             outlive the handle, and me_graph_ops_destroy frees only the
 *             host part) and the call allocates no device memory; NULL: the
 *             handle owns device memory the library allocates.
 *   ws_bytes  size of ws.
 *   out       host; receives a new handle on success (ME_OK or a warning).
 *   info      host, may be NULL; receives eps, mu, eps_iterations, ms_build.
 * Errors: the validation codes above, ME_ERR_WORKSPACE (ws smaller than the
 * query).  The call synchronises `stream`. */
int me_build_graph_ops(const me_csr* W, const me_opts* opts, void* ws, size_t ws_bytes,
                       void* stream, me_graph_ops** out, me_info* info);

/* Scalars of a built handle (host outputs, any may be NULL). */
int me_graph_ops_query(const me_graph_ops* ops, int64_t* n, int64_t* nnz_T,
                       double* eps, double* mu, int* components_gt1);

/* Bytes of device memory held by the handle. */
size_t me_graph_ops_bytes(const me_graph_ops* ops);

/* Copies the operators out, in the caller's node order (device outputs, each
 * may be NULL): T_rowptr int64[n+1], T_col int32[nnz_T] (sorted per row),
 * T_count int32[n], d float64[n] (degrees), qdiag float64[n] (Q_ii),
 * r float64[n] (Gershgorin radii of A), b float64[n].  Synchronises `stream`. */
int me_graph_ops_export(const me_graph_ops* ops, int64_t* T_rowptr, int32_t* T_col,
                        int32_t* T_count, double* d, double* qdiag, double* r,
                        double* b, void* stream);

/* The node order the solver works in (a locality order; outputs are always
 * in the caller's order): perm[i] = caller's node id of solver row i
 * (device int32[n]).  Cuthill-McKee order: start at the lowest-numbered node
 * on the last breadth-first level of a search from node 0 (a
 * pseudo-peripheral node); level l+1 holds the unvisited neighbours of level
 * l, ordered by the position of their first neighbour in level l, then by
 * node id; further components follow, each started at its lowest-numbered
 * unvisited node.  Graphs of at most 48 nodes keep the identity.  A test and
 * diagnostic hook.  Synchronises. */
int me_graph_ops_order(const me_graph_ops* ops, int32_t* perm, void* stream);

/* Applies the operators to a dense block (device, row-major n x k, 1 <= k <= 16):
 * which = 0: Y = A X;  1: Y = Q X;  2: Y = B X.  FP64, difference form.
 * A test and diagnostic hook; not on the solve path. */
int me_apply(const me_graph_ops* ops, int which, int k, const double* X, double* Y,
             void* stream);

/* Device workspace me_embed needs for this graph and K: the solver's blocks,
 * its tables and work lists (0 for a null handle or K outside 1..16). */
size_t me_embed_workspace_bytes(const me_graph_ops* ops, int K, const me_opts* opts);

/* The first K generalized eigenpairs of (A, B) (Section 4.3) by LOBPCG until
 * every one of the K pairs has relative residual
 *   rho_j = |A x_j - lambda_j B x_j|_2 / (|lambda_j| |B x_j|_2) <= tol
 * evaluated in FP64 at exit.  When |lambda_j| < 1e-8 a_max, with a_max the
 * largest diagonal entry of A (the eps = 0 case has lambda_1 = 0), |lambda_j|
 * in the denominator is replaced by a_max.
 *   K        1..16; the internal block is 4, 8 or 16 columns and must satisfy
 *            3 * block <= n (graphs with n <= 48 use a dense solve instead).
 *   tol      > 0.
 *   X0       device n x K float64 starting block, or NULL to use the
 *            library's seeded counter-based generator (opts->seed).
 *   ws       device workspace of at least me_embed_workspace_bytes bytes, or
 *            NULL to let the library allocate (and free) it on `stream`.
 *            Given one, the call makes no allocation of any kind.
 *   X        device n x K float64 output, row-major, X^T B X = I, columns in
 *            ascending lambda order, each column's largest-magnitude entry
 *            positive (lowest row on ties).
 *   lambda   device float64[K] output, ascending.
 *   info     host, may be NULL.
 * Synchronises `stream`. */
int me_embed(const me_graph_ops* ops, int K, double tol, const me_opts* opts,
             const double* X0, void* ws, size_t ws_bytes, double* X, double* lambda,
             me_info* info, void* stream);

/* Upper bound of the device workspace me_embed_batch needs for these
 * graphs: the sum over graphs of the build (as me_build_workspace_bytes)
 * and of the solver state of both solves, plus the batch's tables and work
 * lists.  Reads every graph's row pointers (copied to the host).
 * Synchronises `stream`. */
int me_embed_batch_workspace_bytes(int G, const me_csr* Ws, const int* Ks, const me_opts* opts,
                                   void* stream, size_t* bytes);

/* Embeds G independent graphs in one solve (the method of Section 4 applied
 * to each graph; a batch is a way to run many of them at once, not a change
 * of the problem).  Every graph is built as me_build_graph_ops does; then
 * all eps = lambda_2(Q) solves run together, then all embedding solves run
 * together: each LOBPCG stage is one launch over every unconverged graph,
 * and the small dense steps run one workgroup per graph.  A graph's result
 * does not depend on the other graphs of the batch (its arithmetic is
 * identical to a batch of one).
 *   Ws       host array of G input graphs (device CSR, as for me_build_graph_ops).
 *   Ks       host int[G], 1..16 each (with the block rule of me_embed).
 *   tol      > 0, the rho target of every graph.
 *   opts     host, may be NULL.
 *   ws       device workspace of at least me_embed_batch_workspace_bytes
 *            bytes (no device allocation is made), or NULL (the library
 *            allocates on `stream` and frees before returning).
 *   ws_bytes size of ws.
 *   Xs       host array of G device pointers, graph g's n_g x K_g output.
 *   lambdas  host array of G device pointers, K_g values each.
 *   infos    host me_info[G], may be NULL; per-graph status and report
 *            (ms_build: time until that graph's operators were ready,
 *            ms_solve: the embedding phase of the whole batch).
 * Returns ME_ERR_WORKSPACE if ws is smaller than the query, else the first
 * negative per-graph status if any graph failed (the other graphs' outputs
 * are still valid, see infos), else the largest warning, else ME_OK.
 * Synchronises `stream`. */
int me_embed_batch(int G, const me_csr* Ws, const int* Ks, double tol, const me_opts* opts,
                   void* ws, size_t ws_bytes, double* const* Xs, double* const* lambdas,
                   me_info* infos, void* stream);

/* ---- Serving: continuous batching of independent requests ---------------
 * A server owns one LOBPCG engine on `stream`.  Each request is a graph and
 * K; requests wait in a FIFO queue until their device footprint (an upper
 * bound of operators plus solver state, from W's degrees as in
 * me_build_workspace_bytes) fits `mem_budget` next to the admitted ones and
 * fewer than `max_active` are admitted.  With a caller workspace the
 * footprint is reserved in it as one range when the request is admitted and
 * returned when it retires, and the server allocates no device memory; a
 * request that cannot fit even in an idle server completes with
 * ME_ERR_WORKSPACE.  An admitted request is built on
 * a second stream of the server (default priority) while the engine's
 * current round runs, solves eps = lambda_2(Q) and then its embedding as
 * engine slots beside all other admitted requests, and is retired when its
 * embedding is certified; its memory then admits the next request.  A
 * request's result does not depend on the other requests: it is bitwise that
 * of a batch of one with the same options and ME_ITER_FP32 (a server always
 * stores the Chebyshev iterates in FP32).  One host thread drives a server. */
typedef struct me_server me_server;
typedef struct {
  size_t mem_budget; /* device bytes for admitted requests; 0 = 60% of free memory at creation
                        (with a workspace: its size, > 0)                               */
  int max_active;    /* requests admitted at once, >= 1 (default 256)                  */
  me_opts opts;      /* solver options of every request                               */
  void* workspace;   /* NULL (default) or a caller-owned device region of mem_budget
                        bytes that holds everything the server puts on the device
                        (a 128th of it, at least 256 KiB, for the solver's work lists);
                        it must outlive the server                                     */
} me_server_opts;

void me_server_opts_default(me_server_opts* so);
/* Creates a server; `so` host, may be NULL (defaults). */
int me_server_create(const me_server_opts* so, void* stream, me_server** out);
/* Device footprint the server charges a request of graph W and K (the range
 * it reserves in a caller region): the build as me_build_workspace_bytes
 * bounds it and both solver slots.  Reads W's row pointers; synchronises
 * `stream`.  A region needs, besides its requests, the server's tables and
 * work-list areas (about a 64th of the region). */
int me_server_request_bytes(const me_csr* W, int K, void* stream, size_t* bytes);
/* Queues a request (no GPU work).  W: host struct of device pointers that
 * must stay valid until the request completes; X (n x K) and lambda (K):
 * device outputs, written when the request completes; K 1..16, tol > 0.
 * *ticket receives the request's id (0, 1, 2, ... in submission order). */
int me_server_submit(me_server* s, const me_csr* W, int K, double tol, double* X,
                     double* lambda, int64_t* ticket);
/* One round: enqueues one batch of LOBPCG iterations for every active
 * solve, admits and builds queued requests while those run, then certifies,
 * retires and backfills.  *in_flight (may be NULL) = requests queued or
 * running.  Returns an error only for a failure of the server itself; a
 * request's own failure is reported by me_server_poll. */
int me_server_step(me_server* s, int* in_flight);
/* Completed requests since the last poll, oldest first: up to `max` tickets
 * and me_info (status, iterations, eps, mu, max_residual, orth_error,
 * ms_build = admission to operators ready, ms_solve = operators ready to
 * completion; host arrays, may be NULL).  *count = entries written. */
int me_server_poll(me_server* s, int64_t* tickets, me_info* infos, int max, int* count);
/* Releases the server and every request it still holds. */
void me_server_destroy(me_server* s);

/* Kernel timing (diagnostic).  me_kernel_timing(kind) starts timing every
 * launch of one kernel kind with HIP events recorded on the launching stream
 * (kind 0 = off, 1 = SpMM of A on the embedding block, 2 = Rayleigh-Ritz
 * Gram of the embedding block, 3 = block combine of the embedding block,
 * 4 = Chebyshev preconditioner step of the embedding solve) and
 * clears the totals.  me_kernel_timing_read returns the number of launches,
 * their summed duration in milliseconds and the algorithmic bytes they moved
 * (host outputs).  Totals are updated when me_embed returns. */
int me_kernel_timing(int kind);
int me_kernel_timing_read(int64_t* launches, double* total_ms, double* bytes);

/* Run-time tuner of the FP32 preconditioner step (diagnostic).  A one-graph
 * solve runs each Chebyshev step either with the workgroup's neighbour rows
 * staged in LDS (form 0) or gathered from L2 (form 1); the two give the same
 * results bit for bit.  The first iteration of a kind of solve not seen
 * before in the process (block width, entry range: 1 = one-hop entries of
 * the embedding solve, 2 = two-hop entries of the eps solve, and
 * floor(log2 rows)) times half its steps in each form and keeps the faster
 * for that kind.  me_step_form returns the kept form of a kind (-1: not
 * timed yet or being timed); me_step_form_reset forgets every choice. */
int me_step_form(int block_width, int range, int64_t rows);
void me_step_form_reset(void);

/* ---- kNN graph of points (the step before the path) --------------------
 * The symmetric weighted graph of Section 5.1's kNN construction (the k
 * nearest neighbours by Euclidean distance) with Gaussian weights:
 *   - d2(i, j) = sum over coordinates, in order, of (x_id - x_jd)^2, each
 *     square a plain product (no fused multiply-add), FP64;
 *   - N_k(i) = the k points j != i of smallest d2(i, j), equal distances
 *     ordered by the smaller j (exact: every pair is evaluated);
 *   - edges: the union, (i, j) when j in N_k(i) or i in N_k(j);
 *   - sigma = median over i of sqrt(d2(i, k-th neighbour)) (the mean of the
 *     two middle values for even n);
 *   - w_ij = exp(-d2(i, j) / (sigma * sigma)), raised to the smallest normal
 *     FP64 number if it underflows.
 * The result is a valid input of me_build_graph_ops (sorted columns,
 * symmetric, no self loops, positive weights, no isolated node).
 *   points  device float64[n * dim], row-major (point i at points + i*dim).
 *   n       2 .. 2^31 - 2;  dim 1..64;  k 1..32 and k < n.
 *   ws      device workspace of at least me_knn_workspace_bytes(n, dim, k)
 *           bytes (no device allocation is made), or NULL.
 *   rowptr  device int64[n + 1] output.
 *   col     device int32 output, capacity 2 n k (nnz <= 2 n k).
 *   val     device float64 output, capacity 2 n k.
 *   nnz     host output: the number of entries written.
 *   sigma   host output (may be NULL).
 * Errors: ME_ERR_INVALID_ARG (null pointers, sizes, a non-finite coordinate,
 * squared distances beyond FP64), ME_ERR_K_RANGE, ME_ERR_BAD_WEIGHT (sigma
 * = 0: the median k-th neighbour distance is 0, so the weights are
 * undefined), ME_ERR_WORKSPACE.  Synchronises `stream`. */
size_t me_knn_workspace_bytes(int64_t n, int dim, int k);
int me_knn_graph(const double* points, int64_t n, int dim, int k, void* ws, size_t ws_bytes,
                 int64_t* rowptr, int32_t* col, double* val, int64_t* nnz, double* sigma,
                 void* stream);

/* ---- Clustering the embedding and scoring it (Section 5.1, Table 3) -------
 * The rows of an embedding X (device float64, n x K row-major, K <= 16) are
 * clustered into C <= 64 clusters (C <= n).
 * me_kmeans: k-means++ seeds from the caller's uniforms u[0..C-1] (host,
 *   each in [0, 1)): seed 0 is point floor(u_0 n); seed t is the first point
 *   whose running sum of D^2 (squared distance to its nearest seed so far)
 *   exceeds u_t times the total.  Then Lloyd iterations: each point joins its
 *   nearest centre (ties to the lower index; squared distances summed over
 *   coordinates in order, plain products), each centre becomes the mean of
 *   its points (an empty cluster keeps its centre), until no point moves or
 *   max_iter updates.  Outputs: labels (device int32[n]), centres (device
 *   float64[C * K]), *iters (host) = centre updates made.
 * me_gmm: EM for a C-component Gaussian mixture with full covariances from
 *   the partition labels0 (device int32[n], values in 0..C-1): weights =
 *   cluster fractions, means = cluster means (the data mean for an empty
 *   one), covariances = within-cluster covariances; every covariance gets
 *   reg I added, reg = 1e-6 times the mean per-coordinate variance of X.
 *   Stops when the log-likelihood changes by at most tol times its
 *   magnitude, or after max_iter steps.  Outputs: labels (most responsible
 *   component, ties to the lower index), weights (device float64[C]),
 *   means (C * K), covs (C * K * K), *loglik and *iters (host).
 *   ME_ERR_BREAKDOWN if a covariance stops being positive definite.
 * me_cluster_scores: Rand index, Precision (pairs), Purity and NMI
 *   (I / sqrt(H_classes H_clusters)) of clusters (device int32[n], values in
 *   0..n_clusters-1) against classes (0..n_classes-1), both counts <= 256:
 *   scores (host float64[4]).
 * Workspace: at least me_cluster_workspace_bytes(n, K, C) bytes (any of the
 * three calls), or NULL.  All three synchronise `stream`. */
size_t me_cluster_workspace_bytes(int64_t n, int K, int C);
int me_kmeans(const double* X, int64_t n, int K, int C, const double* u, int max_iter, void* ws,
              size_t ws_bytes, int32_t* labels, double* centres, int* iters, void* stream);
int me_gmm(const double* X, int64_t n, int K, int C, const int32_t* labels0, int max_iter,
           double tol, void* ws, size_t ws_bytes, int32_t* labels, double* weights, double* means,
           double* covs, double* loglik, int* iters, void* stream);
int me_cluster_scores(const int32_t* classes, const int32_t* clusters, int64_t n, int n_classes,
                      int n_clusters, void* ws, size_t ws_bytes, double* scores, void* stream);

/* ---- Manifold-graph check: betweenness centrality and its variance -------
 * Section 3.3 (eq. (3), Table 1) accepts a graph as a manifold graph when the
 * variance of its nodes' betweenness centralities (VBC) is small:
 *   C_B(i) = sum over ordered pairs (s, t), s != t, s != i, t != i, of
 *            sigma_st(i) / sigma_st,
 * sigma_st the number of shortest paths from s to t (counted in edges: the
 * weights of W do not enter) and sigma_st(i) those through i; pairs in
 * different components add nothing; VBC = (1/n) sum_i (C_B(i) - mean)^2.
 * Path counts are held in FP64 (exact below 2^53).  O(n |E|) work: meant for
 * graphs of up to some 10^5 nodes.
 *   W    host struct of device pointers; rowptr and col are read (val is
 *        not), columns sorted, symmetric, no self loops (isolated nodes are
 *        allowed: their centrality is 0).
 *   ws   device workspace of at least me_betweenness_workspace_bytes(n)
 *        bytes, or NULL.
 *   cb   device float64[n] output.   vbc  host output (may be NULL).
 * Errors: ME_ERR_INVALID_ARG (malformed CSR), ME_ERR_NOT_SYMMETRIC,
 * ME_ERR_WORKSPACE.  Synchronises `stream`. */
size_t me_betweenness_workspace_bytes(int64_t n);
int me_betweenness(const me_csr* W, void* ws, size_t ws_bytes, double* cb, double* vbc,
                   void* stream);

/* ---- Without device allocation ------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * me_embed_noalloc is me_embed whose workspace is a file-scope device array
 * of the library, me_embed_noalloc_max_bytes() bytes (64 MiB) on each
 * device the library runs on, held until the process ends.  The call makes
 * no allocation of any kind.  Arguments, results and errors as me_embed
 * (there is no workspace argument), plus ME_ERR_WORKSPACE, outputs
 * untouched, when me_embed_workspace_bytes for this graph and K exceeds the
 * array: about 880 000 rows x block width (n <= 110 000 at K <= 8).  Calls
 * on one device share the array; the library serialises them (a second call
 * waits until the first has returned), so calls that would overlap on one
 * device do not race. */
size_t me_embed_noalloc_max_bytes(void);
int me_embed_noalloc(const me_graph_ops* ops, int K, double tol, const me_opts* opts,
                     const double* X0, double* X, double* lambda, me_info* info, void* stream);

/* Releases a handle (NULL is allowed). */
void me_graph_ops_destroy(me_graph_ops* ops);

#ifdef __cplusplus
}
#endif
#endif /* MEMBED_H */
