/*
 * tde -- eigenvalues of real symmetric tridiagonal matrices by boundary-row
 * divide and conquer, FP64, on AMD Instinct MI355X (gfx950).
 *
 * Method: Zhan & Zhang, "Reducing Internal State in Eigenvalue-Only
 * Divide-and-Conquer Tridiagonal Eigensolvers".  T (diagonal d, off-diagonal
 * e) is torn recursively into two children plus a rank-one term (Section 3.1,
 * Eq. dc-split); each merge solves the secular equation of
 * diag(D) + rho z z^T with D the children's spectra and z built from the last
 * row of the left child's eigenvector matrix and the first row of the right
 * child's (Eq. merge-problem).  Only those boundary rows are propagated up
 * the tree (Section 3.2, Eq. boundary-state; Algorithm 1), so device memory is
 * linear in n.
 *
 * Conventions for every entry point:
 *  - All array arguments are DEVICE pointers (hipMalloc'd or equivalent) on the
 *    current HIP device, unless stated otherwise.  The caller owns every buffer;
 *    the library never frees caller memory.
 *  - The matrix T of size n has diagonal d[0..n) and off-diagonal e[0..n-1),
 *    e[i] coupling rows i and i+1.  Output eigenvalues are ascending.
 *  - Calls are asynchronous on the given HIP stream (hipStream_t passed as
 *    void*, NULL = default stream).  Argument errors are returned
 *    synchronously (negative codes).  Errors found on the device (non-finite
 *    input, non-convergence) are recorded in a status word inside the
 *    workspace, read back by tde_get_status.
 *  - The first call for a given problem shape (sizes and leaf size) builds and
 *    caches a plan: small device tables describing the merge tree, allocated
 *    once per shape and device.  The first call for a given plan and set of
 *    buffers (d, e, lambda, workspace) also captures the whole solve into a
 *    HIP graph on an internal stream; later calls with the same plan and
 *    buffers replay it with one hipGraphLaunch on the caller's stream and
 *    allocate nothing.  TDE_FLAG_NO_GRAPH, or timing mode, enqueues the
 *    kernels one by one instead.  Both caches are bounded (32 plans, 64
 *    graphs, least recently used out): a graph is destroyed only after its
 *    last launch has completed, a plan's tables only after the device is
 *    idle; tde_release_plans empties them.  The caches are guarded by one
 *    lock held for the duration of each call.
 *  - Inputs and outputs must not overlap.  Concurrent calls on different
 *    streams need distinct workspaces.
 *  - No exceptions cross this interface and nothing is printed.
 */
#ifndef TDE_H
#define TDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes (LAPACK-like: < 0 bad argument or runtime failure, > 0 numerical). */
#define TDE_OK 0
#define TDE_EINVAL (-1)     /* bad argument (size, pointer, offsets, option, workspace too small) */
#define TDE_ENOMEM (-2)     /* plan tables could not be allocated */
#define TDE_EDEVICE (-3)    /* HIP runtime error while enqueuing */
#define TDE_ENONFINITE (-4) /* device status: NaN or Inf in d or e */
#define TDE_ENOCONV 1       /* device status: a leaf QL or secular iteration hit its cap */

/* Options.  Pass NULL for defaults. */
#define TDE_FLAG_NO_GRAPH 1 /* enqueue every kernel eagerly instead of replaying a captured graph */
#define TDE_FLAG_LEAF_DC 2  /* forward passes (tde_eigvals, tde_eigvals_batched, tde_eigvals_rows) solve
                               each leaf by running its own divide-and-conquer tree (halving down to
                               single columns) inside one 64-lane wave instead of by QL; the
                               checkpointing forward of reverse mode always uses QL leaves */
typedef struct {
    int leaf;       /* largest leaf size of the merge tree, 1..64; 0 = default (8) */
    int flags;      /* TDE_FLAG_* bits; other bits are rejected */
    int sweep_cols; /* target poles per lane in the root-parallel sweeps: each root
                       gets G = min(16, 2^ceil(log2(largest merge / sweep_cols)))
                       lanes; 0 = default (8) */
    int wide_min;   /* merges with at least this many active (non-deflated) roots
                       solve them with the wide sweep (64 roots per workgroup, the
                       poles split over 4 waves); >= 2, 0 = default (1024) */
    int max_sweeps; /* secular iterations allowed per root, 1..96; 0 = default (96).
                       A root still unconverged at the cap sets TDE_ENOCONV (a
                       small cap forces that path from the host, for tests) */
    int group_max;  /* most lanes per root (4, 8 or 16) in the merges with at most
                       512 active roots, which run one workgroup per merge; 0 = by
                       level (16 on levels of fewer than 1024 merges, else 4).  The
                       sums are formed in one fixed order whatever the lane count,
                       so this changes speed, not results */
    int wide_blocks; /* most workgroups of each wide-sweep launch, 0..2^20; 0 = default
                       (4096).  Those launches loop over their 64-root items;
                       fewer blocks cost less where they find no work, more keep
                       more waves per compute unit where they carry the solve */
    int fuse_few;   /* on levels of fewer than 1024 merges, the most active roots a
                       merge may have for one workgroup to solve it, 2..512; 0 =
                       default (512).  The larger merges of those levels go to the
                       root-parallel kernels (the wide sweeps from wide_min on),
                       which spread a merge's roots over many workgroups */
    int reserved[1]; /* must be 0 */
} tde_opts;

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int tde_version(void);

/* Bytes of device workspace needed to solve B problems with n_total columns in
 * total (n_total = n for a single problem).  Linear in n_total (about 285 bytes
 * per column).  Returns 0 on a bad argument. */
size_t tde_workspace_bytes(int64_t n_total, int64_t batch, const tde_opts* opts);

/* All eigenvalues of one n x n symmetric tridiagonal T.
 *   d      [n]     diagonal (device, read only)
 *   e      [n-1]   off-diagonal (device, read only; may be NULL when n <= 1)
 *   n      >= 0; n == 0 is a no-op
 *   lambda [n]     output eigenvalues, ascending (device)
 *   ws     workspace of ws_bytes >= tde_workspace_bytes(n, 1, opts) (device)
 * Returns TDE_OK or a negative code; device-side failures via tde_get_status. */
int tde_eigvals(const double* d, const double* e, int64_t n, double* lambda, void* ws, size_t ws_bytes,
                void* hip_stream, const tde_opts* opts);

/* All eigenvalues of B independent tridiagonals packed back to back.
 *   offsets [B+1]  HOST array, offsets[0] = 0, nondecreasing; problem b owns
 *                  d[offsets[b] .. offsets[b+1]) and e over the same range
 *                  (its last slot, offsets[b+1]-1, is ignored).
 *   lambda  [offsets[B]] output, ascending within each problem.
 * Every merge of one tree height, across all problems, runs in the same
 * launches (level-aligned schedule). */
int tde_eigvals_batched(const double* d, const double* e, const int64_t* offsets, int64_t B, double* lambda,
                        void* ws, size_t ws_bytes, void* hip_stream, const tde_opts* opts);

/* Driver pre-pass: split at negligible couplings, then solve the blocks.
 *
 * The outer structure of a tridiagonal eigensolver driver (the paper's CPU
 * driver validates, splits at negligible off-diagonal entries and scales each
 * unreduced block before the D&C, Section 4.2): every coupling with
 * |e_i| <= eps sqrt|d_i| sqrt|d_(i+1)| is dropped (no eigenvalue moves by more
 * than eps ||T||), each resulting block is solved as a problem of its own
 * (own power-of-two scale, own merge tree, all blocks of all problems in the
 * level-aligned batched schedule), and the blocks' ascending spectra are
 * merged back into each problem's ascending output.  Reducible and graded
 * matrices become many small problems.
 *   d, e, offsets, B, lambda: as tde_eigvals_batched (offsets = {0, n} for one
 *                   problem; e of a single problem needs only n-1 entries)
 *   ws            workspace of ws_bytes >= tde_workspace_bytes(offsets[B],
 *                   offsets[B], opts) (room for every column being a block)
 *   nblocks       HOST, may be NULL: receives the number of blocks solved
 * Unlike the other entry points this one waits for the stream once (the block
 * boundaries are read back to plan the solve); the rest is asynchronous. */
int tde_eigvals_split(const double* d, const double* e, const int64_t* offsets, int64_t B, double* lambda,
                      void* ws, size_t ws_bytes, void* hip_stream, const tde_opts* opts, int64_t* nblocks);

/* Eigenvalues and the first and last rows of the eigenvector matrix.
 *
 * The paper propagates only rows 0 and n-1 of each node's eigenvector matrix
 * up the tree (Section 3.2) and skips them at the top merge (root-only mode,
 * Section 3.3).  This entry point keeps them at the top as well (Algorithm 1
 * with the requested rows sigma = {first, last} at the root), so for every
 * output eigenvalue lambda_k it also returns q_0k and q_(n-1)k, the first and
 * last components of its unit eigenvector.  With q_0k, the Golub-Welsch
 * Gauss-quadrature weights of a Jacobi matrix are mu_0 q_0k^2.
 *   offsets, B, d, e, lambda, ws: as tde_eigvals_batched (offsets = {0, n} for
 *                   one problem)
 *   qfirst [offsets[B]]  output q_0k per eigenvalue (device), or NULL
 *   qlast  [offsets[B]]  output q_(n-1)k per eigenvalue (device), or NULL
 *                   (at least one of the two must be given)
 * Each pair is signed so that q_0k >= 0 (q_(n-1)k >= 0 when q_0k = 0). */
int tde_eigvals_rows(const double* d, const double* e, const int64_t* offsets, int64_t B, double* lambda,
                     double* qfirst, double* qlast, void* ws, size_t ws_bytes, void* hip_stream,
                     const tde_opts* opts);

/* Requested eigenvector rows: Algorithm 1 with an arbitrary row list.
 *
 * The paper's recursion takes at every node a list sigma_v of requested local
 * rows and returns the node's eigenvalues with those rows of its eigenvector
 * matrix: the requested rows of Q_v = (Q_L (+) Q_R) S_v are the requested rows
 * of the children's matrices times S_v (Lemma 2, selected-row
 * multiplication), and repeated or unordered requests are resolved by
 * metadata (the text after Algorithm 1).  For one tridiagonal this returns
 * every eigenvalue and the rows `rows` of the eigenvector matrix:
 *   rows   [m]    HOST row indices in [0, n), any order, repeats allowed (m >= 0)
 *   lambda [n]    output eigenvalues, ascending (device)
 *   Q      [m*n]  output (device, row-major): Q[i*n + k] = q_(rows[i]),k, the
 *                 rows[i]-th component of the unit eigenvector of lambda_k, each
 *                 column signed so that q_0k >= 0 (q_(n-1)k >= 0 when q_0k = 0),
 *                 the convention of tde_eigvals_rows; may be NULL when m = 0
 *   ws     ws_bytes >= tde_selrows_workspace_bytes(n, m, opts) (device): the
 *                 forward workspace, a checkpoint of the nodes' spectra and
 *                 boundary rows per tree level, and 5 n doubles + m ints
 * Leaves are solved by QL (TDE_FLAG_LEAF_DC is ignored).  One forward solve
 * records every level's node spectra and boundary rows; then each pair of
 * distinct requested rows takes one more pass up the same tree, riding in
 * the two row channels the boundary rows use (deflation decisions and roots
 * are those of the first pass, bit for bit), so the cost is about
 * 1 + ceil(distinct rows / 2) forward solves.  Kernels are enqueued one by
 * one (no graph); the call waits for the stream once at the end.  Returns
 * TDE_OK or a negative code (TDE_EINVAL for a row outside [0, n)); device
 * status via tde_get_status(ws).  tde_selrows_workspace_bytes returns 0 on a
 * bad argument. */
size_t tde_selrows_workspace_bytes(int64_t n, int64_t m, const tde_opts* opts);
int tde_eigvals_selrows(const double* d, const double* e, int64_t n, const int64_t* rows, int64_t m,
                        double* lambda, double* Q, void* ws, size_t ws_bytes, void* hip_stream,
                        const tde_opts* opts);

/* Dense front end: eigenvalues of a dense real symmetric matrix.
 *
 * Dense symmetric EVD first reduces A to a tridiagonal T = Q^T A Q by
 * orthogonal transformations, whose eigenvalues are those of A, and then
 * solves T (Section 2.1); for eigenvalues only Q is not kept.  This entry
 * point reduces A on the device (blocked Householder reflectors in panels of
 * 32 columns: per column a reflector and the product of the trailing matrix
 * with it, per panel one rank-64 update of the trailing matrix on the FP64
 * matrix cores) and solves T by boundary-row divide and conquer.
 *   A      [lda*n]  device, column-major, the whole symmetric matrix (both
 *                   triangles, which must agree); destroyed: the reduction
 *                   updates its trailing blocks in place
 *   lda    >= n
 *   lambda [n]      output eigenvalues of A, ascending (device)
 *   d_out  [n], e_out [n-1]  device, may be NULL: the diagonal and subdiagonal of T
 *   ws     ws_bytes >= tde_dense_workspace_bytes(n, opts) (device): the
 *                   solver's workspace (first, so tde_get_status(ws) reads its
 *                   status), then 64 n + 3 n + 32 doubles of reduction scratch
 * Asynchronous on the stream; the reduction's kernels are enqueued one by
 * one (three per column, one per panel).  Returns TDE_OK or a negative code.
 * tde_dense_workspace_bytes returns 0 on a bad argument. */
size_t tde_dense_workspace_bytes(int64_t n, const tde_opts* opts);
int tde_dense_eigvals(double* A, int64_t n, int64_t lda, double* lambda, double* d_out, double* e_out, void* ws,
                      size_t ws_bytes, void* hip_stream, const tde_opts* opts);

/* Reverse mode (gradients of the eigenvalues).
 *
 * The paper computes eigenvalues only; these entry points add the adjoint of
 * the same computation: for a loss L = sum_k g_k lambda_k they return
 * dL/dd and dL/de, i.e. g_d[i] = sum_k g_k q_ik^2 and
 * g_e[i] = 2 sum_k g_k q_ik q_(i+1)k for the unit eigenvectors q_k of T
 * (ascending order), without forming any eigenvector.  The pass runs the
 * merge tree top-down: per merge, the implicit-function derivatives of the
 * secular roots f(lambda) = 1 + rho sum_j z_j^2/(D_j - lambda) = 0 and of the
 * boundary rows (Section 3.2) with respect to the poles, z, rho and the
 * children's rows; the deflation rotations and the couplings deflation drops;
 * the leaves' eigenproblems; and the tear (Section 3.1).
 *
 * Problems are given as in tde_eigvals_batched (HOST offsets[B+1]; a single
 * problem is offsets = {0, n}).  Both calls must use the same d, e, offsets and
 * options (leaf, sweep_cols), since the checkpoint is tied to the plan.
 *
 * tde_checkpoint_bytes: device bytes of the checkpoint, about 36 bytes per
 * column per tree level (ceil(log2(n / leaf)) levels).  0 on a bad argument.
 * tde_backward_workspace_bytes: workspace of tde_eigvals_backward (about 545
 * bytes per column), a superset of the forward's.  0 on a bad argument.
 *
 * tde_eigvals_ckpt: as tde_eigvals_batched, and also records in ckpt
 *   [ckpt_bytes] (device, caller-owned) what the reverse pass needs: per tree
 *   level the children's spectra and boundary rows read by its merges and the
 *   secular roots in their (origin pole, offset) form.  ws as for the forward.
 * tde_eigvals_backward:
 *   glambda [offsets[B]]  dL/dlambda for each output eigenvalue (device, read only)
 *   ckpt                  written by tde_eigvals_ckpt on the same inputs; not modified
 *   gd      [offsets[B]]  output dL/dd (device)
 *   ge      [offsets[B]]  output dL/de, same layout as e in the batched form; the
 *                         slot offsets[b+1]-1 of every problem is set to 0
 *   ws      ws_bytes >= tde_backward_workspace_bytes(...) (device)
 * Returns TDE_OK or a negative code; device status via tde_get_status(ws).
 * Gradients of eigenvalues that are (numerically) multiple are not unique: a
 * loss that weights such a cluster unevenly has no well-defined gradient. */
size_t tde_checkpoint_bytes(const int64_t* offsets, int64_t B, const tde_opts* opts);
size_t tde_backward_workspace_bytes(int64_t n_total, int64_t batch, const tde_opts* opts);
int tde_eigvals_ckpt(const double* d, const double* e, const int64_t* offsets, int64_t B, double* lambda,
                     void* ckpt, size_t ckpt_bytes, void* ws, size_t ws_bytes, void* hip_stream,
                     const tde_opts* opts);
int tde_eigvals_backward(const double* d, const double* e, const int64_t* offsets, int64_t B,
                         const double* glambda, const void* ckpt, size_t ckpt_bytes, double* gd, double* ge,
                         void* ws, size_t ws_bytes, void* hip_stream, const tde_opts* opts);

/* Allocation-free solve, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  As tde_eigvals for one tridiagonal of n <= 65536 columns, but
 * without a workspace argument: the workspace and the merge-tree tables live
 * in a fixed 24 MiB device array inside the library, one per GPU, held until
 * the process ends.  The call copies the tree tables into it with
 * asynchronous host-to-device copies on the stream and enqueues the kernels
 * one by one (no graph); it calls no hipMalloc or hipFree and allocates no
 * other device memory (host-side plans are cached, bounded).
 *   d, e, n, lambda, hip_stream, opts: as tde_eigvals (TDE_FLAG_NO_GRAPH is
 *            implied; timing mode does not apply)
 *   status   (device int, may be NULL) receives the solve's status bits in
 *            stream order: 0 ok, 1 non-finite input, 2 or 4 a leaf or secular
 *            iteration hit its cap
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents: calls on one stream are ordered, calls that overlap on one GPU
 * (two streams or threads at once) race.  Returns TDE_EINVAL for n > 65536 or
 * a bad argument, TDE_EDEVICE if the array's address cannot be looked up. */
int tde_eigvals_noalloc(const double* d, const double* e, int64_t n, double* lambda, int* status,
                        void* hip_stream, const tde_opts* opts);

/* Waits for the stream, then reads the device status word of the last solve
 * that used ws: TDE_OK, TDE_ENONFINITE or TDE_ENOCONV.  Returns a negative code
 * if the read itself fails. */
int tde_get_status(const void* ws, void* hip_stream);

/* Measurement aids (not needed to solve).
 *
 * tde_get_counters: waits for the stream, then copies n (<= 20) counters of the
 * algorithmic work of the last solve that used ws:
 *   [0] pole-term evaluations in secular sweeps, [1] (pole, root) pairs in the
 *   Loewner products, [2] (root, pole) pairs in the boundary-row dot products,
 *   [3] secular roots, [4] secular sweeps, [5] columns solved by leaves,
 *   [6] plane rotations applied by QL leaves, [7] columns passed through
 *   merges (summed over tree levels, in-wave leaf merges included);
 *   [8..11] as [0..3] for the merges run inside leaves solved by divide and
 *   conquer in one wave (TDE_FLAG_LEAF_DC), which [0..4] do not include;
 *   [12..15] the part of [0..3] done by the fused kernel for merges with at
 *   most 512 active roots (one workgroup per merge; terms, Loewner pairs, row
 *   pairs, roots); [16..19] the same for the workgroups that run whole merges
 *   of levels of small merges.
 *
 * tde_timing_enable(1): from then on every launch the library enqueues is
 * bracketed by two HIP events recorded on the caller's stream (this adds
 * host work per launch; leave it off when timing whole solves).
 * tde_timing_read: waits for the recorded events and returns, per launch kind
 * (0 setup, 1 leaves, 2 merge/sort, 3 deflation and compaction, 4 secular
 * roots, 5 Loewner products, 6 boundary rows, 7 assembly, 8 reverse pass,
 * 9 fused roots + Loewner + rows of merges with few active roots, 10 whole
 * merges of levels of small merges), the summed
 * milliseconds and launch count since the last read; then forgets them. */
int tde_get_counters(const void* ws, void* hip_stream, uint64_t* out, int n);
int tde_timing_enable(int on);
int tde_timing_read(double* ms, int64_t* launches, int nkinds);

/* Frees every cached plan (device tables), captured graph and split
 * schedule, after waiting for the launches that may still use them. */
void tde_release_plans(void);

/* Current sizes of the library's caches: out[0] plans, out[1] captured graphs,
 * out[2] split merge schedules (the first n of them).  TDE_OK or TDE_EINVAL. */
int tde_cache_sizes(int64_t* out, int n);

/* Human-readable name of a status code (static string). */
const char* tde_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* TDE_H */
