/*
 * ctp.h -- C interface of the compressed-threshold-pivoting supernode library
 * for AMD Instinct MI355X (gfx950).
 *
 * The library factors one dense supernode (Hogg & Scott, "Compressed
 * threshold pivoting for sparse symmetric indefinite systems", arXiv
 * 1305.2353, Section 1, display (1.1)):
 *
 *        A = [ A11 ]   A11: p x p symmetric (lower triangle used)
 *            [ A21 ]   A21: (n-p) x p,   n >= p
 *
 * performing the tasks of Section 1 with the pivot rules of Sections 2-4:
 *
 *   Factor  A11 = L11 D11 L11^T with a symmetric permutation, 1x1 and 2x2
 *           pivots accepted by the threshold tests (2.1)/(2.2); candidates
 *           that fail are delayed;
 *   Solve   L21 = A21 (D11 L11^T)^-1 (on the column-permuted A21);
 *   Form    S = L21 D11 L21^T (the Schur complement the parent subtracts).
 *
 * Conventions shared by every entry point
 * --------------------------------------
 * Memory.  Every array argument is DEVICE memory owned by the caller (for
 *   example torch tensors).  The library never allocates, never
 *   synchronises the host and keeps no state between calls; scratch memory
 *   comes from the caller's workspace (ctp_supernode_noalloc alone uses a
 *   static device array of the library instead).  All work is enqueued on the given
 *   HIP stream; results (including nelim and status) are ready when that
 *   stream reaches them.  Integers stored on the device are int32.
 * Layout.  Matrices are column-major with a leading dimension; the panel
 *   a has n rows and p columns, entry (i, j) at a[i + j*lda], lda >= n.
 * Indices are 0-based.  Positions are final pivot positions.
 * Outputs of the factorization (in place in a):
 *   rows 0..p-1 hold A11 symmetrically permuted; for an eliminated
 *   position k < nelim: a(k,k) = D(k,k); a(k+1,k) = D(k+1,k) when k starts
 *   a 2x2 pivot; every other entry below the diagonal of column k is L(i,k)
 *   (L is unit lower triangular, its unit diagonal and the in-block zero of
 *   a 2x2 pivot are implicit).  Columns k >= nelim hold the delayed block
 *   updated by all eliminations (lower triangle) and the rows L_dE.
 *   Rows p..n-1 (A21) are never permuted: columns k < nelim hold L21 and
 *   columns k >= nelim hold the delayed columns A21_d - L21 D L_dE^T.
 *   The strict upper triangle of rows 0..p-1 is used as working storage by
 *   the pivot search (A11 is held there as a full square) and is
 *   overwritten; its contents on return are unspecified.
 *   perm[k] = original column (0-based) now at position k.
 *   piv[k]  = CTP_PIV_1X1, CTP_PIV_2X2_FIRST / CTP_PIV_2X2_SECOND (the two
 *             positions of a 2x2 pivot), CTP_PIV_ZERO (a column whose
 *             entries were all below `small`: D = 0, L column 0), or
 *             CTP_PIV_DELAYED for k >= nelim.
 *   d[2k] = D(k,k); d[2k+1] = D(k+1,k) if k starts a 2x2 pivot, else 0.
 *   *nelim = number of eliminated positions; p - nelim columns are delayed.
 * Errors.  Return 0 on success.  -k means argument k (1-based) is invalid
 *   (LAPACK convention); CTP_ERR_HIP_BASE - e reports HIP error e from a
 *   launch.  Numerical events are not errors: delays come back in nelim;
 *   the device status word collects CTP_STATUS_* bits.
 */
#ifndef CTP_H
#define CTP_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Pivot rules. */
#define CTP_TPP 0        /* threshold partial pivoting on the whole panel (Section 2) */
#define CTP_STRICT 1     /* compressed, strict C, eq. (4.2), abs update eq. (4.4) (Section 4.1) */
#define CTP_RELAXED 2    /* compressed, relaxed C (Section 4.2) */
#define CTP_RESTRICTED 3 /* pivots tested against A11 only (Section 3.2) */

/* Pivot-type codes (piv[] entries). */
#define CTP_PIV_ZERO 0
#define CTP_PIV_1X1 1
#define CTP_PIV_2X2_FIRST 2
#define CTP_PIV_2X2_SECOND (-2)
#define CTP_PIV_DELAYED (-1)

/* Device status bits. */
#define CTP_STATUS_ZERO_PIVOT 1     /* a zero pivot was recorded */
#define CTP_STATUS_NONFINITE 2      /* a NaN/Inf was read by a pivot test or by the compression */
#define CTP_STATUS_RELAXED_RESCAN 4 /* relaxed C needed a full column rescan (only panels of
                                       more than 16384 A21 rows, and the batched calls, walk
                                       top-8 candidate lists that can run out; a diagnostic
                                       of the search, not of C) */
#define CTP_STATUS_ROOT_FALLBACK 8  /* CTP_FLAG_ROOT: a column was eliminated regardless of u */
#define CTP_STATUS_BAD_MAP 16       /* extend-add: a map or perm entry out of range (entry skipped) */

/* ctp_opts.flags bits. */
#define CTP_FLAG_ROOT 1u   /* last panel of a factorization: eliminate every column
                              (a pass without progress eliminates the column at
                              position nelim regardless of u: 1x1 unless below
                              small, else a 2x2 with the next column if its
                              determinant is safely nonzero, else a zero pivot) */
#define CTP_FLAG_S_TILED 4u /* ctp_supernode and batches: S is stored as the 128 x 128 tiles of
                              its lower triangle, tile t = tm (tm + 1) / 2 + tn (tn <= tm)
                              at s + s_off + t * 16384, each column-major with ld 128
                              (rows past n - p of edge tiles are not written) */
#define CTP_FLAG_ONE_WG 2u /* run the whole pivot search in one workgroup (decide
                              and apply in the same kernel, no per-batch
                              launches); same results, bit for bit */
#define CTP_FLAG_S_SUBTRACT 8u /* batches: the Form subtracts L21 D L21^T from the lower
                              triangle held at s + s_off (ld lds) instead of storing
                              it -- the trailing update of a right-looking
                              factorization; not with CTP_FLAG_S_TILED */

#define CTP_ERR_HIP_BASE (-1000)
#define CTP_ERR_PANEL_TOO_WIDE (-900)  /* dense: delays grew a panel past CTP_MAX_P */
#define CTP_ERR_SCRATCH_TOO_SMALL (-901) /* ctp_supernode_noalloc: the panel needs more
                                            than CTP_NOALLOC_SCRATCH_BYTES of workspace */

/* Device scratch of ctp_supernode_noalloc (bytes, per GPU). */
#define CTP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* Largest p supported by the single-workgroup pivot search and the solve. */
#define CTP_MAX_P 512

typedef struct ctp_opts {
  int method;      /* CTP_TPP, CTP_STRICT, CTP_RELAXED or CTP_RESTRICTED */
  double u;        /* threshold, 0 < u <= 0.5 (Section 2; default 0.01) */
  double small;    /* entries below small count as zero (default 1e-20) */
  int prec;        /* arithmetic of the Solve and the Form: 0 = FP64;
                      1 = FP32 matrix cores; 2 = BF16 matrix-core operands.
                      Both reduced modes accumulate in FP32; the pivot search,
                      the 2x2 inverses and D^-1 stay FP64 (Factor is always
                      FP64).  Supernode: ctp_solve_supernode (and the batched
                      Solve) run the triangular solve with it and leave the
                      reduced-precision operand rows of L21 and W at the end
                      of the workspace; ctp_schur and the fused call form S
                      from those (S stored as FP64; needs work).  The batched
                      Form stays FP64.  Dense factorization: the panels'
                      Solve and the trailing update, on an FP32 trailing
                      matrix. */
  int tile;        /* Form kernel schedule variant (all give the same bits).
                      With a stored W: -1 or 0 = default (operands loaded
                      straight into a ring of four LDS buffers, 8 k per chunk,
                      product taken as S^T = W L21^T so that stores are whole
                      lines); 1 = register-staged, staging at the end of the
                      chunk; 2 = register-staged mid-chunk; 3 = 2 + padded LDS
                      rows; 4 = 3 + split staging rows; 5 = 2 + split staging
                      rows; 6 = LDS ring with the plain product.
                      Batched Form: 0 = default, 1-3 = register-staged.  With
                      work = NULL 1 = two rows per staging thread */
  unsigned flags;  /* CTP_FLAG_* bits, default 0 */
} ctp_opts;

/* Fill *opts with the defaults: relaxed, u = 0.01, small = 1e-20. */
void ctp_default_opts(ctp_opts* opts);

/* Library version string (static storage). */
const char* ctp_version(void);

/* Bytes of device workspace that ctp_factor_supernode / ctp_supernode /
 * ctp_compress need for an n x p panel with opts->method (and, for
 * opts->prec != 0, the reduced-precision operand rows of the Form); written
 * to *bytes.  The same workspace may be reused by later calls on the
 * stream. */
int ctp_workspace_size(int n, int p, const ctp_opts* opts, size_t* bytes);

/* Compression step alone (Section 4, Fig. 4.1 (a)-(b)): builds the p x p
 * compressed matrix of A21 = rows p..n-1 of a.
 *   method CTP_STRICT:  c(j,k) = max |a(i,k)| over the rows i whose largest
 *                       |entry| lies in column j (lowest column on ties),
 *                       0 for an empty set (eq. (4.2)).
 *   method CTP_RELAXED: for j = 0..p-1 in order, row j of C is the signed
 *                       A21 row with the largest |a(i,j)| among rows not yet
 *                       taken (lowest row on ties); zero rows once every
 *                       row is taken.  crow[j] = that A21 row or -1.
 * c: p x p column-major output, ldc >= p.  crow may be NULL for strict.
 * The result is exact (comparisons only).  a is not modified.
 * Requires p <= 2*CTP_MAX_P. */
int ctp_compress(int n, int p, const double* a, int lda, int method,
                 double* c, int ldc, int* crow, int* status,
                 void* work, size_t lwork, hipStream_t stream);

/* Factor task (Section 1) with the pivot search of Section 2 on
 *   TPP:        the whole panel [A11; A21] -- A21 is updated as the search
 *               goes, so on return rows p..n-1 already hold L21 and the
 *               delayed columns (Factor and Solve combined, as in the
 *               paper's TPP kernel);
 *   STRICT /    the 2p x p trapezoid [A11; C] (Fig. 4.1 (b)-(c)); A21 is
 *   RELAXED:    left untouched for ctp_solve_supernode;
 *   RESTRICTED: A11 alone.
 * perm[p], piv[p], d[2p], nelim[1], status[1]: device outputs (status is
 * cleared first).  work: device workspace of lwork >= ctp_workspace_size
 * bytes.  Requires p <= CTP_MAX_P.  The pivot search is enqueued as a fixed
 * sequence of kernels (batches of up to 8 eliminated columns are applied to
 * the trailing matrix by a grid-wide kernel), so the call stays
 * graph-capturable whatever the data. */
int ctp_factor_supernode(int n, int p, double* a, int lda, const ctp_opts* opts,
                         int* perm, int* piv, double* d, int* nelim, int* status,
                         void* work, size_t lwork, hipStream_t stream);

/* Solve task (Section 1; Fig. 4.1 (d)-(e)) after ctp_factor_supernode.
 * Compressed and restricted rules: rows p..n-1 of a are replaced, in place,
 * by L21 = (A21 P^T)_E (D L_EE^T)^-1 in columns 0..nelim-1 and by the
 * delayed columns (A21 P^T)_d - L21 D L_dE^T in columns nelim..p-1.
 * Threshold partial pivoting (CTP_TPP): the factorization already produced
 * L21 and the panel is left as it is.
 * For every rule the call also leaves W = L21 D (n-p rows, nelim columns)
 * in the workspace, the second operand of the Form task (ctp_schur).
 * perm, piv, d, nelim are the device outputs of the factorization.  work:
 * the workspace sized by ctp_workspace_size for the same n, p and method
 * (it also holds the column-permuted A21 while the panel is overwritten).
 * opts->prec 1 / 2: the triangular solve on the FP32 / BF16 matrix cores
 * (FP32 substitution and accumulation, D^-1 and the 2x2 inverses FP64),
 * then L21 and W converted for the reduced-precision Form.
 * Requires p <= CTP_MAX_P. */
int ctp_solve_supernode(int n, int p, double* a, int lda, const int* perm,
                        const int* piv, const double* d, const int* nelim,
                        const ctp_opts* opts, void* work, size_t lwork,
                        hipStream_t stream);

/* Factor, Solve and Form in one call (Section 1's three tasks on one
 * supernode; Fig. 4.1 (a)-(e) for the compressed rules): ctp_factor_supernode,
 * ctp_solve_supernode, then, when s is not NULL, the whole lower triangle of
 * S = L21 D11 L21^T (order n-p) in one launch:
 *   default:          column-major, entry (i, j), j <= i, at s[i + j*lds],
 *                     lds >= n-p; entries above the diagonal are not written;
 *   CTP_FLAG_S_TILED: the packed 128 x 128 tiles of the lower triangle, tile
 *                     (tm, tn), tn <= tm, at s + 16384 (tm (tm+1)/2 + tn),
 *                     column-major with ld 128 (lds ignored; rows and
 *                     columns past n-p of edge tiles are not written).
 * s = NULL: Factor and Solve only.  Arguments otherwise as for
 * ctp_factor_supernode.  Errors: -12 lds too small, -13 workspace too
 * small, others as for the three steps. */
int ctp_supernode(int n, int p, double* a, int lda, const ctp_opts* opts,
                  int* perm, int* piv, double* d, int* nelim, int* status,
                  double* s, int lds, void* work, size_t lwork, hipStream_t stream);

/* ctp_supernode for callers that cannot allocate memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same call without a workspace argument.  The workspace is a static
 * device array of CTP_NOALLOC_SCRATCH_BYTES (64 MiB) inside the library,
 * one copy per GPU, held from the first call on that GPU until the process
 * ends; the call allocates nothing.  Panels whose workspace
 * (ctp_workspace_size) exceeds it are rejected with
 * CTP_ERR_SCRATCH_TOO_SMALL, e.g. about n - p > 14000 at p = 512.  Every
 * call on a GPU uses that GPU's one array, so calls that overlap on the
 * same GPU (concurrent streams, threads) race; calls in one stream order
 * are safe.  The stream must belong to the current device.  No step of the
 * call relies on the array's contents from an earlier call. */
int ctp_supernode_noalloc(int n, int p, double* a, int lda, const ctp_opts* opts,
                          int* perm, int* piv, double* d, int* nelim, int* status,
                          double* s, int lds, hipStream_t stream);

/* Form task (Section 1): rows row0..row0+nrows-1 of the lower triangle of
 * S = L21 D11 L21^T, S of order n-p indexed like the rows of A21.  Entry
 * (i, j), j <= i, is written to s[(i-row0) + j*lds]; s holds nrows rows and
 * row0+nrows columns, lds >= nrows; entries above the diagonal are not
 * written.  a, piv, d, nelim as returned by the factorization (L21 in rows
 * p..n-1, columns 0..nelim-1).
 * work / lwork: either the workspace that ctp_solve_supernode (or
 * ctp_supernode) filled for this panel, unchanged since, with lwork >=
 * ctp_workspace_size; then S = L21 W^T is formed from the stored W = L21 D
 * (the fast path).  Or work = NULL: W is formed from L21, piv and d inside
 * the kernel.  Errors: -14 when work is given and lwork is too small.
 * FP64 matrix-core arithmetic; with opts->prec 1 / 2 the product runs on the
 * FP32 / BF16 matrix cores (FP32 accumulation, S stored as FP64) from the
 * operand rows the reduced-precision Solve left in the workspace (work is
 * then required: -13 without it). */
int ctp_schur(int n, int p, const double* a, int lda, const int* piv, const double* d,
              const int* nelim, int row0, int nrows, double* s, int lds,
              const ctp_opts* opts, const void* work, size_t lwork, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Batches of independent supernodes (one level of a multifrontal tree,
 * Section 1): Factor + Solve (+ Form) of every node in a fixed sequence of
 * launches over the whole batch, with no host synchronization, so the call
 * can be captured in a HIP graph.  Compressed and restricted rules only
 * (opts->method CTP_STRICT / CTP_RELAXED / CTP_RESTRICTED).
 *   1. compression of every A21 (one grid over all nodes);
 *   2. the pivot search of each node in one workgroup (CTP_FLAG_ONE_WG);
 *   3. Solve of every node;
 *   4. Form: one persistent launch whose workgroups take 128 x 128 tiles of
 *      all the nodes' S from a shared counter (opts->tile picks the tile
 *      schedule, as for ctp_schur).
 * ------------------------------------------------------------------------ */

typedef struct ctp_node {
  int n, p;            /* shape: 1 <= p <= CTP_MAX_P, n >= p */
  int lda;             /* panel leading dimension, >= n */
  int lds;             /* S leading dimension, >= n - p (ignored without S or with
                          CTP_FLAG_S_TILED) */
  long long a_off;     /* panel: panels + a_off (doubles), column-major n x p */
  long long s_off;     /* S: s + s_off (doubles), (n-p) x (n-p) lower; -1: no Form */
  long long out_off;   /* perm / piv + out_off (p ints), d + 2*out_off (2p doubles) */
  long long work_off;  /* set by ctp_batch_plan: the node's workspace (bytes) */
  long long tile_off;  /* set by ctp_batch_plan: its first Form tile */
} ctp_node;

typedef struct ctp_batch_info {
  size_t work_bytes;   /* workspace bytes for the batch */
  long long tiles;     /* Form tiles over all nodes with S */
  int count, max_p, max_r, max_chunks;
  int form_workgroups; /* persistent Form workgroups (0: default 512) */
} ctp_batch_info;

/* Host-side plan: checks every node of nodes[count] (host memory), fills
 * work_off and tile_off, and the totals in *info.  The caller then copies
 * the nodes array to the device for ctp_supernode_batched. */
int ctp_batch_plan(int count, ctp_node* nodes, const ctp_opts* opts, ctp_batch_info* info);

/* Factor + Solve (+ Form where s_off >= 0 and s != NULL) of every node.
 * nodes: device copy of the planned array; panels: every node's panel (in
 * place, as ctp_supernode); s: the S buffer (may be NULL); perm, piv, d:
 * outputs at each node's out_off; nelim[count], status[count]: device
 * outputs per node.  work: info->work_bytes bytes.  No host
 * synchronization, no allocation.  The same as the three calls below in
 * order on one workspace. */
int ctp_supernode_batched(int count, const ctp_node* nodes, const ctp_batch_info* info, double* panels,
                          double* s, int* perm, int* piv, double* d, int* nelim, int* status,
                          const ctp_opts* opts, void* work, size_t lwork, hipStream_t stream);

/* The three tasks of a batch one at a time (Section 1: Factor, Solve,
 * Form of every node).  Factor: compression (steps 1-2 above) and pivot
 * search of every node, outputs as for ctp_supernode_batched (status and
 * nelim cleared first).  Solve: L21 and the delayed columns of every node
 * from the factorization's perm, piv, d and nelim, leaving each node's
 * W = L21 D in its part of the workspace.  Form: S of every node with
 * s_off >= 0 (opts->flags CTP_FLAG_S_TILED / CTP_FLAG_S_SUBTRACT as for
 * ctp_supernode_batched) from the panels and the W the Solve left.  The
 * three calls take the same nodes, info and workspace; between them the
 * workspace must not be changed.  Errors as ctp_supernode_batched (-5: a
 * missing perm for the Solve or s for the Form). */
int ctp_factor_supernode_batched(int count, const ctp_node* nodes, const ctp_batch_info* info, double* panels,
                                 int* perm, int* piv, double* d, int* nelim, int* status, const ctp_opts* opts,
                                 void* work, size_t lwork, hipStream_t stream);
int ctp_solve_supernode_batched(int count, const ctp_node* nodes, const ctp_batch_info* info, double* panels,
                                const int* perm, const int* piv, const double* d, const int* nelim,
                                const ctp_opts* opts, void* work, size_t lwork, hipStream_t stream);
int ctp_schur_batched(int count, const ctp_node* nodes, const ctp_batch_info* info, const double* panels,
                      const int* piv, const double* d, const int* nelim, double* s, const ctp_opts* opts,
                      void* work, size_t lwork, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Scatter (Section 1, the fourth task; delayed pivots move to a later
 * supernode): extend-add of a factored front's contribution block into its
 * parent front, for multifrontal chaining of the calls above.
 *
 * The child front has order n and p panel columns; after Factor + Solve its
 * panel (ld lda) holds the delayed block (A11 rows, positions nelim..p-1,
 * lower triangle) and the updated delayed columns (A21 rows), and the
 * caller has formed its boundary block s = A22 - L21 D L21^T (n-p) x (n-p),
 * lower triangle, ld lds: the Form with CTP_FLAG_S_SUBTRACT on the front's
 * own trailing entries (zero when the boundary entries belong to ancestors).
 * The contribution block is the trailing symmetric matrix over positions
 * nelim..n-1.  Position t stands for the child's original local index
 * v = perm[t] (t < p) or t (t >= p); map[v] (n ints, device) is its row in
 * the parent front (order np, panel width pp, 1 <= pp <= np).  Entry
 * (ti, tj), ti >= tj >= nelim, is added into the parent's lower triangle at
 * (R, C) = (max, min)(map[v(ti)], map[v(tj)]): f[C*ldf + R] (the parent's
 * np x pp panel) when C < pp, else f22[(C-pp)*ld22 + (R-pp)] (the parent's
 * trailing (np-pp) x (np-pp) block, the input of its own Form with
 * CTP_FLAG_S_SUBTRACT).  map must be injective on the positions read
 * (entries of eliminated variables are not read); then every parent entry
 * gets at most one add and the result does not depend on the schedule.
 * An out-of-range map or perm entry skips that entry and ORs
 * CTP_STATUS_BAD_MAP into *status (status may be NULL).  nelim and perm are
 * device pointers (the factorization's outputs), so no host
 * synchronization is needed.  Plain FP64 adds.
 * ------------------------------------------------------------------------ */

int ctp_extend_add(int n, int p, const double* a, int lda, const double* s, int lds, const int* perm,
                   const int* nelim, const int* map, int np, int pp, double* f, int ldf, double* f22,
                   int ld22, int* status, hipStream_t stream);

/* One child of a batched extend-add; offsets in doubles (ints for map and
 * perm) into the buffers of ctp_extend_add_batched. */
typedef struct ctp_scatter_task {
  int n, p, lda, lds;    /* child front, as for ctp_extend_add */
  int np, pp, ldf, ld22; /* parent front */
  int node;              /* the child's index into nelim[] */
  long long a_off;       /* child panel: panels + a_off */
  long long s_off;       /* child boundary block: s + s_off; -1 when n == p */
  long long out_off;     /* child perm: perm + out_off */
  long long map_off;     /* map + map_off (n ints) */
  long long f_off;       /* parent panel: fpanels + f_off */
  long long f22_off;     /* parent trailing block: f22 + f22_off; -1 when pp == np */
  long long tile_off;    /* set by ctp_scatter_plan */
} ctp_scatter_task;

/* Host-side plan: checks tasks[count] (host memory), sets tile_off and
 * *tiles (the launch size).  Errors: -(100 + k) for task k. */
int ctp_scatter_plan(int count, ctp_scatter_task* tasks, long long* tiles);

/* Extend-add of every task in one launch (tasks: device copy of the planned
 * array).  No two tasks of one call may write the same parent entry (in a
 * tree: at most one child per parent per call); several calls in stream
 * order chain the children of a parent.  nelim: the child level's per-node
 * outputs, indexed by task.node. */
int ctp_extend_add_batched(int count, const ctp_scatter_task* tasks, long long tiles, const double* panels,
                           const double* s, const int* perm, const int* nelim, const int* map,
                           double* fpanels, double* f22, int* status, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Dense symmetric indefinite LDL^T from supernode panels (Section 1: the
 * Factor / Solve / Form tasks chained right-looking, failed pivots delayed
 * to the next panel, the last panel eliminating every column).
 *
 * Panel = the delayed columns of the previous panel followed by the next pw
 * columns, with every row below them; each is one ctp_supernode call with
 * the rule in opts->method (the last with CTP_FLAG_ROOT), and the trailing
 * matrix receives the Form product, subtracted.  With opts->prec = 1 / 2
 * the trailing matrix is kept in FP32 and updated on the FP32 / BF16 matrix
 * cores; the panels are still factorized in FP64.
 * ------------------------------------------------------------------------ */

/* Workspace bytes for ctp_ldlt_dense / ctp_ldlt_solve / ctp_ldlt_refine
 * with order N, panel width pw (1..CTP_MAX_P), opts->method / prec, and up
 * to nrhs_max right-hand sides (0..16) per solve. */
int ctp_dense_workspace_size(int N, int pw, const ctp_opts* opts, int nrhs_max, size_t* bytes);

/* P A P^T = L D L^T.  a: N x N column-major, lda >= N, device; on entry its
 * lower triangle holds A (the upper triangle is not read).  On exit the
 * lower triangle holds L below the diagonal and D on the diagonal and on
 * the sub-diagonal of each 2x2 block (as for a supernode), and the strict
 * upper triangle holds L^T (with zeros for the 2x2 sub-diagonals), which
 * the solve reads.  perm[N]: A row / column at position i is perm[i];
 * piv[N], d[2N]: pivot types and D as for a supernode.  status: device
 * int, OR of the panels' CTP_STATUS_* bits.  npanels: host int (may be
 * NULL), number of panels.  work: ctp_dense_workspace_size bytes; it also
 * keeps the inverses of L's diagonal blocks for ctp_ldlt_solve, so pass the
 * same workspace, unchanged, to the solve.  The factorization runs on two
 * streams of the library's own (one pair per device, created on first use):
 * the chain of panels, and the trailing updates beyond the next panel, which
 * overlap the next panel's factorization (look-ahead).  They start after
 * the work already on `stream` and
 * `stream` waits for them; the call synchronizes the chain once per panel
 * (panel widths depend on the delays).  Errors:
 * -1..-12 argument k, CTP_ERR_PANEL_TOO_WIDE when delays pile up past
 * CTP_MAX_P, supernode errors passed through. */
int ctp_ldlt_dense(int N, int pw, double* a, int lda, const ctp_opts* opts, int* perm, int* piv,
                   double* d, int* status, int* npanels, void* work, size_t lwork,
                   hipStream_t stream);

/* b <- A^-1 b for nrhs (<= 16) columns, with the factors of ctp_ldlt_dense
 * (a, perm, piv, d and the same workspace; opts and pw as for the
 * factorization).  FP64. */
int ctp_ldlt_solve(int N, int nrhs, const double* a, int lda, const int* perm, const int* piv,
                   const double* d, double* b, int ldb, const ctp_opts* opts, int pw, void* work,
                   size_t lwork, hipStream_t stream);

/* Iterative refinement in FP64 (Section 7 measures accuracy by the
 * backward error): x = solve(b), then x += solve(b - A0 x) until
 *     max_c ||b - A0 x||_inf / (||A0||_inf ||x||_inf + ||b||_inf) <= tol
 * or max_steps corrections.  a0: the original matrix with BOTH triangles
 * (lda0), f / ldf: the factor array of ctp_ldlt_dense; x (N x nrhs, ldx)
 * output.  steps (host, may be NULL): corrections applied; bwd_hist (host,
 * may be NULL, max_steps + 1 entries): backward error before each
 * correction and after the last.  A NaN or an overflow in the residual or
 * the iterate gives an infinite backward error, which ends the refinement
 * (reported as such in bwd_hist, not converged).  Synchronizes once per
 * step. */
int ctp_ldlt_refine(int N, int nrhs, const double* a0, int lda0, const double* f, int ldf,
                    const int* perm, const int* piv, const double* d, const double* b, int ldb,
                    double* x, int ldx, const ctp_opts* opts, int pw, double tol, int max_steps,
                    int* steps, double* bwd_hist, void* work, size_t lwork, hipStream_t stream);

/* Adjoint of x = A^-1 b with the stored factors, pivots frozen (the
 * derivative of the solve; not in the paper).  For symmetric A:
 *     bbar = A^-1 xbar,   Abar = -(1/2) sum_c (bbar_c x_c^T + x_c bbar_c^T).
 * xbar (N x nrhs, ldxb) is overwritten by bbar; abar (N x N, ldg) receives
 * the full symmetric Abar.  a, perm, piv, d, opts, pw, work as for
 * ctp_ldlt_solve; x: the forward solution. */
int ctp_ldlt_adjoint(int N, int nrhs, const double* a, int lda, const int* perm, const int* piv,
                     const double* d, const double* x, int ldx, double* xbar, int ldxb, double* abar,
                     int ldg, const ctp_opts* opts, int pw, void* work, size_t lwork,
                     hipStream_t stream);

/* ------------------------------------------------------------------------
 * Batches of dense systems: count independent symmetric indefinite
 * matrices of order N, system s at a + s * stride (column-major, lda >= N,
 * stride >= lda * N when count > 1), each factorized as ctp_ldlt_dense
 * does (FP64 trailing updates: opts->prec must be 0; rules strict, relaxed
 * or restricted).  Every panel step runs for all systems at once: one
 * ctp_supernode_batched call for the panels with rows below them (the Form
 * subtracted into the trailing matrices, CTP_FLAG_S_SUBTRACT) and one with
 * CTP_FLAG_ROOT for the systems at their last panel, then the per-system
 * bookkeeping; the host reads the nelim of every system back once per
 * step.  Pivots, L and D of each system are those ctp_ldlt_dense computes.
 * ------------------------------------------------------------------------ */

/* Workspace bytes for the three calls below (one workspace serves the
 * factorization and the later solves / adjoints of the same batch). */
int ctp_dense_batched_workspace_size(int count, int N, int pw, const ctp_opts* opts, size_t* bytes);

/* perm, piv: count x N ints (system s at s * N); d: count x 2N doubles;
 * status: count device ints (OR of each system's panel status bits);
 * nsteps: host int (may be NULL), panel steps taken.  Synchronizes the
 * stream once per step.  Errors: -1..-14 argument k,
 * CTP_ERR_PANEL_TOO_WIDE, batched supernode errors passed through. */
int ctp_ldlt_dense_batched(int count, int N, int pw, double* a, int lda, long long stride,
                           const ctp_opts* opts, int* perm, int* piv, double* d, int* status,
                           int* nsteps, void* work, size_t lwork, hipStream_t stream);

/* b <- A^-1 b for every system (nrhs <= 16 columns each; system s's
 * right-hand sides at b + s * bstride, ldb), with the factors and the
 * workspace of ctp_ldlt_dense_batched.  FP64. */
int ctp_ldlt_solve_batched(int count, int N, int nrhs, const double* a, int lda, long long stride,
                           const int* perm, const int* piv, const double* d, double* b, int ldb,
                           long long bstride, const ctp_opts* opts, int pw, void* work, size_t lwork,
                           hipStream_t stream);

/* ctp_ldlt_adjoint for every system: xbar (overwritten by bbar) at
 * xbar + s * xbstride, x at x + s * xstride, Abar (full, symmetric) at
 * abar + s * gstride with ld ldg. */
int ctp_ldlt_adjoint_batched(int count, int N, int nrhs, const double* a, int lda, long long stride,
                             const int* perm, const int* piv, const double* d, const double* x, int ldx,
                             long long xstride, double* xbar, int ldxb, long long xbstride, double* abar,
                             int ldg, long long gstride, const ctp_opts* opts, int pw, void* work,
                             size_t lwork, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* CTP_H */
