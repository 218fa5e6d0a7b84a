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
 *   comes from the caller's workspace.  All work is enqueued on the given
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
#define CTP_STATUS_NONFINITE 2      /* a NaN/Inf reached a pivot test */
#define CTP_STATUS_RELAXED_RESCAN 4 /* relaxed C needed a full column rescan */

#define CTP_ERR_HIP_BASE (-1000)

/* Largest p supported by the single-workgroup pivot search and the solve. */
#define CTP_MAX_P 512

typedef struct ctp_opts {
  int method;      /* CTP_TPP, CTP_STRICT, CTP_RELAXED or CTP_RESTRICTED */
  double u;        /* threshold, 0 < u <= 0.5 (Section 2; default 0.01) */
  double small;    /* entries below small count as zero (default 1e-20) */
  int prec;        /* reserved: 0 = FP64 arithmetic everywhere */
  int tile;        /* Form kernel schedule variant: -1 or 0 = default; with a stored W
                      1 = no LDS padding, 2 = no padding + mid-chunk staging;
                      with work = NULL 1 = two rows per staging thread */
  unsigned flags;  /* reserved, 0 */
} ctp_opts;

/* Fill *opts with the defaults: relaxed, u = 0.01, small = 1e-20. */
void ctp_default_opts(ctp_opts* opts);

/* Library version string (static storage). */
const char* ctp_version(void);

/* Bytes of device workspace that ctp_factor_supernode / ctp_supernode /
 * ctp_compress need for an n x p panel with opts->method; written to
 * *bytes.  The same workspace may be reused by later calls on the stream. */
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
 * Requires p <= CTP_MAX_P. */
int ctp_solve_supernode(int n, int p, double* a, int lda, const int* perm,
                        const int* piv, const double* d, const int* nelim,
                        const ctp_opts* opts, void* work, size_t lwork,
                        hipStream_t stream);

/* Factor + Solve in one call (ctp_factor_supernode then
 * ctp_solve_supernode, for every rule). */
int ctp_supernode(int n, int p, double* a, int lda, const ctp_opts* opts,
                  int* perm, int* piv, double* d, int* nelim, int* status,
                  void* work, size_t lwork, hipStream_t stream);

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
 * FP64 matrix-core arithmetic. */
int ctp_schur(int n, int p, const double* a, int lda, const int* piv, const double* d,
              const int* nelim, int row0, int nrows, double* s, int lds,
              const ctp_opts* opts, const void* work, size_t lwork, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* CTP_H */
