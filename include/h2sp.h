/*
 * h2sp — non-extensive sparsification A = U S V^T of an H^2 matrix on MI355X.
 *
 * C ABI of the library libh2sp.so.  Every function is extern "C", never throws
 * and returns an int status (H2_OK = 0, negative on failure); the message of the
 * last failure on the calling thread is h2_last_error().  Handles own all their
 * memory (host and device) and release it in h2_*_destroy; callers own every
 * buffer they pass in.  All device work is ordered on the stream given to
 * h2_set_stream (default: the null stream of the current HIP device).
 *
 * Method (Sushnikova & Oseledets, "Simple non-extensive sparsification of the
 * hierarchical matrices"):
 *   - the H^2 matrix is Definition 4.9: close part + sum over the interaction
 *     lists of R_t D_ts E_s^T with nested cluster bases (Section 4.1);
 *   - Section 2 (eqs. usv, fin, main_fact) and Section 4 (4.2, 4.3) turn it into
 *     A = U S V^T, S sparse of the same size, U and V orthogonal products of
 *     block-diagonal and permutation matrices;
 *   - A x = b is solved as S y = U^T b, x = V y (eq. sp0).
 * The kernel is symmetric and rows and columns share one cluster tree, so
 * U = V (Proposition 2.1) and S is stored as its upper block triangle.
 */
#ifndef H2SP_H
#define H2SP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------- */
enum {
  H2_OK = 0,
  H2_EINVAL = -1,       /* bad argument (sizes, NaN or duplicate points, ...)        */
  H2_ENOMEM = -2,       /* host or device allocation failed                         */
  H2_EDEVICE = -3,      /* a HIP call failed                                        */
  H2_ESINGULAR = -4,    /* a pivot block of S is numerically singular               */
  H2_ENOCONV = -5,      /* refinement stopped above the tolerance (x still written) */
  H2_EUNSUPPORTED = -6  /* option outside what the library supports                */
};

/* ---- options --------------------------------------------------------------- */
enum { H2_KERNEL_INVDIST = 0,   /* A_ij = scale / |x_i - x_j| (i != j), A_ii = diag */
       H2_KERNEL_EXP = 1,       /* A_ij = scale exp(-|x_i - x_j|^2) (i != j), A_ii =
                                   diag: Example 5.2 of Section 5.1 (its matrix
                                   2 delta_ij + exp(-|r_i - r_j|^2) is scale 1,
                                   diag 3).                                    */
       H2_KERNEL_IFMM = 2 };    /* A_ij = scale r / d for 0 < r < d and scale d / r
                                   for r >= d, r = |x_i - x_j|, d = param > 0,
                                   A_ii = diag: Example 5.4 of Section 5.5 (scale
                                   1, diag 1).  h2_sparsify_batch takes matrices
                                   of one kernel kind and parameter
                                   (H2_EUNSUPPORTED otherwise).                */
enum { H2_FP64 = 0,             /* every step in FP64                                */
       H2_MIXED = 1 };          /* transforms, S and its factor in FP32 (MFMA), basis
                                   QR, pivot-block inversion and residuals in FP64   */

typedef struct {
  int kind;      /* H2_KERNEL_INVDIST, H2_KERNEL_EXP or H2_KERNEL_IFMM          */
  double scale;  /* c in c / |x - y|, c exp(-|x - y|^2), c r / d or c d / r     */
  double diag;   /* value of A_ii                                               */
  double param;  /* d of H2_KERNEL_IFMM (> 0); ignored by the other kinds       */
} h2_kernel;

typedef struct {
  int leaf;              /* max points per leaf cluster, 2..128                 */
  int cheb;              /* Chebyshev nodes per axis, 2..4 (p^dim <= 64)         */
  double recompress_tol; /* 0: keep the Chebyshev bases; else relative SVD cut   */
  int rank_cap;          /* upper bound of the recompressed ranks (<= p^dim)     */
  double eta;            /* admissibility: dist >= eta * max diam; 0 = weak      */
} h2_build_opts;

typedef struct {
  int precision;         /* H2_FP64 or H2_MIXED                                  */
} h2_sparsify_opts;

enum { H2_FACTOR_EXACT = 0,     /* block LU of S with its fill (exact up to rounding) */
       H2_FACTOR_ILU0 = 1,      /* block ILU(0): S's own pattern, no fill (default)  */
       H2_FACTOR_ILUT = 2 };    /* block threshold ILU with drop tolerance tau (the
                                   ILUt of Section 5.5, read for a symmetric S):
                                   over the fill of the exact mode, a fill block
                                   (i, j) above the diagonal is set to zero once
                                   row i is finished if its Frobenius norm is below
                                   tau times that of block row i of S (both
                                   triangles, as given); its mirror below the
                                   diagonal goes with it.  tau = 0 is the exact
                                   factor, tau = inf block ILU(0)                   */

typedef struct {
  int mode;              /* H2_FACTOR_EXACT, H2_FACTOR_ILU0 or H2_FACTOR_ILUT    */
  double tau;            /* drop tolerance of H2_FACTOR_ILUT (>= 0, inf allowed)  */
} h2_factor_opts;

enum { H2_SOLVE_AUTO = 0,       /* iterative refinement; when its contraction stalls
                                   (residual ratio above 0.9 for 3 steps) or it
                                   diverges (ratio above 2, or not finite), the
                                   best x so far is kept and flexible GMRES
                                   continues from it (GMRES-based refinement)   */
       H2_SOLVE_REFINE = 1,     /* iterative refinement only                       */
       H2_SOLVE_GMRES = 2 };    /* flexible GMRES from the start (Section 5.5 uses
                                   the factor of S as a GMRES preconditioner)     */

typedef struct {
  double tol;            /* stop when max_col ||b - A x||_2 / ||b||_2 <= tol     */
  int max_iter;          /* preconditioner applications in all (refinement
                            steps plus GMRES steps), >= 1                        */
  int method;            /* H2_SOLVE_AUTO, H2_SOLVE_REFINE or H2_SOLVE_GMRES      */
  int restart;           /* GMRES restart length, 1..64 (0: 30)                  */
} h2_solve_opts;

typedef struct {
  int iters;                   /* preconditioner applications (refinement steps
                                  plus GMRES steps)                              */
  double max_rel_residual;     /* final max_col ||b - A_H2 x|| / ||b||            */
  double seconds[3];           /* device s of the preconditioner applications
                                  (U^T, triangular solves, V), of the FP64 H^2
                                  matvecs, and host s building the plans       */
  int gmres_steps;             /* of iters, the steps taken by GMRES             */
  int refine_steps;            /* of iters, the refinement steps                 */
} h2_solve_info;

typedef struct h2_matrix h2_matrix;   /* tree, block tree, H^2 coefficients       */
typedef struct h2_sparse h2_sparse;   /* Q_t of every cluster, S, plan            */
typedef struct h2_factor h2_factor;   /* block L D L^T of S (exact or ILU(0))      */

/* ---- library state --------------------------------------------------------- */
const char* h2_last_error(void);
/* All later device work of this thread goes to `stream` (a hipStream_t). */
int h2_set_stream(void* stream);

/* ---- construction of the H^2 matrix (Section 4.1: the input of the method) -- */
/*
 * h2_build: points `pts` (HOST, row-major n x dim, dim 2 or 3, finite, pairwise
 * distinct) -> kd cluster tree (longest axis of the tight box, median split,
 * equal-depth leaves), block cluster tree (Definitions 4.2-4.4), tensor
 * Chebyshev bases, transfers and couplings, optionally recompressed.  Host
 * work only; the coefficients go to the current device on first device use
 * (h2_matvec, h2_sparsify).  EINVAL on bad
 * sizes, NaN / infinite or duplicate points; ENOMEM / EDEVICE on allocation.
 */
int h2_build(const double* pts, int64_t n, int dim, const h2_kernel* kernel,
             const h2_build_opts* opts, h2_matrix** out);

/*
 * h2_import: same tree and block tree as h2_build (derived from the points),
 * but the coefficients of the H^2 format (cluster bases R_t with their
 * transfer matrices, couplings D_b; Definitions 4.7 and 4.9) come from the
 * caller (HOST arrays):
 *   rank[ncl]            r_t per cluster in heap order (0 for clusters without
 *                        a basis, i.e. without farfield of their own or of an
 *                        ancestor; must match that set exactly)
 *   nodes[ncl * P * dim] Chebyshev nodes of each cluster (rows of P x dim,
 *                        row-major); read only for clusters with r_t > 0
 *   proj                 concatenation over clusters with r_t > 0 (heap order)
 *                        of P_t, r_t x P column-major: coupling D_ts =
 *                        P_t K(nodes_t, nodes_s) P_s^T
 *   leaf_basis           concatenation over leaves with r_t > 0 of R_t,
 *                        |t| x r_t column-major, rows in tree order
 *   transfer             concatenation over non-root clusters c whose father
 *                        has r > 0 (heap order) of T_c, r_c x r_father
 *                        column-major
 * P = cheb^dim.  The opts fields recompress_tol and rank_cap are ignored.
 */
int h2_import(const double* pts, int64_t n, int dim, const h2_kernel* kernel,
              const h2_build_opts* opts, const int32_t* rank, const double* nodes,
              const double* proj, const double* leaf_basis, const double* transfer,
              h2_matrix** out);

/* Sizes of the tree: depth L (leaves on level 0), cluster count 2^(L+1)-1. */
int h2_matrix_info(const h2_matrix* h, int* depth, int64_t* ncl, int* cheb_points);
/* HOST copies: perm[n] (tree position -> original index), rank[ncl]. */
int h2_matrix_export_tree(const h2_matrix* h, int64_t* perm, int32_t* rank);

/*
 * h2_matvec: y = A_H2 x in FP64 on the device (close part from the kernel
 * blocks of the near leaf pairs, far part by the nested bases; Definition 4.9).
 * The first product for a right-hand-side count builds a plan kept with the
 * matrix; it writes the close blocks out once when they take at most a quarter
 * of the free device memory (H2SP_CLOSE_RESIDENT=0: never), else every product
 * evaluates them from the points.  x, y: DEVICE pointers, column-major
 * n x nrhs with leading dimension ld >= n, ORIGINAL point order; nrhs <= 512.
 */
int h2_matvec(const h2_matrix* h, const double* x, double* y, int64_t nrhs, int64_t ld);

/* ---- sparsification (Section 2, Algorithm 1 as realised in Section 4) ------- */
/*
 * h2_sparsify: level sweep from the leaves to the root: batched Householder QR
 * completing every cluster basis to a square orthogonal Q_t (FP64), two-sided
 * transforms of the close blocks, couplings moved into the father's close
 * block, strips of finalised rows, S assembled as a block-sparse matrix of the
 * size of A.  The handle keeps a reference to `h` (do not destroy h first).
 */
int h2_sparsify(h2_matrix* h, const h2_sparsify_opts* opts, h2_sparse** out);

/* Sizes: blocks of the upper block triangle of S, its scalar entries. */
int h2_sparse_info(const h2_sparse* sp, int64_t* nnz_blocks, int64_t* nnz_entries);
/*
 * HOST copies of the combinatorial output (bit-exact contract):
 *   n_act, kept, nonbasis [ncl]: n_t, k_t, m_t;  soff[ncl]: first row of
 *   cluster t in S (S order: level 0 first, clusters left to right, the
 *   permutations P_rk of Section 2);  elim[ncl]: clusters in the elimination
 *   order of the factorisation (levels from the leaves up; inside a level by
 *   greedy colour of the close graph, then cluster index; clusters without
 *   non-basis rows last on their level);  rowptr[ncl+1], colidx[nnz_blocks]:
 *   the stored upper block triangle in that order (block rows by elimination
 *   position, column cluster ids sorted by elimination position).
 * Any pointer may be NULL.
 */
int h2_sparse_export_plan(const h2_sparse* sp, int64_t* n_act, int64_t* kept,
                          int64_t* nonbasis, int64_t* soff, int64_t* elim,
                          int64_t* rowptr, int64_t* colidx);
/*
 * h2_sparsify_batch: sparsifies `count` independent H^2 matrices (uneven
 * sizes, ranks and depths allowed; one precision and one kernel kind for
 * all, H2_EUNSUPPORTED for matrices of different kernels) in one level sweep:
 * level k of every instance (from the leaves up) runs in the same QR,
 * transform and strip launches, their work lists concatenated.  outs[i]
 * receives the handle of hs[i], as h2_sparsify would return it; on error no
 * handle is returned.  A matrix may appear once (EINVAL otherwise).
 * h2_last_timings / h2_last_work report the whole batch.
 */
int h2_sparsify_batch(h2_matrix* const* hs, int count, const h2_sparsify_opts* opts, h2_sparse** outs);

/* HOST copy of block (t, s) of S (m_t x m_s column-major, FP64) for any (t, s)
 * in the pattern (either orientation); EINVAL when (t, s) is not in it. */
int h2_sparse_export_block(const h2_sparse* sp, int64_t t, int64_t s, double* out);
/* HOST copy of Q_t (n_t x n_t column-major, FP64). */
int h2_sparse_export_q(const h2_sparse* sp, int64_t t, double* out);

/* ---- factorisation of S (the sparse-solver step of Sections 5.3-5.5) -------- */
/*
 * h2_factor_S: block factorisation of S in the elimination order, symmetric
 * form S = L D L^T with L^T_kj = D_k^{-1} S_kj (S is symmetric, Proposition
 * 2.1); the sparse direct factorisation of Sections 5.3-5.4 (H2_FACTOR_EXACT)
 * or its incomplete form used as a preconditioner in Section 5.5
 * (H2_FACTOR_ILU0).  EXACT first extends S's block pattern by its symbolic
 * fill (new blocks start at zero) and so re-lays `sp`'s S; ENOMEM if the
 * filled S does not fit in device memory.  Pivot blocks D_k are inverted in
 * FP64 by Gauss-Jordan with partial pivoting; the Schur updates run in the
 * precision of `sp`.  Left-looking, a few launches per level of the
 * elimination DAG.  opts NULL = ILU(0).  The factors overwrite S: a sparse
 * handle is factored once (EINVAL on a second call).  ESINGULAR if a pivot
 * block is singular.  The handle keeps a reference to `sp`.
 */
int h2_factor_S(h2_sparse* sp, const h2_factor_opts* opts, h2_factor** out);

/* Host-only counts of the plan of a matrix (no device work, nothing kept):
 * the sizes the storage study of Sections 5.1-5.2 compares.  Entries, not
 * bytes; S and U = V as the method defines them (A = U S V^T, eq. main_fact). */
typedef struct {
  int64_t n, clusters, depth;
  int64_t s_blocks;          /* blocks of the upper block triangle of S             */
  int64_t s_entries;         /* entries of S, both triangles (the nonzeros of S)     */
  int64_t s_upper_entries;   /* entries of the upper block triangle (stored)          */
  int64_t q_entries;         /* entries of the orthogonal blocks Q_t that form U = V  */
  int64_t h2_entries;        /* the H^2 matrix as given: leaf bases, transfers,
                                couplings of the admissible pairs, close blocks       */
  int64_t h2_close_entries;  /* of which close blocks                                 */
  int64_t filled_entries;    /* upper triangle of the exact factor's pattern, or -1   */
  double exact_flops;        /* flops of the exact factor's Schur updates, or -1     */
} h2_plan_counts;
/* with_fill = 1 also runs the symbolic fill of the exact mode (may be slow). */
int h2_plan_report(h2_matrix* h, int with_fill, h2_plan_counts* out);

/* Host-only symbolic analysis of the exact mode, before factoring: entries of
 * the filled upper block triangle of S and the flops of its Schur updates
 * (2 m_i m_j m_k per update).  Either pointer may be NULL. */
int h2_factor_analyze(const h2_sparse* sp, int64_t* filled_entries, double* exact_flops);

/*
 * h2_solve: x = A_H2^{-1} b with M^{-1} = V (L D L^T)^{-1} U^T (eq. sp0 with the
 * factor of S) as the approximate inverse, against the FP64 H^2 matvec
 * (Definition 4.9), until max_col ||b - A_H2 x||_2 / ||b||_2 <= tol:
 * iterative refinement x += M^{-1} r, r = b - A_H2 x, or right-preconditioned
 * flexible GMRES (Saad 1993: the search directions M^{-1} v_j are kept, so an
 * FP32 M^{-1} need not be an exactly fixed linear map; restarted, modified by
 * classical Gram-Schmidt applied twice), chosen by opts->method.
 * b, x: DEVICE pointers, column-major n x nrhs, leading dimension ld >= n,
 * ORIGINAL point order; 1 <= nrhs <= 512.  opts NULL: tol 1e-10, max_iter 30,
 * H2_SOLVE_AUTO.  ENOCONV (x written, info filled) if max_iter is hit above
 * the tolerance.  GMRES keeps 2 restart + 1 vectors of n x nrhs FP64 on the
 * device (ENOMEM when they do not fit).
 */
int h2_solve(h2_factor* f, const double* b, double* x, int64_t nrhs, int64_t ld,
             const h2_solve_opts* opts, h2_solve_info* info);

/*
 * h2_solve_with: as h2_solve, for the operator `a` (its FP64 H^2 matvec), with
 * the factor f of another H^2 matrix of the same points and cluster tree as
 * M^{-1} (EINVAL otherwise).  Section 5.5 preconditions GMRES on an accurate
 * H^2 matrix by the sparsification of a coarse one of the same kernel.
 */
int h2_solve_with(const h2_matrix* a, h2_factor* f, const double* b, double* x, int64_t nrhs,
                  int64_t ld, const h2_solve_opts* opts, h2_solve_info* info);

/*
 * Batched factorisation and solve of independent instances: each instance as
 * h2_factor_S / h2_solve, run concurrently on a pool of streams that start
 * after the work queued on the current stream and that the current stream
 * waits for on return.  b[i], x[i]: device pointers of instance i (its own
 * nrhs[i], ld[i]); infos may be NULL.  A handle may appear once per batch,
 * and the factors of one solve batch must belong to different matrices
 * (EINVAL otherwise: a matrix keeps one matvec plan and its vectors).
 * Any instance failing fails the call (first error reported); ENOCONV after
 * every instance ran if one of them stopped above the tolerance.  A batched
 * factorisation times each instance as a whole only: h2_last_timings gives
 * the sum of the instances' totals in [7] and zero for the per-level phases
 * [4], [5] and [8..10].
 */
int h2_factor_S_batch(h2_sparse* const* sps, int count, const h2_factor_opts* opts, h2_factor** outs);
int h2_solve_batch(h2_factor* const* fs, int count, const double* const* b, double* const* x,
                   const int64_t* nrhs, const int64_t* ld, const h2_solve_opts* opts, h2_solve_info* infos);

/* One application of the preconditioner: x = V (L D L^T)^{-1} U^T b (device),
 * i.e. the solve S y = U^T b, x = V y of eq. sp0 (Introduction) with the
 * block factorisation of S in place of S; b, x: device, column-major n x nrhs,
 * leading dimension ld >= n, 1 <= nrhs <= 512; EINVAL otherwise. */
int h2_apply_inverse(h2_factor* f, const double* b, double* x, int64_t nrhs, int64_t ld);

/* h2_apply_inverse for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same result, with every vector and work list in
 * one static device array of the library (64 MiB per GPU, held until the
 * process ends) instead of memory of its own; no hipMalloc, hipFree or other
 * allocating routine is called.  Requests whose vectors and work lists do not
 * fit the array (about 4 n nrhs doubles plus the lists) return EINVAL with a
 * message.  Every call on a GPU shares that GPU's array: calls that overlap on
 * one GPU (other streams or threads) race; the array keeps the last call's
 * contents, and each call writes everything it reads.  Work runs on the
 * stream of h2_set_stream and the call returns when it is done. */
int h2_apply_inverse_noalloc(h2_factor* f, const double* b, double* x, int64_t nrhs, int64_t ld);

void h2_matrix_destroy(h2_matrix* h);
void h2_sparse_destroy(h2_sparse* sp);
void h2_factor_destroy(h2_factor* f);

/* Device time (ms) of the last sparsify / factor call's kernels, by phase:
 * [0] QR, [1] close transforms, [2] couplings, [3] strips, [4] factor pivots,
 * [5] factor Schur updates, [6] sparsify total, [7] factor total, [8], [9],
 * [10] the Schur updates split by kernel (tile class): tiles with at most 4
 * blocks of 16 along both sides, with 5 along the longer side, with 6 to 8
 * (FP32 only).  Measured with HIP events; count up to 12. */
int h2_last_timings(double* ms, int count);
/* Algorithmic work of the last sparsify / factor call on this thread, same
 * phase order as h2_last_timings: flop counts of the GEMMs and QRs as planned
 * (2 m n k per product), [6] = bytes the QR phase must move at least,
 * [7] = Schur targets of the factorisation whose sum over pivots was split
 * into parts (long K; the environment variable H2SP_SCHUR_SPLIT_K sets the
 * smallest K of a part, default 512), [8] = Schur kernel launches of the
 * factorisation, [9] = stored S entries the factorisation worked on (after
 * the fill in exact mode), [10] / [11], [12] / [13], [14] / [15] flops and
 * launches of the Schur kernels of tile classes 0, 1, 2 (as in
 * h2_last_timings [8..10]), [16] / [17] fill blocks dropped / kept by
 * H2_FACTOR_ILUT (fill blocks that no update reached, zero throughout, are
 * counted in neither).  count may be up to 20. */
int h2_last_work(double* work, int count);

/* ---- tuning table and autotuner ---------------------------------------------- */
/*
 * The tile shape of every batched GEMM kind (precision, role, operand layout,
 * bucket of item rows) and the Schur work-list knobs come from a tuning
 * table.  Built-in defaults apply until a JSON cache replaces them: one
 * object per GPU architecture ("gfx950": {key: integer, ...}), read once per
 * process from H2SP_TUNE_FILE or else tune.json beside the library (a missing
 * default file means the defaults; a malformed one, or an entry that is not
 * built, makes every call that plans work fail with EINVAL).  Entries change
 * speed only, never a result bit.  Keys:
 *   "gemm.<f32|f64>.<transform|factor|solve|matvec>.a<A>b<B>.m<R>": the tile
 *     variant (0..5, those built for the kind) of GEMM batches whose operand
 *     layouts are A and B and whose largest item has <= 16, 32, 64 or more
 *     rows (R = 0..3);
 *   "schur.split_k" (16..2^30, default 512): smallest K of a split Schur part;
 *   "schur.key_z" (0 or 1, default 0): order Schur tiles by Z position;
 *   "schur.order_min" (default 16384): reorder levels with at least this many
 *     tiles;
 *   "schur.split_big" (0 or 1, default 0): cut targets of 6 to 8 blocks of 16
 *     into tiles of half the edge (more waves per SIMD, more operand reads);
 *   "solve.split_k" (16..2^30, default 2048): the triangular solves cut a
 *     target whose sources add up to more than 1.5 times this many rows into
 *     parts of about this many (partial sums reduced in a fixed order);
 *   "solve.transpose" (0 or 1, default 0): the backward sweep reads a
 *     transposed copy of the factored S (made once per factor, when it fits
 *     in a third of the memory the device can give) instead of S itself.
 * The environment variables below override the Schur knobs.  Work lists
 * already planned are planned again after any change.  h2_tune_set replaces
 * one entry (EINVAL for unknown keys, values out of range or variants that are
 * not built); h2_tune_get reads an entry of the table (EINVAL when it holds
 * none: the default applies); h2_tune_clear returns to the defaults;
 * h2_tune_load reads the object of the current device's architecture from a
 * file (NULL: the default path); h2_tune_save writes the table there, keeping
 * the other architectures' objects; h2_tune_report writes JSON text
 * {"arch", "source", "used": {key: value}} naming every entry the planned
 * work consulted since the last load (EINVAL if len is too small).
 *
 * h2_autotune: on the caller's matrix, in `precision`, with nrhs right-hand
 * sides (1..512), measures every built variant of each GEMM kind that the
 * sparsification, the ILU(0) factorisation, the preconditioner application
 * and the FP64 product plan, and the Schur knobs (split_k in {256, 512, 1024,
 * 2048}, key_z and split_big in {0, 1}; the solve's split_k in {512, 1024, 2048, 4096,
 * 2^30}), one key at a time with the others fixed (device
 * time of the phase, or the time of the synchronous call), keeps the fastest
 * of each in the table and, with a path, saves it.  Runs each phase several
 * times: seconds to minutes.  Uses the stream of h2_set_stream.
 */
int h2_tune_set(const char* key, int64_t value);
int h2_tune_get(const char* key, int64_t* value);
int h2_tune_clear(void);
int h2_tune_load(const char* path);
int h2_tune_save(const char* path);
int h2_tune_report(char* buf, int64_t len);
int h2_autotune(h2_matrix* h, int precision, int64_t nrhs, const char* path);

/* Environment variables read by the library (tuning and diagnostics only; the
 * results do not depend on them beyond rounding order):
 *   H2SP_TRACE=1 host phase timings and statistics on stderr; =2 adds one line
 *     per factorisation level (tiles, flops, time, XCD spread, operand bytes);
 *     =3 also times every launch of a preconditioner application (run eagerly)
 *     and sums them by launch size;
 *   H2SP_SCHUR_UNITS (default 32768) and H2SP_SCHUR_SPLIT_K (default 512):
 *     split-K granularity of the Schur update (tile units per level, smallest
 *     K of a part);
 *   H2SP_SCHUR_ORDER: levels of at least 16384 Schur tiles reorder them
 *     inside each XCD's share; =0 keeps target order on every level, =2
 *     reorders every level (the order changes no result bit);
 *   H2SP_SCHUR_KEY: the key of that order, by default the target's row and
 *     then the place of its column cluster in space; =z the Z position where
 *     the tile's first segment starts;
 *   H2SP_SCHUR_TILED=0: the Schur update reads the S_kj operands in place
 *     instead of from copies in 16 x 16 tiles (the copies take about 1.3 times
 *     the memory of S and are made only when they fit);
 *   H2SP_SCHUR_MERGE: on a pattern extended by fill (H2_FACTOR_EXACT,
 *     H2_FACTOR_ILUT) a run of pivots whose Z_ki and tiled S_kj blocks follow
 *     each other in memory (the supernodal runs of the filled pattern) is one
 *     Schur segment, with the S_kj copies in column order; on S's own pattern
 *     one segment per pivot and the copies in row order.  =0 / =1 forces
 *     either (the same sums, grouped differently inside the MFMA steps);
 *   H2SP_ILUT_PRUNE=0: H2_FACTOR_ILUT plans every level on the full structural
 *     fill; by default (with merged runs) each level is planned after the
 *     previous level's drop decisions, without the blocks dropped so far
 *     (zero from then on); the planning then waits for the device level by
 *     level instead of running ahead of it;
 *   H2SP_CLOSE_RESIDENT=0: never keep the matvec's close blocks on the device;
 *   H2SP_GRAPHS=0: run the solve and matvec sweeps eagerly instead of as
 *     captured HIP graphs;
 *   H2SP_TUNE_FILE: the tuning cache to read (see h2_tune_load);
 *   H2SP_DEVICE_CACHE_FRACTION (default 0.9): idle device memory the library
 *     keeps for reuse, as a fraction of the device's memory; all of it is
 *     released when an allocation of the library fails. */

#ifdef __cplusplus
}
#endif
#endif /* H2SP_H */
