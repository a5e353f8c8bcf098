/* bie.h -- C ABI of the dense EFIE method-of-moments library (libbie.so, gfx950).
 *
 * The library follows the paper's statement of the problem (Sec. II): a closed
 * PEC surface Gamma, meshed by triangles, and a wavenumber k define the
 * discretised EFIE  T j = e  (eq:discretizedEFIE) with
 *     T = jk T_A - (jk)^-1 T_Phi                               (eq:efie)
 *     [T_A]_mn   =  int int f_m(x) . g(x,y) f_n(y)              (eq:matTA)
 *     [T_Phi]_mn = -int int div f_m(x) g(x,y) div f_n(y)        (eq:matTPhi)
 *     g(x,y) = exp(-jk|x-y|)/(4 pi |x-y|), time factor exp(+j w t),
 * in RWG functions without edge-length normalisation, and the excitation
 * [e]_m = int f_m . e_inc (Sec. II).  The paper solves this system with an
 * iterative method and then evaluates the scattered field from the radiation
 * potentials of the current (Sec. II): hence the calls operator -> apply ->
 * solve -> far field.
 *
 * Conventions for every call
 *   - Host arrays (const pointers named host) are read during the call only.
 *   - Device arrays are caller-owned allocations on the operator's device
 *     (e.g. torch tensors); the library never frees them.
 *   - Complex data are interleaved (re, im): complex128 = 2 x double,
 *     complex64 = 2 x float, as in torch.complex128 / torch.complex64.
 *   - A block of R vectors of length N is stored R x N, each vector
 *     contiguous (row r starts at offset r*N).
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *     their kernels on it; calls that return host results synchronise it.
 *   - Return value: BIE_OK (0), BIE_NOT_CONVERGED (1, a warning: outputs are
 *     valid), or a negative error code; bie_last_error() returns a message for
 *     the calling thread.  No C++ exception crosses this interface.
 *
 * RWG numbering (a reading; the paper only draws the basis in Sec. VI-A):
 * one unknown per interior edge, edges sorted lexicographically by
 * (lower vertex index, higher vertex index); c+ is the triangle that traverses
 * the edge from the lower to the higher vertex index, c- the other one.
 */
#ifndef BIE_H
#define BIE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    BIE_OK = 0,
    BIE_NOT_CONVERGED = 1,   /* warning: best iterate returned, see stats */
    BIE_EINVAL = -1,         /* bad argument (NULL pointer, size, option) */
    BIE_EMESH = -2,          /* open / non-manifold / mis-oriented mesh, zero-area triangle */
    BIE_ENOMEM = -3,         /* device allocation failed */
    BIE_EDEVICE = -4,        /* HIP runtime error */
    BIE_ENUMERIC = -5        /* NaN or Inf in an input vector */
};

/* Storage of the impedance matrix. */
typedef enum {
    BIE_C128 = 0,   /* complex FP64 fill and storage */
    BIE_C64 = 1,    /* complex FP32 storage; regular pairs integrated in FP32,
                       touching / near pairs always in FP64 */
    BIE_SPLIT_BF16 = 2  /* FP64 matrix plus a split-BF16 copy (hi + lo pairs) for the
                           block product on the matrix cores (FP32 accumulation) */
} bie_dtype;

typedef struct bie_op bie_op;   /* opaque: owns the device matrix and workspaces */

typedef struct {
    int storage;          /* bie_dtype, default BIE_C128 */
    double near_factor;   /* pairs with centroid distance < near_factor * longest edge
                             (or sharing a vertex) get singularity subtraction; default 2.0 */
    int keep_fp64;        /* with storage BIE_C64: also keep the FP64 matrix (for FP64
                             residuals / iterative refinement); default 0 */
    int star;             /* 1: star-split form (Sec. VI-A, star factorisation): the
                             operator stores T_A' = jk T_A (packed N x N) and
                             V' = V / (jk) (packed F x F, V the piecewise-constant single
                             layer with basis 1/A) and every product is
                             T x = T_A' x + Sigma V' Sigma^T x, Sigma the sparse star matrix
                             (+-1 for the triangles of each RWG).  The scalar part then
                             vanishes exactly on solenoidal (loop) currents whatever the
                             storage precision.  Not with BIE_SPLIT_BF16; solves with the
                             standard criterion only (RSCC needs assembled rows); no
                             warm start, batched solve or bie_op_matrix (BIE_EINVAL).
                             Default 0 */
} bie_fill_opts;

/* Operator: mesh + wavenumber -> dense impedance matrix T on the current device.
 * (Sec. II, eq:discretizedEFIE, eq:matTA, eq:matTPhi.)
 *   verts  host, nv x 3 double, vertex coordinates (m)
 *   tris   host, nt x 3 int32, vertex indices, counter-clockwise seen from outside
 *   k      wavenumber (rad/m), > 0
 *   opts   NULL for defaults
 * Quadrature: Radon's 7-point degree-5 rule on both triangles of every pair;
 * flagged pairs use subtraction of the static kernel with closed-form inner
 * integrals, averaged over both orderings, so T is exactly symmetric.
 * Errors: BIE_EMESH for an invalid mesh, BIE_ENOMEM when N x N does not fit.
 * The matrix is complete when the call returns (it synchronises `stream`). */
int bie_op_create(const double *verts, int64_t nv, const int32_t *tris, int64_t nt,
                  double k, const bie_fill_opts *opts, void *stream, bie_op **out);
void bie_op_destroy(bie_op *op);

/* Fast operator (the paper's method, Sec. III-V): T x = N x + F x with no dense
 * matrix.  F is the multilevel B-spline far field of bie_farml_create (leaf
 * cubes of side `box`, `levels` octree levels, s splines of degree p on the
 * leaves) over the pairs of far leaf cubes; N holds the entries T_mn between
 * the RWG functions of near leaf cubes (index distance <= 1), computed as the
 * dense fill computes them (Radon 7-point rule on both triangles, the singular
 * treatment on the pairs flagged by near_factor, as bie_op_create) and kept in
 * CSR.  The operator serves bie_apply (complex128, no conjugate), bie_solve
 * (GMRES, precision 0, SCC, no preconditioner), bie_rhs_planewave, bie_farfield,
 * bie_rcs and the far-field entry points; the calls that need a stored matrix
 * (bie_op_matrix, the allocation-free product, batched solves, the Calderon
 * preconditioner, block GMRES, CGNR, RSCC) return BIE_EINVAL.  Memory: 20 B per
 * near entry, 144 B per flagged pair, and the far field's. */
typedef struct {
    double box;            /* leaf cube side (m) */
    int levels;            /* octree levels of the far field, 1..12 */
    int s;                 /* splines per axis on a leaf cube */
    int p;                 /* spline degree: 1, 3 or 5 */
    double near_factor;    /* flagged pairs as in bie_fill_opts (default 2) */
} bie_fast_opts;
typedef struct {
    int64_t near_entries;  /* stored near entries (ordered pairs m, n) */
    int64_t leaf_cubes;    /* non-empty leaf cubes */
    int levels;
} bie_fast_info;
int bie_op_create_fast(const double *verts, int64_t nv, const int32_t *tris, int64_t nt, double k,
                       const bie_fast_opts *opts, void *stream, bie_op **out);
int bie_op_fast_info(const bie_op *op, bie_fast_info *info);

/* Number of unknowns N (= number of edges = 3 nt / 2). */
int64_t bie_op_n(const bie_op *op);

/* RWG table, host out N x 4 int32: (lower vertex, higher vertex, c+, c-). */
int bie_op_edges(const bie_op *op, int32_t *out);

/* Flagged (touching or near) triangle pairs p <= q used by the fill.
 * host out: up to cap pairs as 2 x int32 each; returns the total count
 * (>= 0) or a negative error code. */
int64_t bie_op_near_pairs(const bie_op *op, int32_t *out, int64_t cap);

/* Copy of the matrix into a caller buffer.  dst: device, N x N row-major
 * (T_mn at m*N + n), complex128 if dtype == BIE_C128 (converted from the
 * stored precision), complex64 if dtype == BIE_C64 (only for BIE_C64 storage). */
int bie_op_matrix(const bie_op *op, void *dst, int dtype, void *stream);

/* Plane-wave excitation (Sec. II, right-hand side):
 *   [e]_m = int f_m . p exp(-jk d . r) dS  for R waves.
 *   dirs  host R x 3, unit propagation directions d
 *   pols  host R x 3, real unit polarisation vectors p (p . d = 0)
 *   B     device R x N complex128 (output). */
int bie_rhs_planewave(const bie_op *op, const double *dirs, const double *pols, int64_t R,
                      void *B, void *stream);

/* Matrix-vector / matrix-block product (the solver's MVP):
 *   Y = T X   (conj = 0)   or   Y = T^H X = conj(T conj(X))   (conj = 1, T = T^T)
 *   X, Y  device R x N, complex128 (vec = BIE_C128) or complex64 (vec = BIE_C64);
 *         vec = BIE_SPLIT_BF16: complex128 vectors through the split-BF16 block
 *         product on the matrix cores (storage BIE_SPLIT_BF16, conj = 0);
 *         vec = BIE_APPLY_F64_BLOCK: complex128 vectors through the FP64 block
 *         product on the matrix cores (FP64 matrix stored, conj = 0; a dense
 *         FP64 copy of 16 N^2 bytes is made on first use and kept);
 *         X and Y must not overlap.  Complex128 vectors use the FP64 matrix when
 *         stored (else the FP32 matrix with FP64 accumulation); complex64 vectors
 *         use the FP32 matrix with FP32 accumulation. */
#define BIE_APPLY_F64_BLOCK 3
int bie_apply(const bie_op *op, const void *X, void *Y, int64_t R, int vec, int conj,
              void *stream);

/* Allocation-free form of bie_apply, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): Y = T X (conj = 0) or T^H X (conj = 1) through the packed
 * product, vec = BIE_C128 (FP64 matrix if stored, else FP32 with FP64
 * accumulation) or BIE_C64 (FP32 matrix), assembled operators only.  The
 * product's partial sums (R x P x 64 complex values, P the operator's partial
 * slots: about 8 MB per complex128 vector at N = 7680) go to a static device
 * array of 128 MiB that each device holds for the life of the process; larger
 * requests return BIE_EINVAL before any launch (use fewer vectors per call).
 * Nothing is allocated and no profiling events are recorded.  Every call on a
 * device shares that array: calls that overlap on one device (other streams or
 * threads) race; calls ordered on one stream do not.  The operator's device
 * must be current.  Results are bitwise those of bie_apply. */
int bie_apply_noalloc(const bie_op *op, const void *X, void *Y, int64_t R, int vec, int conj, void *stream);

typedef enum { BIE_GMRES = 0, BIE_CGNR = 1, BIE_BGMRES = 2 } bie_method;
typedef enum { BIE_SCC = 0, BIE_RSCC = 1, BIE_CCC = 2 } bie_crit;

typedef struct {
    int method;          /* bie_method; default BIE_GMRES */
    int restart;         /* GMRES restart length m (1..64); default 30 */
    double tol;          /* relative to ||b||_2; default 1e-6 */
    int64_t max_mvp;     /* cap on products per right-hand side; default 10000 */
    int crit;            /* bie_crit; default BIE_SCC (precision 1: BIE_SCC only) */
    int64_t rscc_rows;   /* S, default 512 (min(S, N) used) */
    uint64_t rscc_seed;  /* default 1234 */
    int use_x0;          /* 1: X holds the initial guess on entry; 2: the same with
                            fallback: a guess with ||b - T x0|| >= ||b|| (the solver's
                            first residual) is replaced by zero.  That residual is FP64,
                            except in mixed-precision block GMRES, where every residual
                            of the refinement is taken with the 3-term split-BF16
                            product (see precision) */
    int precision;       /* 0: products with the stored matrix (FP64 if stored);
                            1: mixed precision with iterative refinement: outer FP64
                               residual and criterion (SCC), inner GMRES on the
                               split-BF16 matrix (storage BIE_SPLIT_BF16) or on the
                               FP32 matrix (storage BIE_C64 with keep_fp64).  Block
                               GMRES takes each outer residual first with the 3-term
                               split-BF16 product (relative error near 1e-5): a
                               right-hand side above max(tol, 1e-3) only starts its
                               next correction from it, one at or below is taken again
                               in FP64, which decides convergence */
    double inner_tol;    /* precision 1: inner tolerance relative to the outer residual
                            (0: default 1e-3) */
    int64_t slots;       /* precision 1: right-hand sides in flight (continuous batch:
                            a converged one hands its slot to the next); 0: all R */
    int inner_terms;     /* precision 1, split-BF16: terms of the inner block product,
                            3 (hi/lo matrix x hi/lo vector, lo x lo dropped) or 2
                            (hi/lo matrix x BF16 vector; the inner tolerance is then
                            raised to at least 1e-2, the rounding of the vectors
                            bounding what the inner solve can attain); 0: default 3 */
    int basis;           /* precision 1, split-BF16: storage of the inner Krylov basis
                            (column and block GMRES), 0 complex64 (default) or 1 FP16
                            pairs (half the traffic of the Arnoldi kernels; the 3-term
                            split of an FP16 vector into BF16 hi/lo is exact; the
                            basis is orthonormal to about 1e-3, for inner tolerances
                            of 1e-2 and above).  BIE_EINVAL for 1 with another
                            precision or storage */
    int block;           /* BIE_BGMRES: right-hand sides per block Krylov space
                            (1..32); 0: 32 */
    const struct bie_calderon *calderon;
                         /* NULL, or a Calderon preconditioner built for this
                            operator (bie_calderon_create): GMRES then runs on
                            T M u = b with x = M u (right preconditioning, so the
                            GMRES residual and the criteria stay those of T x = b).
                            Method BIE_GMRES with precision 0, or BIE_BGMRES (the
                            steps form T (M V_j) with two block products, split-BF16
                            with precision 1; each cycle ends with X += M U in FP64);
                            BIE_EINVAL otherwise, or if it was built for another
                            operator */
} bie_solve_opts;

typedef struct {
    int64_t iters;        /* Krylov iterations */
    int64_t mvps;         /* products with T or T^H (RSCC checks count S/N, rounded up) */
    double relres_est;    /* last recursive estimate |g_{j+1}|/||b|| (GMRES) or ||r||/||b|| (CGNR) */
    double relres_true;   /* last criterion value on the true residual */
    int converged;        /* criterion met */
    int checks;           /* criterion evaluations */
    int x0_kept;          /* 1 if an initial guess was given and kept (use_x0 = 2 may drop it) */
} bie_solve_stat;

/* Solve T x = b for R right-hand sides to the selected criterion.
 * Criteria (named in the paper's acronym list, not defined there; readings):
 *   SCC:  ||b - T x||_2 / ||b||_2 <= tol;
 *   RSCC: sqrt((N/S) sum_{i in S} |b_i - (T x)_i|^2) / ||b||_2 <= tol over S
 *         rows drawn by Floyd's algorithm from SplitMix64 seeded with
 *         rscc_seed + (number of earlier checks of that right-hand side);
 *   CCC:  combined: the RSCC value gates each check, and a right-hand side whose
 *         RSCC value is <= tol is accepted only if the SCC holds as well (its
 *         full residual then also restarts the method when it does not).
 *   RSCC and CCC need the FP64 matrix (assembled operator) and precision 0.
 * Block GMRES (BIE_BGMRES; the paper names GMRES only, block GMRES is a
 * reading for many right-hand sides): consecutive groups of at most `block`
 * right-hand sides that have not converged share one block Krylov space
 * span{R0, T R0, ..., T^{j-1} R0} per restart cycle, and every column takes the
 * element of it that minimises its own residual.  R0 holds the residuals scaled
 * to unit norm, orthonormalised with rank revealing (directions below 1e-6 of
 * the largest are left out); block classical Gram-Schmidt (with the FP64
 * basis a second pass when a column keeps less than half its norm squared; the
 * complex64 basis of precision 1 takes one pass), Cholesky QR of the new block,
 * block Householder QR of the block Hessenberg matrix.  A cycle ends when every
 * column's estimate meets its target, after `restart` block steps, or on a
 * partial breakdown (a new direction at or below 1e-6 of the largest column of
 * T V_j).  Then every column is checked on its FP64 residual (SCC), converged
 * ones leave and the rest are regrouped.  Precision 0: FP64 basis and FP64
 * block products, target tol ||b||; precision 1 (split-BF16 storage):
 * complex64 basis and split-BF16 products, one cycle per refinement step to
 * inner_tol relative to the FP64 residual.  SCC only; slots > 0 solves the
 * right-hand sides in consecutive chunks of that many.  Counts: one iteration
 * and one product per block step for every column of the block.  The operator
 * keeps the block solver's device and pinned buffers and its two side streams
 * between calls (grown when a call needs more, freed by bie_op_destroy); calls
 * on one operator must not overlap.
 * GMRES(m): Arnoldi with classical Gram-Schmidt and selective
 * reorthogonalisation (a second pass when the first removes more than half of
 * ||w||^2), FP64 Givens rotations; a cycle ends when the estimate <= tol or j = m, then the
 * criterion is evaluated on the true residual.  CGNR: CG on T^H T x = T^H b.
 *   B      device R x N complex128
 *   X      device R x N complex128 (in: initial guess if use_x0; out: solution)
 *   stats  host array of R entries (may be NULL)
 * Returns BIE_NOT_CONVERGED if any right-hand side missed the criterion
 * within max_mvp, BIE_ENUMERIC if B or X0 holds NaN/Inf.  ||b|| = 0 gives x = 0. */
int bie_solve(const bie_op *op, const void *B, void *X, int64_t R, const bie_solve_opts *opts,
              bie_solve_stat *stats, void *stream);

/* Batched solves: the right-hand sides of nops operators of different sizes
 * (meshes, wavenumbers) solved together with GMRES(m) (method BIE_GMRES; other
 * options as in bie_solve, use_x0 0/1/2).  Criteria: SCC, or RSCC / CCC as in
 * bie_solve (S = min(rscc_rows, N_p, 4096) rows per right-hand side, drawn per
 * check; needs the FP64 matrices: FP64 storage or precision 1): at the end of a
 * cycle whose estimate meets tol, RSCC accepts on the sampled value, CCC
 * confirms a sampled acceptance on the full residual; an initial guess is
 * checked on its full residual.  Precision 0: products with the stored matrices (all FP64 or
 * all FP32), residuals on the same.  Precision 1 (every operator stored as
 * BIE_C64 with keep_fp64): the Arnoldi products on the FP32 tiles, every
 * residual -- the vector each restart cycle starts from and the criterion --
 * on the FP64 tiles, so a cycle is one step of iterative refinement and the
 * criterion is certified in FP64.
 * Every right-hand side keeps its own Krylov basis, Hessenberg matrix and
 * criterion; the products of all operators share one grouped launch per
 * iteration and each restart cycle is replayed as one captured HIP graph.
 * Work runs on a library stream ordered after `stream`; the call returns
 * when the solutions are written.
 *   ops    host array of nops operators (one device)
 *   B, X   host arrays of nops device pointers: R[p] x N_p complex128 each
 *          (X in: initial guesses if use_x0; out: solutions)
 *   R      host array of nops right-hand-side counts (0 allowed)
 *   stats  host, sum(R) entries in operator order.
 * Returns BIE_NOT_CONVERGED if any right-hand side missed the criterion. */
int bie_batch_solve(const bie_op *const *ops, int64_t nops, const void *const *B, void *const *X,
                    const int64_t *R, const bie_solve_opts *opts, bie_solve_stat *stats, void *stream);

/* Batched solves as bie_batch_solve, right-preconditioned per operator with the
 * multiplicative Calderon preconditioner of Sec. VI-A and VII (M = -G^-1 T_BC
 * G^-T, see bie_calderon_create): GMRES on T_p M_p u = b with x = M_p u, so residuals and
 * criterion stay those of T_p x = b.  Each Arnoldi step forms T (M v) with two
 * grouped launches (M of every operator, then T); each cycle ends with
 * x += M (V y).  M is applied in the precision of the Arnoldi products: its
 * FP64 tiles with FP64 matrices, an FP32 copy of them (made on first use and
 * kept with the preconditioner) with FP32 matrices or precision 1.
 *   pcs    host array of nops preconditioners, pcs[p] built for ops[p]; NULL
 *          gives bie_batch_solve.  opts->calderon must be NULL.
 * Other arguments, results and errors as in bie_batch_solve; BIE_EINVAL for a
 * NULL entry or a preconditioner built for another operator. */
int bie_batch_solve_pc(const bie_op *const *ops, const struct bie_calderon *const *pcs, int64_t nops,
                       const void *const *B, void *const *X, const int64_t *R, const bie_solve_opts *opts,
                       bie_solve_stat *stats, void *stream);

/* The grouped product of the batched solves on its own (Sec. I/II: the O(N^2)
 * product T x, here for several operators of different sizes at once):
 * Y_p = T_p X_p for the R[p] columns of every operator p, all in one tile
 * launch over (operator, unit of tiles, group of columns) work items and one
 * reduce launch, as inside bie_batch_solve.
 *   ops    host array of nops assembled dense operators (one device)
 *   X, Y   host arrays of nops device pointers: R[p] x N_p complex128 each,
 *          each column contiguous (X read, Y written; distinct buffers)
 *   R      host array of nops column counts (0 allowed; sum at most 65535)
 *   mat    0: the FP64 tiles (FP64 accumulation); 1: the FP32 tiles on the
 *          vector units (FP64 accumulation); 2: the FP32 tiles on the FP32
 *          matrix cores (vectors rounded to FP32, FP32 accumulation within a
 *          unit, partial sums and their reduction in FP64); 3: the FP64 tiles
 *          on the FP64 matrix cores (FP64 throughout; the residual pass of
 *          precision-1 batches with matrix cores on)
 *   unit_tiles     tiles per work unit, 1..64 (0: 8)
 *   cols_per_item  columns per work item, 1..4096, at most 32 with mat 2 or 3
 *                  (0: 8, or 32 with mat 2 or 3)
 * The columns go through library buffers (allocated per call); the call
 * returns when Y is written.  BIE_EINVAL for a NULL argument, a star-split or
 * fast operator, a missing matrix of the requested precision, operators on
 * several devices or sizes out of range. */
int bie_batch_apply(const bie_op *const *ops, int64_t nops, const void *const *X, void *const *Y, const int64_t *R,
                    int mat, int unit_tiles, int cols_per_item, void *stream);

/* Batched solves, for measurement and tests: tiles per work unit of the
 * grouped product (0, the default: tiles per unit in {4, 8, 16} and columns per
 * work item in {4, 8, 16, 32} chosen per batch shape by timing the candidates
 * on the batch; the choices are kept for the process and appended to the file
 * named by BIE_AUTOTUNE_CACHE if set; > 0: that many tiles per unit, 8 columns
 * per item; -1: each operator's own single-product units, 8 columns per item,
 * which makes every column bitwise equal to its single solve), graph replay
 * (1: default) and, for precision 1 on FP32 tiles, the grouped products on the
 * FP32 matrix cores (matrix_cores 1, the default: every work item takes up to 32
 * columns of its unit at once, vectors rounded to FP32 and FP32 accumulation
 * within a unit, partial sums and their reduction in FP64; the FP64 residuals
 * then on the FP64 matrix cores; 0: the VALU passes with FP64 accumulation).
 * BIE_EINVAL outside -1..64. */
int bie_batch_config(int unit_tiles, int use_graph, int matrix_cores);
/* Tiles per unit chosen for this batch shape so far (0: none); for operators
 * holding both matrices, the choice for FP64 products if one was made, else the
 * one for FP32 products. */
int bie_batch_tuned(const bie_op *const *ops, int64_t nops, const int64_t *R);

/* ---------------------------------------------------------------------------
 * Multiplicative Calderon preconditioner (Andriulli et al., IEEE TAP 56(8),
 * 2008), used by the paper in all of its simulations (Sec. VI-A, remark on the
 * star-split operator; Sec. VII).  M = -G^{-1} T_BC G^{-T} with T_BC the EFIE
 * matrix in the Buffa-Christiansen basis (built on the barycentric refinement
 * of the mesh: charge spread uniformly over each dual cell, flux 1/2 through
 * each half of the dual edge, none through the halves of the primal edge) and
 * G_mn = <n x b_m, f_n> the mixed Gram matrix; M T discretises the square of the
 * EFIE operator (spectrum accumulating at -1/4).  M is complex symmetric and
 * kept in FP64 in the same packed tiles as T, so a preconditioned product is
 * two packed products. */
typedef struct bie_calderon bie_calderon;
typedef struct {
    int64_t N, Nb;             /* unknowns of the mesh and of its barycentric refinement (9 F) */
    int64_t nnz_bc;            /* nonzeros of the BC coefficient map (N x Nb) */
    int64_t nnz_gram;          /* nonzeros of G */
    int64_t cg_iters[2];       /* iterations of the two Gram solves (all N columns at once):
                                  Chebyshev steps, plus CG steps on the normal equations
                                  where Chebyshev fell back */
    double cg_relres[2];       /* their final relative residuals, max over columns (<= 1e-13) */
    double setup_ms;           /* wall time of bie_calderon_create */
} bie_calderon_info;

/* Builds M for an assembled operator (not star-split) with N <= 12288.  Fills
 * the refined mesh on the device (the fill's pair scratch, 1152 N^2 bytes,
 * beside the refined FP64 matrix, 288 N^2; then that matrix, its dense copy,
 * 576 N^2, and five N x N work matrices; the pair scratch stays allocated
 * through the rest of the setup only when free device memory allows, else it
 * is freed after the fill, so the peak is at most 1440 N^2 bytes when memory
 * is short), forms T_BC in column chunks, solves
 * with G for all N columns (Chebyshev iteration, CG on the normal equations if
 * it fails; the environment variable BIE_CALDERON_GRAM=cgnr selects CG on the
 * normal equations from the start, for comparison and tests) and stores M
 * (16 N^2 / 2 bytes).  The operator must outlive the preconditioner.  The
 * setup's three largest buffers are kept per device while any preconditioner
 * lives and reused by the next setup (freed when the last one is destroyed);
 * setups run one at a time.  BIE_ENUMERIC if a Gram solve misses 1e-13. */
int bie_calderon_create(const bie_op *op, void *stream, bie_calderon **out);
/* Y = M X for R complex128 vectors (device, R x N each, vectors contiguous); FP64
 * throughout (packed product below 8 vectors, the FP64 matrix cores from 8). */
int bie_calderon_apply(const bie_calderon *pc, const void *X, void *Y, int64_t R, void *stream);
int bie_calderon_get_info(const bie_calderon *pc, bie_calderon_info *info);
void bie_calderon_destroy(bie_calderon *pc);

/* Radiation vector F(r) = int j(y) exp(jk r . y) dS of the solutions X for M
 * unit directions (Sec. II, scattered field from the radiation potentials);
 * the far field is E_s ~ -jk exp(-jkr)/(4 pi r) (I - r r) . F and the bistatic
 * RCS (k^2/(4 pi)) |r x F|^2.
 *   X    device R x N complex128;  obs  host M x 3;  F  device R x M x 3 complex128. */
int bie_farfield(const bie_op *op, const void *X, int64_t R, const double *obs, int64_t M,
                 void *F, void *stream);

/* Bistatic radar cross section (m^2) of the solutions X for a plane wave of
 * unit amplitude: sigma(r) = (k^2 / (4 pi)) |r x F(r)|^2 with F the radiation
 * vector above (the unknown is the current times the wave impedance, Sec. II,
 * so no further factor enters).
 *   X      device R x N complex128
 *   obs    host M x 3 unit directions (|r| = 1 to 1e-9, else BIE_EINVAL)
 *   sigma  device R x M double (row r: the M directions for solution r).
 * Synchronises `stream`. */
int bie_rcs(const bie_op *op, const void *X, int64_t R, const double *obs, int64_t M, double *sigma, void *stream);

/* ---------------------------------------------------------------------------
 * Single-level far field by tensor-product B-spline interpolation of g (the
 * paper's Sec. III: eq:TAfactor, eq:TAfactorBspline; buffer knots, Sec. III-B;
 * stabilised knots, Sec. V-B; knot insertion, Sec. IV-B).  The operator's mesh
 * is covered by cubes of side `box`; an RWG function belongs to the cube that
 * holds the mean of its two triangle centroids; two cubes are far when their
 * indices differ by more than one along some axis.  Each cube carries degree-p
 * splines (p odd: 1, 3 or 5) on an open equidistant knot vector of s splines
 * per axis extended by buffer knots covering the supports that protrude, with
 * (p - 1)/2 knots removed next to each end; their interpolation points lie on
 * one lattice, so g between cubes is read from one table.  The product is
 *   [Z~_far x]_m = sum over far cubes of  jk sum_d m~_d,m^T G m~_d,n x_n
 *                                         + (1/(jk)) m~_div,m^T G m~_div,n x_n
 * with m~ the moments of the RWG function (vector components and divergence)
 * against the splines, taken with the fill's quadrature rule and mapped by
 * B_stab^-1 C.  Only the far part is applied (near cubes: the dense matrix). */
typedef struct bie_far bie_far;
typedef struct {
    double box;            /* cube side (m), > 0 */
    int s;                 /* splines per axis over one cube side, >= p + 1 + (p - 1) */
    int p;                 /* degree: 1, 3 or 5 */
} bie_far_opts;
typedef struct {
    int64_t boxes;         /* non-empty cubes */
    int64_t far_pairs;     /* ordered pairs of far cubes */
    int64_t buffer_knots;  /* per side */
    int64_t splines;       /* equidistant splines per axis, buffer included */
    int64_t points_per_axis;  /* interpolation points per axis (stabilised splines) */
    double protrusion;     /* largest protrusion of a support beyond its cube, in cube sides */
    double origin[3];      /* lower corner of cube (0, 0, 0) */
} bie_far_info;
/* Builds the cube level, the moments (device kernels) and the table of g.
 * BIE_EINVAL for bad options, a star-split operator, buffers that reach half a
 * cube (the buffered domains of cubes two apart would touch: use larger cubes
 * or more splines) or more than 24 splines per axis. */
int bie_far_create(const bie_op *op, const bie_far_opts *opts, void *stream, bie_far **out);
/* Y = Z~_far X for R complex128 vectors (device, R x N each). */
int bie_far_apply(bie_far *far, const void *X, void *Y, int64_t R, void *stream);
int bie_far_get_info(const bie_far *far, bie_far_info *info);
/* Cube index (3 x int32, host out, N rows) of every RWG function. */
int bie_far_boxes(const bie_far *far, int32_t *out);
void bie_far_destroy(bie_far *far);

/* Multilevel B-spline far field (Sec. IV; FFT translations, Sec. III-C).  A
 * regular octree over the cubes of side `box` of bie_far_create (level 0, the
 * leaves); the cube of level l holding leaf cube (i, j, k) is (i, j, k) >> l,
 * up to `levels` levels.  Each level has its own splines: while the parent's
 * cubes are smaller than half a wavelength it keeps s and takes ceil(sb/2)
 * buffer knots (Sec. IV-C), otherwise 2 s - p splines and the same sb
 * (Sec. IV-D).  Moments of the leaves (equidistant splines) move up by the
 * knot-insertion transfers of eq:interleveltransfer (exact: nested knot
 * vectors), are translated on each level between the cube pairs whose cubes
 * are far and whose parents are near (every far pair on the top level), with
 * G applied as a three-level Toeplitz convolution by FFT (eq:TAfactorBspline:
 * one symbol per cube offset), and come down by the transposed transfers to
 * the test functions.  The product covers exactly the pairs of far leaf cubes,
 * the same set as bie_far with the same box.  p odd (1, 3, 5); at most 18
 * equidistant splines and 16 interpolation points per axis on any level.
 * Memory per level: about 4 (2 L^3 + 2 n^3 + nst^3) x 16 B per cube (L = 16 or
 * 32, the FFT size) plus L^3 x 16 B per distinct cube offset. */
typedef struct bie_farml bie_farml;
typedef struct {
    double box;            /* leaf cube side (m), > 0 */
    int levels;            /* octree levels used, 1..12 (1: single level) */
    int s;                 /* splines per axis over one leaf cube side */
    int p;                 /* degree: 1, 3 or 5 */
} bie_farml_opts;
/* BIE_EINVAL for bad options, buffers that reach half a cube on some level,
 * or too many splines or points per axis on some level. */
int bie_farml_create(const bie_op *op, const bie_farml_opts *opts, void *stream, bie_farml **out);
/* Y = Z~_far X for R complex128 vectors (device, R x N each), one vector after
 * another. */
int bie_farml_apply(bie_farml *f, const void *X, void *Y, int64_t R, void *stream);
/* Per level (0 = leaves): cubes, pairs translated there (far_pairs), buffer
 * knots, equidistant splines and interpolation points per axis; protrusion and
 * origin as for the leaves. */
int bie_farml_level_info(const bie_farml *f, int level, bie_far_info *info);
void bie_farml_destroy(bie_farml *f);

/* Row sample of the random-sampling criterion: S distinct sorted indices in
 * [0, N) for `seed` (host out, S int64).  Exposed so callers can reproduce the
 * rows a given check used. */
int bie_rscc_rows(int64_t N, int64_t S, uint64_t seed, int64_t *out);

/* ---------------------------------------------------------------------------
 * Learned warm start.  Not part of the paper: a production form beside the
 * plain solve.  A POD basis U (K modes) of solutions the method computed and a
 * small network map the incidence to K coefficients: x0 = U c.  The network
 * takes (d_x, d_y, d_z, s) with d the propagation direction and s = +1 / -1
 * for theta-hat / phi-hat polarisation, has two tanh layers of `hidden` units
 * and a linear output layer of 2K values (Re, Im of c divided by one global
 * RMS scale), FP32, trained on the device with mean squared error and Adam
 * (0.9, 0.999, 1e-8), learning rate cosine-decayed lr_max -> lr_min.
 * Glorot-uniform initial weights (SplitMix64(seed), in layer order, row-major
 * (out, in)) and per-epoch Fisher-Yates shuffles (SplitMix64(seed + 1 + epoch)).
 * Parameter layout (float): W1 (hidden x 4), b1, W2 (hidden x hidden), b2,
 * W3 (2K x hidden), b3.  Plain GMRES from zero stays the fallback: the
 * solver's residual of the prediction decides whether it is kept (see
 * bie_ws_predict). */
typedef struct bie_ws bie_ws;

typedef struct {
    int pod_rank;        /* K, default 256 */
    int hidden;          /* default 512 */
    int epochs;          /* default 3000 */
    int batch;           /* default 256 */
    double lr_max;       /* default 1e-3 */
    double lr_min;       /* default 1e-5 */
    uint64_t seed;       /* default 555 */
    int oversample;      /* POD range finder: L = K + oversample columns, default 32 */
    int power_iters;     /* POD range finder power iterations, default 2 */
    int pol_model;       /* 0: inputs (d, s), 2K outputs; 1: linear in the polarisation:
                            input d, outputs f_x, f_y, f_z (3 x 2K) and the coefficients
                            for polarisation e are sum_c e_c f_c (smooth on the whole
                            sphere, unlike the theta/phi frame); default 0 */
} bie_ws_opts;

/* Train from S solutions.  feats host S x 4; pols host S x 3 real unit
 * polarisations (needed for pol_model 1, else may be NULL); X device S x N
 * complex128 (the solutions, e.g. from bie_solve).  POD: randomised range finder with power
 * iterations and CholeskyQR2 on the device; the small (K + oversample)-sized
 * Cholesky and Hermitian eigenproblems on the host.  The returned object
 * refers to `op` (which must outlive it). */
int bie_ws_train(const bie_op *op, const double *feats, const double *pols, const void *X, int64_t S,
                 const bie_ws_opts *opts, void *stream, bie_ws **out);

/* Train the network of ws on S given inputs and targets with the kernels and
 * schedule of bie_ws_train (mini-batches of `batch` in the order of a
 * Fisher-Yates shuffle from SplitMix64(seed + 1 + epoch), Adam (0.9, 0.999,
 * 1e-8) with bias correction, learning rate cosine-decayed from lr_max at the
 * first step to lr_min at the last), starting from its current parameters and
 * fresh Adam moments.  For callers with their own coefficients, and for
 * comparing the training with an independent implementation.
 *   feats    host S x 4 (pol_model 1 ignores the fourth input)
 *   pols     host S x 3 real unit polarisations (pol_model 1; else may be NULL)
 *   targets  host S x 2K float (Re then Im of the scaled coefficients)
 *   final_loss  host out (may be NULL): mean squared error over the last epoch
 * The inputs are copied to the device during the call; it synchronises `stream`. */
int bie_ws_fit(bie_ws *ws, const double *feats, const double *pols, const float *targets, int64_t S, int epochs,
               int batch, double lr_max, double lr_min, uint64_t seed, double *final_loss, void *stream);

/* Predict x0 = U c for R inputs (feats host R x 4; pols host R x 3 for
 * pol_model 1, else may be NULL) into X0 (device R x N complex128).  If B (device R x N) is given, a prediction is kept only where
 * ||b - T x0|| < ||b|| and set to 0 otherwise; used[r] (host, may be NULL)
 * tells which were kept. */
int bie_ws_predict(bie_ws *ws, const double *feats, const double *pols, int64_t R, const void *B, void *X0,
                   int32_t *used, void *stream);

/* Sizes and training summary; sigma (host, K entries, may be NULL): POD singular values. */
int bie_ws_info(const bie_ws *ws, int64_t *pod_rank, int64_t *hidden, int64_t *nparams, double *scale,
                double *final_loss, double *sigma);
/* Copy of the POD basis: U device K x N complex128 (mode k contiguous). */
int bie_ws_basis(const bie_ws *ws, void *U, void *stream);
/* Network parameters (host float array of nparams): read (set = 0) or write (set = 1). */
int bie_ws_params(bie_ws *ws, float *host, int set);
/* Mean squared error of the network on R inputs (host R x 4) against targets
 * (host R x 2K) and its gradient (host float nparams, may be NULL), computed by
 * the device forward and backward kernels.  pol_model 1: the error is that of
 * the combination sum_c e_c f_c with the polarisations pols (host R x 3);
 * pols may be NULL for pol_model 0. */
int bie_ws_loss_grad(bie_ws *ws, const double *feats, const double *pols, const float *targets, int64_t R,
                     double *loss, float *grad);
/* Raw network outputs (host R x O, O = 2K, or 6K for pol_model 1) for R inputs
 * (pol_model 1 ignores the fourth input). */
int bie_ws_forward(bie_ws *ws, const double *feats, int64_t R, float *out);
/* Untrained network with Glorot-uniform weights (no POD basis); pol_model as in
 * bie_ws_opts. */
int bie_ws_create(const bie_op *op, int pod_rank, int hidden, uint64_t seed, int pol_model, bie_ws **out);
int bie_ws_save(const bie_ws *ws, const char *path);
int bie_ws_load(const bie_op *op, const char *path, bie_ws **out);
void bie_ws_destroy(bie_ws *ws);

/* Autotuner (launch shapes chosen by timing on the device): with on != 0 (the
 * default; the environment variable BIE_AUTOTUNE=0 starts with it off) the
 * packed product's work units (4, 8 or 16 tiles, or balanced runs) are chosen
 * per matrix size and precision when an operator is created, and the
 * split-BF16 block product's wave tiles (128 x 64, 64 x 128, 128 x 128) and K
 * slices, and the FP64 block product's K slices, per matrix and column shape
 * at their first launch of that shape (not while the stream is being
 * captured); each choice is kept for the process (and, with BIE_AUTOTUNE_CACHE
 * naming a file, appended there and read by later processes).  Off: the fixed
 * defaults.  The batched solves' units and column groups are chosen the same
 * way (bie_batch_config).  Results differ between shapes only in the order of
 * floating-point sums. */
int bie_autotune(int on);
/* The choices so far, one line "key value..." each, NUL-terminated into buf
 * (at most cap bytes, may be NULL); returns the length needed. */
int64_t bie_autotune_report(char *buf, int64_t cap);

/* Measurement support (not part of the method): with on != 0 every launch of
 * the dense product kernels (from bie_apply and inside bie_solve) is bracketed
 * by HIP events on the stream it runs on.  bie_prof_read waits for the
 * recorded events of `kernel` (0: tile pass of the packed symmetric product,
 * 1: split-BF16 block product, 2: FP64 block product, 3: reduction of the
 * packed product's partial sums, 4: block GMRES first-pass dots V^H W with
 * their reduction, 5: block GMRES first-pass update W -= V C, 6: regular
 * triangle pairs of an FP64 fill (columns: triangle pairs p <= q), 7: flagged
 * triangle pairs of a fill (columns: flagged pairs), 8: assembly of the packed
 * matrix (columns: unknowns), 9: regular triangle pairs of an FP32 fill;
 * BIE_EINVAL otherwise) and returns the number of launches, their summed duration in
 * ms and (columns, may be NULL) the summed number of right-hand sides of those
 * launches (the packed product counts every column of its grid, skipped ones
 * included; record 4 counts basis vector x column pairs, sum of K r over the
 * groups, record 5 the basis vectors read, sum of K) since the previous read,
 * then clears that record. */
int bie_prof_enable(int on);
int bie_prof_read(int kernel, int64_t *launches, double *total_ms, int64_t *columns);

const char *bie_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BIE_H */
