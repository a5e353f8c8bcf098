// Internal declarations of libbie: operator state, error plumbing, launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <functional>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/bie.h"

namespace bie {

// Error carried to the C boundary as a status code.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define BIE_HIP(expr)                                                                   \
    do {                                                                                \
        hipError_t _e = (expr);                                                         \
        if (_e != hipSuccess)                                                           \
            throw ::bie::Error(_e == hipErrorOutOfMemory ? BIE_ENOMEM : BIE_EDEVICE,    \
                               std::string(#expr) + ": " + hipGetErrorString(_e));      \
    } while (0)

// Host-side RWG table and pair list (mesh.cpp).
struct Mesh {
    int64_t nv = 0, F = 0, N = 0;
    std::vector<double> V;          // nv x 3
    std::vector<int32_t> T;         // F x 3
    std::vector<int32_t> edges;     // N x 4: lo, hi, c+, c-
    std::vector<int32_t> slot_m;    // F x 3: RWG of local slot a (edge opposite vertex a)
    std::vector<int8_t> slot_s;     // F x 3: +1 on c+, -1 on c-
    std::vector<double> area;       // F
    std::vector<double> cent;       // F x 3
    std::vector<double> longest;    // F
    std::vector<int32_t> near;      // flagged pairs (p <= q), 2 per pair
};

// Builds and validates; throws Error(BIE_EMESH) for invalid meshes.
Mesh build_mesh(const double *verts, int64_t nv, const int32_t *tris, int64_t nt, double near_factor);

// SplitMix64 + Floyd row sample (rng.cpp).
std::vector<int64_t> rscc_rows(int64_t N, int64_t S, uint64_t seed);

// Per-triangle data uploaded for the fill kernels.  Quadrature points are
// stored relative to the triangle centroid; the centroid itself in FP64.
struct TriDev {
    double *cent = nullptr;     // F x 3
    double *loc = nullptr;      // F x 7 x 3   quadrature points - centroid
    double *vfree = nullptr;    // F x 3 x 3   free vertex of slot a - centroid
    double *verts = nullptr;    // F x 3 x 3   absolute vertex coordinates (singular kernel)
    double *area = nullptr;     // F
    int8_t *sgn = nullptr;      // F x 3
    int32_t *slot_m = nullptr;  // F x 3
    int32_t *edges = nullptr;   // N x 4
};

struct Workspace;  // solver workspaces (krylov.hip)
struct FastOp;     // fast operator (fast.hip)

// Packed symmetric storage of T (T = T^T exactly): only tiles (I, J) with
// I <= J of TB x TB entries are stored, each tile row-major and contiguous,
// tiles in row-major order over the upper triangle; entries beyond N are 0.
constexpr int TB = 64;
struct Packed {
    int64_t N = 0, nT = 0, ntiles = 0, nunits = 0;
    int32_t *units = nullptr;      // device, nunits x 3: (I, J0, J1) = tiles J0..J1-1 of tile row I
    int32_t *unit_ptr = nullptr;   // device, nT + 1: units of tile row I are unit_ptr[I] .. unit_ptr[I+1]-1
    int32_t *run_ptr = nullptr;    // device, nruns + 1: block b of the tile pass takes units run_ptr[b] ..
    int64_t nruns = 0;
    std::vector<int32_t> h_units, h_unit_ptr;   // host copies of the unit tables
    std::vector<int64_t> h_seg;
    int64_t *seg = nullptr;        // device, nT + 1: partial vectors of row block I occupy slots seg[I]..seg[I+1]-1
    int64_t nslots = 0;            // partial vectors per product vector (= seg[nT])
    void *part = nullptr;          // device partial sums of the product, sized for part_R vectors
    int64_t part_R = 0;
    size_t part_elem = 0;          // bytes per complex element of the partials buffer
    int unit_len = -1;             // tiles per work unit (0: balanced runs)
};
// One problem of a grouped (several-operator) packed product.
struct GProb {
    const void *Z;                 // packed matrix tiles (FP64 or FP32)
    int64_t N, nT, nslots;
    const int32_t *units, *unit_ptr;
    const int64_t *seg;
    int32_t c0, c1;                // its columns: c0 .. c1-1
};
// Columns of a grouped product (device tables indexed by column).
struct GCols {
    const int32_t *prob;   // problem of column c
    const int64_t *xoff;   // offset of its input vector (complex elements)
    const int64_t *yoff;   // offset of its output vector (and of the subtrahend)
    const int64_t *poff;   // offset of its partial vectors (64-entry vectors)
    int64_t xstep;         // input at xoff + xstep * N (basis vector xstep of a Krylov basis)
};
__host__ __device__ inline int64_t tile_of(int64_t I, int64_t J, int64_t nT)
{
    return I * nT - I * (I - 1) / 2 + (J - I);
}
// inverse of tile_of: linear index b -> (I, J), I <= J
__host__ __device__ inline void tile_decode(int64_t b, int64_t nT, int64_t &I, int64_t &J)
{
    const double n2 = 2.0 * double(nT) + 1.0;
    I = int64_t((n2 - sqrt(n2 * n2 - 8.0 * double(b))) * 0.5);
    if (I < 0) I = 0;
    if (I > nT - 1) I = nT - 1;
    while (I > 0 && tile_of(I, I, nT) > b) --I;
    while (I + 1 < nT && tile_of(I + 1, I + 1, nT) <= b) ++I;
    J = I + (b - tile_of(I, I, nT));
}

}  // namespace bie

struct bie_ws;   // learned warm start (warmstart.hip)
struct bie_far;    // single-level B-spline far field (bspline.hip)
struct bie_farml;  // multilevel B-spline far field (bspline.hip)

struct bie_op {
    int device = 0;
    double k = 0.0;
    int storage = BIE_C128;
    bie::Mesh mesh;
    bie::TriDev tri;
    void *Z64 = nullptr;   // packed symmetric tiles, complex128 (storage C128 or keep_fp64); star: T_A' = jk T_A
    void *Z32 = nullptr;   // packed symmetric tiles, complex64 (storage C64); star: T_A'
    bie::Packed pk;
    int star = 0;          // star-split operator: T = T_A' + Sigma V' Sigma^T
    void *V64 = nullptr, *V32 = nullptr;   // star: V' = V / (jk), packed F x F tiles (complex128 / complex64)
    bie::Packed pkv;       // tables of the F x F tiles
    void *star_buf = nullptr;   // star product scratch: u and w, star_R x F each (complex128 sized)
    int64_t star_R = 0;
    void *Abf = nullptr;          // split-BF16 matrix for the block product: hi plane, lo plane, [Mp][Kp]
    int64_t gemm_Mp = 0, gemm_Kp = 0;
    void *Bbf = nullptr;          // split-BF16 staging of the right-hand block, [NCp][Kp] x 2
    int64_t bstage_cols = 0;
    void *gemm_part = nullptr;    // split-K partial tiles, FP32 [KS][Mp][NCp]
    size_t gemm_part_elems = 0;
    void *A64 = nullptr;          // dense FP64 copy [d64_Mp][d64_Kp] (re/im interleaved) for the FP64 block product
    int64_t d64_Mp = 0, d64_Kp = 0;
    void *d64_part = nullptr;     // its split-K partial tiles, FP64
    size_t d64_part_elems = 0;
    bie::Workspace *ws = nullptr;
    void *bcache = nullptr;       // block GMRES buffers, arenas and side streams (bgmres.hip), kept between solves
    int pooled = 0;               // Z64 and A64 belong to the preconditioner setup pool (not freed with the op)
    bie::FastOp *fast = nullptr;  // fast operator: sparse near field + multilevel far field (fast.hip)
};

namespace bie {

// tune.cpp: the autotuner's registry of chosen launch shapes.
bool tune_enabled();
void tune_set_enabled(bool on);
bool tune_get(const std::string &key, std::vector<int> &v);
void tune_put(const std::string &key, const std::vector<int> &v);
std::string tune_report();
bool stream_capturing(hipStream_t s);
float time_launches(hipStream_t s, int reps, const std::function<void()> &fn);

// blas.hip: choose the packed product's work units for the operator by timing
// (once per matrix size and precision; no-op when tuning is off).
void tune_packed(bie_op *op, hipStream_t s);

// bgmres.hip: release the block solver's cached buffers of an operator.
void free_block_cache(bie_op *op);

// calderon.hip: the large transient buffers of preconditioner setups (slot 0 the
// fill's pair scratch, 1 the refined packed matrix, 2 its dense copy), kept
// between setups while any preconditioner lives.  Active only inside a setup.
bool setup_pool_active();
void *setup_pool_get(int slot, size_t bytes);

// calderon.hip: the multiplicative Calderon preconditioner.
bie_calderon *calderon_create(const bie_op *op, hipStream_t s);
void calderon_destroy(bie_calderon *pc);
const bie_op *calderon_operator(const bie_calderon *pc);
const bie_calderon_info &calderon_info(const bie_calderon *pc);
// The operator holding M (packed FP64 tiles), for products through the library's
// kernels; split: also its split-BF16 copy (made on first use).
bie_op *calderon_view(const bie_calderon *pc, bool split, hipStream_t s);
bie_op *calderon_view32(const bie_calderon *pc, hipStream_t s);
// The product T M as one dense operator (split-BF16 copy only), for the block
// products of the preconditioned inner solves; made by bie_calderon_create when
// the operator has a split-BF16 copy, else on first use.
bie_op *calderon_tm(const bie_calderon *pc, hipStream_t s);
// Y = M X (R complex128 vectors; columns with skip[c * sks] != 0 left untouched).
void calderon_apply(const bie_calderon *pc, const void *X, int64_t ldx, void *Y, int64_t ldy, int64_t R,
                    const int *skip, int64_t sks, hipStream_t s);
// Two R x N complex128 blocks owned by the preconditioner (grown on demand).
double2 *calderon_scratch(const bie_calderon *pc, int64_t R, hipStream_t s);
void add_into(int64_t n, const void *a, void *x, hipStream_t s);   // x += a (n complex)
void zero_into(int64_t n, void *x, hipStream_t s);

// fill.hip
constexpr int QPTS = 7;               // points of the triangle rule (Radon's degree-5 rule)
void quad_weights(double *w);         // its weights, relative to the triangle area
void upload_triangles(bie_op *op, hipStream_t s);
void fill_matrix(bie_op *op, bool fp64_regular, bool want64, bool want32, hipStream_t s);
void rhs_planewave(const bie_op *op, const double *dirs, const double *pols, int64_t R, void *B,
                   hipStream_t s);
// radiation vectors (R x M x 3 complex128), or with rcs the bistatic RCS (R x M double)
void farfield(const bie_op *op, const void *X, int64_t R, const double *obs, int64_t M, void *out, bool rcs,
              hipStream_t s);

// blas.hip: products with the packed symmetric matrix.
void packed_setup(Packed &pk, int64_t n);   // tables of the packed n x n tiles
// work units of U tiles along each tile row, and the partial-vector slots
void build_units(int64_t nT, int U, std::vector<int32_t> &units, std::vector<int32_t> &uptr,
                 std::vector<int64_t> &seg);
// Grouped packed product y_c = T_p(c) x_c (or b_c - that) for the columns of
// several problems: one tile launch over (problem, unit, group of G columns)
// items, each going through its columns, and one reduce launch over (column,
// row block) items.  mat64: FP64 tiles, else FP32.
// mfma: the matrix cores, at most 32 columns per item (FP32 tiles: FP32
// vectors and accumulation within a unit; FP64 tiles: FP64 throughout)
void grouped_product(bool mat64, const GProb *probs, const GCols &gc, const int32_t *items, int64_t nitems, int G,
                     const int32_t *ritems, int64_t nritems, const void *X, void *part, void *Y, const void *B,
                     const int *skip, int64_t sks, hipStream_t s, bool mfma = false);        // unit table (host -> device)
void packed_free(Packed &pk);
// Y = T X, T^H X (conj) or B - T X (B != NULL) for R vectors with the FP64
// (mat64) or FP32 matrix; vectors complex128 (vec64, FP64 accumulation) or
// complex64 (FP32 matrix only).
// mat: MAT64 (packed FP64), MAT32 (packed FP32), MATBF16 (split-BF16 block product,
// complex128 vectors only, no conj).
enum { MAT64 = 0, MAT32 = 1, MATBF16 = 2 };
void product(const bie_op *op, int mat, bool vec64, const void *X, int64_t ldx, void *Y, int64_t ldy,
             const void *B, int64_t ldb, int64_t R, const int *skip, int64_t sks, bool conj, hipStream_t s);
// Y = T X (or T^H X) with the packed matrix, partial sums in the library's
// static per-device scratch (no allocation); BIE_EINVAL when they do not fit.
void product_noalloc(const bie_op *op, bool vec64, const void *X, void *Y, int64_t R, bool conj, hipStream_t s);
// packed -> full row-major complex128
void unpack_c128(const bie_op *op, bool from64, void *dst, hipStream_t s);
// sampled rows of T x (complex128): out[r*S + i] = |b_i - (T x_r)_i|^2, i in rows[r*S ..]
void sampled_residual(const bie_op *op, const void *B, const void *X, int64_t R, int64_t S, const int64_t *rows,
                      double *out, const int *mask, hipStream_t s);
void convert_c128_to_c64(const void *src, void *dst, int64_t n, hipStream_t s);
void convert_c64_to_c128(const void *src, void *dst, int64_t n, hipStream_t s);
bool has_nonfinite(const void *x, int64_t n_doubles, hipStream_t s);
void prof_enable(bool enable);
void prof_read(int kernel, int64_t *launches, double *total_ms, int64_t *columns);
bool prof_active();
void prof_begin(int kernel, hipStream_t s, int64_t ncols);
void prof_end(int kernel, hipStream_t s);
// gemm.hip
void split_matrix(bie_op *op, hipStream_t s);
// split-BF16 operand of a general dense complex128 matrix (column-major, N = op->mesh.N)
void split_dense(bie_op *op, const void *A, hipStream_t s);
// vector element types of the block product's right-hand block
enum { VEC_C128 = 0, VEC_C64 = 1, VEC_F16 = 2 };
// complex value as two FP16 (storage of the FP16 Krylov basis)
struct alignas(4) c32h {
    _Float16 x, y;
};
void gemm_product(const bie_op *op, const void *X, int64_t ldx, int vtype, void *Y, int64_t ldy, const void *Bsub,
                  int64_t ldb, int64_t R, const int *cols, hipStream_t s, int terms = 3);
void dense64_setup(bie_op *op, hipStream_t s);
void gemm64_product(const bie_op *op, const void *X, int64_t ldx, void *Y, int64_t ldy, const void *Bsub,
                    int64_t ldb, int64_t R, const int *cols, hipStream_t s);

// warmstart.hip
bie_ws *ws_train(const bie_op *op, const double *feats, const double *pols, const void *X, int64_t S,
                 const bie_ws_opts &o, hipStream_t s);
double ws_fit(bie_ws *w, const double *feats, const double *pols, const float *targets, int64_t S, int epochs,
              int batch, double lr_max, double lr_min, uint64_t seed, hipStream_t s);
void ws_predict(bie_ws *w, const double *feats, const double *pols, int64_t R, const void *B, void *X0, int *used,
                hipStream_t s);
double ws_loss_grad(bie_ws *w, const double *feats, const double *pols, const float *targets, int64_t R,
                    float *grad_host, hipStream_t s);
void ws_forward(bie_ws *w, const double *feats, int64_t R, float *out_host, hipStream_t s);
bie_ws *ws_create_untrained(const bie_op *op, int K, int H, uint64_t seed, int pol_model);
void ws_params(bie_ws *w, float *host, bool set);
void ws_basis(const bie_ws *w, void *U, hipStream_t s);
void ws_save(const bie_ws *w, const char *path);
bie_ws *ws_load(const bie_op *op, const char *path);
void ws_destroy(bie_ws *w);
void ws_info(const bie_ws *w, int64_t *K, int64_t *H, int64_t *nparams, double *scale, double *loss, double *sigma);

// bspline.hip
bie_far *far_create(const bie_op *op, double a, int s, int p, hipStream_t st);
void far_apply(bie_far *f, const void *X, void *Y, int64_t R, hipStream_t st);
void far_info(const bie_far *f, bie_far_info *info);
void far_boxes(const bie_far *f, int32_t *out);
void far_destroy(bie_far *f);
bie_farml *farml_create(const bie_op *op, double a, int levels, int s, int p, hipStream_t st);
void farml_apply(bie_farml *f, const void *X, void *Y, int64_t R, hipStream_t st);
void farml_level_info(const bie_farml *f, int level, bie_far_info *info);
void farml_destroy(bie_farml *f);
void farml_leaves(const bie_farml *f, std::vector<int32_t> &box_of, std::vector<int32_t> &ijk);
// fill.hip: the flagged pairs' local blocks, compact (18 doubles per pair)
void singular_blocks(const bie_op *op, const int32_t *pairs, int64_t npairs, double *out, hipStream_t s);
// fast.hip
void fast_setup(bie_op *op, double box, int levels, int s, int p, hipStream_t st);
void fast_product(const bie_op *op, const void *X, int64_t ldx, void *Y, int64_t ldy, const void *B, int64_t ldb,
                  int64_t R, hipStream_t st);
void fast_info(const bie_op *op, bie_fast_info *info);
void fast_destroy(FastOp *f);

// krylov.hip
int solve_batch(const bie_op *const *ops, const bie_calderon *const *pcs, int64_t P, const void *const *B,
                void *const *X, const int64_t *R, const bie_solve_opts &o, bie_solve_stat *stats, hipStream_t s);
void batch_config(int unit, int graph, int mfma);
int batch_unit_chosen(const bie_op *const *ops, int64_t P, const int64_t *R);
// grouped product of several operators outside a solve (mat 0: FP64 tiles, 1:
// FP32 tiles, 2: FP32 tiles on the matrix cores, 3: FP64 tiles on the matrix
// cores; unit/G 0: defaults)
void batch_apply(const bie_op *const *ops, int64_t P, const void *const *X, void *const *Y, const int64_t *R,
                 int mat, int unit, int G, hipStream_t s);
int solve(const bie_op *op, const void *B, void *X, int64_t R, const bie_solve_opts &o,
          bie_solve_stat *stats, hipStream_t s);
void free_workspace(bie_op *op);
// bgmres.hip
int solve_block(const bie_op *op, const void *B, void *X, int64_t R, const bie_solve_opts &o,
                bie_solve_stat *stats, hipStream_t s);

}  // namespace bie
