// C ABI of libbie (include/bie.h): argument checks, error codes, dispatch.
#include <cmath>
#include <cstring>
#include <utility>
#include <string>

#include "bie_internal.hpp"

namespace {
thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

template <typename F>
int guarded(F &&f)
{
    try {
        return f();
    } catch (const bie::Error &e) {
        return fail(e.code, e.what());
    } catch (const std::bad_alloc &) {
        return fail(BIE_ENOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(BIE_EDEVICE, e.what());
    } catch (...) {
        return fail(BIE_EDEVICE, "unknown error");
    }
}

hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

void destroy_op(bie_op *op)
{
    if (!op) return;
    if (op->fast) bie::fast_destroy(op->fast);
    bie::free_workspace(op);
    bie::free_block_cache(op);
    bie::packed_free(op->pk);
    bie::packed_free(op->pkv);
    void *ptrs[] = { op->pooled ? nullptr : op->Z64, op->Z32, op->V64, op->V32, op->star_buf, op->Abf, op->Bbf,
                     op->gemm_part, op->pooled ? nullptr : op->A64,
                     op->d64_part, op->tri.cent, op->tri.loc, op->tri.vfree, op->tri.verts, op->tri.area, op->tri.sgn,
                     op->tri.slot_m, op->tri.edges };
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete op;
}
}  // namespace

extern "C" {

const char *bie_last_error(void) { return g_err.c_str(); }

int bie_op_create(const double *verts, int64_t nv, const int32_t *tris, int64_t nt, double k,
                  const bie_fill_opts *opts, void *stream, bie_op **out)
{
    return guarded([&]() -> int {
        if (!out) return fail(BIE_EINVAL, "out is NULL");
        *out = nullptr;
        if (!verts || !tris) return fail(BIE_EINVAL, "NULL mesh array");
        if (!(k > 0.0) || !std::isfinite(k)) return fail(BIE_EINVAL, "wavenumber must be positive and finite");
        bie_fill_opts o{ BIE_C128, 2.0, 0, 0 };
        if (opts) o = *opts;
        if (o.storage != BIE_C128 && o.storage != BIE_C64 && o.storage != BIE_SPLIT_BF16)
            return fail(BIE_EINVAL, "unknown storage");
        if (o.star != 0 && o.star != 1) return fail(BIE_EINVAL, "star must be 0 or 1");
        if (o.star && o.storage == BIE_SPLIT_BF16) return fail(BIE_EINVAL, "the star-split form has no split-BF16 copy");
        if (!(o.near_factor >= 0.0)) return fail(BIE_EINVAL, "near_factor must be >= 0");
        bie::Mesh mesh = bie::build_mesh(verts, nv, tris, nt, o.near_factor);   // host only: EMESH first
        bie_op *op = new bie_op();
        try {
            op->mesh = std::move(mesh);
            BIE_HIP(hipGetDevice(&op->device));
            op->k = k;
            op->storage = o.storage;
            op->star = o.star;
            hipStream_t s = as_stream(stream);
            bie::upload_triangles(op, s);
            bie::packed_setup(op->pk, op->mesh.N);
            if (op->star) bie::packed_setup(op->pkv, op->mesh.F);
            const size_t tile_elems = size_t(op->pk.ntiles) * bie::TB * bie::TB;
            const size_t vtile_elems = op->star ? size_t(op->pkv.ntiles) * bie::TB * bie::TB : 0;
            const bool want64 = o.storage == BIE_C128 || o.storage == BIE_SPLIT_BF16 || o.keep_fp64;
            const bool want32 = o.storage == BIE_C64;
            if (want64 && bie::setup_pool_active()) {   // the refined mesh of a preconditioner setup
                op->pooled = 1;
                op->Z64 = bie::setup_pool_get(1, tile_elems * 16);
            } else if (want64) {
                BIE_HIP(hipMalloc(&op->Z64, tile_elems * 16));
            }
            if (want32) BIE_HIP(hipMalloc(&op->Z32, tile_elems * 8));
            if (want64 && op->star) BIE_HIP(hipMalloc(&op->V64, vtile_elems * 16));
            if (want32 && op->star) BIE_HIP(hipMalloc(&op->V32, vtile_elems * 8));
            if (o.storage == BIE_C128) {
                bie::fill_matrix(op, true, true, false, s);
            } else if (o.storage == BIE_SPLIT_BF16) {
                bie::fill_matrix(op, true, true, false, s);
                bie::split_matrix(op, s);
            } else if (o.keep_fp64) {
                // FP64 fill; the FP32 matrix is its rounding (the best FP32 representation)
                bie::fill_matrix(op, true, true, false, s);
                bie::convert_c128_to_c64(op->Z64, op->Z32, int64_t(tile_elems), s);
                if (op->star) bie::convert_c128_to_c64(op->V64, op->V32, int64_t(vtile_elems), s);
                BIE_HIP(hipStreamSynchronize(s));
            } else {
                bie::fill_matrix(op, false, false, true, s);          // FP32 regular, FP64 singular
            }
            if (!bie::setup_pool_active()) bie::tune_packed(op, s);   // work units of the packed product
        } catch (...) {
            destroy_op(op);
            throw;
        }
        *out = op;
        return BIE_OK;
    });
}

int bie_op_create_fast(const double *verts, int64_t nv, const int32_t *tris, int64_t nt, double k,
                       const bie_fast_opts *opts, void *stream, bie_op **out)
{
    return guarded([&]() -> int {
        if (!out) return fail(BIE_EINVAL, "out is NULL");
        *out = nullptr;
        if (!verts || !tris || !opts) return fail(BIE_EINVAL, "NULL argument");
        if (!(k > 0.0) || !std::isfinite(k)) return fail(BIE_EINVAL, "wavenumber must be positive and finite");
        if (!(opts->near_factor >= 0.0)) return fail(BIE_EINVAL, "near_factor must be >= 0");
        bie::Mesh mesh = bie::build_mesh(verts, nv, tris, nt, opts->near_factor);   // host only: EMESH first
        bie_op *op = new bie_op();
        try {
            op->mesh = std::move(mesh);
            BIE_HIP(hipGetDevice(&op->device));
            op->k = k;
            op->storage = BIE_C128;
            hipStream_t s = as_stream(stream);
            bie::upload_triangles(op, s);
            bie::fast_setup(op, opts->box, opts->levels, opts->s, opts->p, s);
        } catch (...) {
            destroy_op(op);
            throw;
        }
        *out = op;
        return BIE_OK;
    });
}

int bie_op_fast_info(const bie_op *op, bie_fast_info *info)
{
    if (!op || !info) return fail(BIE_EINVAL, "NULL argument");
    if (!op->fast) return fail(BIE_EINVAL, "not a fast operator");
    bie::fast_info(op, info);
    return BIE_OK;
}

void bie_op_destroy(bie_op *op) { destroy_op(op); }

int64_t bie_op_n(const bie_op *op) { return op ? op->mesh.N : int64_t(BIE_EINVAL); }

int bie_op_edges(const bie_op *op, int32_t *out)
{
    if (!op || !out) return fail(BIE_EINVAL, "NULL argument");
    std::memcpy(out, op->mesh.edges.data(), op->mesh.edges.size() * sizeof(int32_t));
    return BIE_OK;
}

int64_t bie_op_near_pairs(const bie_op *op, int32_t *out, int64_t cap)
{
    if (!op) return fail(BIE_EINVAL, "NULL operator");
    const int64_t n = int64_t(op->mesh.near.size() / 2);
    if (out && cap > 0) std::memcpy(out, op->mesh.near.data(), size_t(std::min(n, cap)) * 2 * sizeof(int32_t));
    return n;
}

int bie_op_matrix(const bie_op *op, void *dst, int dtype, void *stream)
{
    return guarded([&]() -> int {
        if (!op || !dst) return fail(BIE_EINVAL, "NULL argument");
        if (op->star) return fail(BIE_EINVAL, "a star-split operator holds no assembled matrix");
        if (op->fast) return fail(BIE_EINVAL, "a fast operator holds no dense matrix");
        hipStream_t s = as_stream(stream);
        if (dtype == BIE_C128) {
            bie::unpack_c128(op, op->Z64 != nullptr, dst, s);
        } else if (dtype == BIE_C64) {
            if (!op->Z32) return fail(BIE_EINVAL, "no FP32 matrix stored");
            void *tmp = nullptr;
            const int64_t NN = op->mesh.N * op->mesh.N;
            BIE_HIP(hipMalloc(&tmp, size_t(NN) * 16));
            bie::unpack_c128(op, false, tmp, s);
            bie::convert_c128_to_c64(tmp, dst, NN, s);
            BIE_HIP(hipStreamSynchronize(s));
            (void)hipFree(tmp);
        } else {
            return fail(BIE_EINVAL, "unknown dtype");
        }
        BIE_HIP(hipStreamSynchronize(s));
        return BIE_OK;
    });
}

int bie_rhs_planewave(const bie_op *op, const double *dirs, const double *pols, int64_t R, void *B, void *stream)
{
    return guarded([&]() -> int {
        if (!op || !dirs || !pols || !B) return fail(BIE_EINVAL, "NULL argument");
        if (R < 0 || R > 65535) return fail(BIE_EINVAL, "R out of range (0..65535)");
        if (R == 0) return BIE_OK;
        for (int64_t i = 0; i < 3 * R; ++i)
            if (!std::isfinite(dirs[i]) || !std::isfinite(pols[i])) return fail(BIE_ENUMERIC, "non-finite direction");
        bie::rhs_planewave(op, dirs, pols, R, B, as_stream(stream));
        return BIE_OK;
    });
}

int bie_apply(const bie_op *op, const void *X, void *Y, int64_t R, int vec, int conj, void *stream)
{
    return guarded([&]() -> int {
        if (!op || !X || !Y) return fail(BIE_EINVAL, "NULL argument");
        if (R < 0 || R > 65535) return fail(BIE_EINVAL, "R out of range (0..65535)");
        if (R == 0) return BIE_OK;
        const int64_t N = op->mesh.N;
        hipStream_t s = as_stream(stream);
        if (op->fast) {
            if (vec != BIE_C128 || conj) return fail(BIE_EINVAL, "the fast operator takes complex128 vectors, no conjugate");
            bie::fast_product(op, X, N, Y, N, nullptr, 0, R, s);
            return BIE_OK;
        }
        if (vec == BIE_C128) {
            // FP64 matrix if stored, else the FP32 matrix with FP64 accumulation
            bie::product(op, op->Z64 ? bie::MAT64 : bie::MAT32, true, X, N, Y, N, nullptr, 0, R, nullptr, 1, conj != 0,
                         s);
        } else if (vec == BIE_C64) {
            if (!op->Z32) return fail(BIE_EINVAL, "complex64 vectors need BIE_C64 storage");
            bie::product(op, bie::MAT32, false, X, N, Y, N, nullptr, 0, R, nullptr, 1, conj != 0, s);
        } else if (vec == BIE_SPLIT_BF16) {
            // complex128 vectors through the split-BF16 block product
            if (!op->Abf) return fail(BIE_EINVAL, "no split-BF16 matrix stored");
            if (conj) return fail(BIE_EINVAL, "the block product has no conjugate form");
            bie::product(op, bie::MATBF16, true, X, N, Y, N, nullptr, 0, R, nullptr, 1, false, s);
        } else if (vec == BIE_APPLY_F64_BLOCK) {
            if (!op->Z64) return fail(BIE_EINVAL, "the FP64 block product needs the FP64 matrix");
            if (op->star) return fail(BIE_EINVAL, "no FP64 block product for a star-split operator");
            if (conj) return fail(BIE_EINVAL, "the block product has no conjugate form");
            bie::gemm64_product(op, X, N, Y, N, nullptr, 0, R, nullptr, s);
        } else {
            return fail(BIE_EINVAL, "unknown vector dtype");
        }
        return BIE_OK;
    });
}

int bie_apply_noalloc(const bie_op *op, const void *X, void *Y, int64_t R, int vec, int conj, void *stream)
{
    return guarded([&]() -> int {
        if (!op || !X || !Y) return fail(BIE_EINVAL, "NULL argument");
        if (R < 0 || R > 65535) return fail(BIE_EINVAL, "R out of range (0..65535)");
        if (R == 0) return BIE_OK;
        if (vec != BIE_C128 && vec != BIE_C64)
            return fail(BIE_EINVAL, "the allocation-free product takes complex128 or complex64 vectors");
        if (op->fast) return fail(BIE_EINVAL, "the allocation-free product takes an operator with a stored matrix");
        bie::product_noalloc(op, vec == BIE_C128, X, Y, R, conj != 0, as_stream(stream));
        return BIE_OK;
    });
}

int bie_solve(const bie_op *op, const void *B, void *X, int64_t R, const bie_solve_opts *opts,
              bie_solve_stat *stats, void *stream)
{
    return guarded([&]() -> int {
        if (!op || !B || !X) return fail(BIE_EINVAL, "NULL argument");
        if (R < 0 || R > 4096) return fail(BIE_EINVAL, "R out of range (0..4096)");
        if (R == 0) return BIE_OK;
        bie_solve_opts o{ BIE_GMRES, 30, 1e-6, 10000, BIE_SCC, 512, 1234, 0, 0, 0.0, 0, 0, 0, 0, nullptr };
        if (opts) o = *opts;
        if (o.method != BIE_GMRES && o.method != BIE_CGNR && o.method != BIE_BGMRES)
            return fail(BIE_EINVAL, "unknown method");
        if (o.crit != BIE_SCC && o.crit != BIE_RSCC && o.crit != BIE_CCC) return fail(BIE_EINVAL, "unknown criterion");
        if (o.precision == 1 && o.crit != BIE_SCC)
            return fail(BIE_EINVAL, "mixed precision decides convergence by the standard criterion");
        if ((o.method == BIE_GMRES || o.method == BIE_BGMRES) && (o.restart < 1 || o.restart > 64))
            return fail(BIE_EINVAL, "restart must be 1..64");
        if (o.method == BIE_BGMRES) {
            if (o.block < 0 || o.block > 32) return fail(BIE_EINVAL, "block must be 0..32");
            if (o.crit != BIE_SCC) return fail(BIE_EINVAL, "block GMRES decides convergence by the standard criterion");
            if (op->star) return fail(BIE_EINVAL, "block GMRES needs an assembled operator");
            if (o.precision == 1 && !op->Abf)
                return fail(BIE_EINVAL, "mixed-precision block GMRES needs split-BF16 storage");
            if (!op->Z64) return fail(BIE_EINVAL, "block GMRES needs the FP64 matrix");
        }
        if (o.calderon) {
            if (o.method == BIE_CGNR || (o.method == BIE_GMRES && o.precision != 0))
                return fail(BIE_EINVAL, "the Calderon preconditioner takes GMRES with precision 0 or block GMRES");
            if (bie::calderon_operator(o.calderon) != op)
                return fail(BIE_EINVAL, "the Calderon preconditioner was built for another operator");
        }
        if (!(o.tol > 0.0)) return fail(BIE_EINVAL, "tol must be > 0");
        if (o.max_mvp < 1) return fail(BIE_EINVAL, "max_mvp must be >= 1");
        if (o.rscc_rows < 1) return fail(BIE_EINVAL, "rscc_rows must be >= 1");
        if (o.precision != 0 && o.precision != 1) return fail(BIE_EINVAL, "precision must be 0 or 1");
        if (!(o.inner_tol >= 0.0 && o.inner_tol < 1.0)) return fail(BIE_EINVAL, "inner_tol must be in [0, 1)");
        if (o.slots < 0) return fail(BIE_EINVAL, "slots must be >= 0");
        if (o.use_x0 < 0 || o.use_x0 > 2) return fail(BIE_EINVAL, "use_x0 must be 0, 1 or 2");
        if (o.inner_terms != 0 && o.inner_terms != 2 && o.inner_terms != 3)
            return fail(BIE_EINVAL, "inner_terms must be 0, 2 or 3");
        if (o.basis != 0 && o.basis != 1) return fail(BIE_EINVAL, "basis must be 0 or 1");
        if (op->star && o.crit != BIE_SCC)
            return fail(BIE_EINVAL, "the random-sampling criterion needs assembled rows (not a star-split operator)");
        if (o.basis == 1 && (o.precision != 1 || !op->Abf))
            return fail(BIE_EINVAL, "the FP16 basis is for mixed precision with split-BF16 storage");
        const int64_t N = op->mesh.N;
        hipStream_t s = as_stream(stream);
        if (bie::has_nonfinite(B, 2 * R * N, s)) return fail(BIE_ENUMERIC, "non-finite right-hand side");
        if (o.use_x0 && bie::has_nonfinite(X, 2 * R * N, s)) return fail(BIE_ENUMERIC, "non-finite initial guess");
        const int rc = o.method == BIE_BGMRES ? bie::solve_block(op, B, X, R, o, stats, s)
                                              : bie::solve(op, B, X, R, o, stats, s);
        if (rc == BIE_NOT_CONVERGED) g_err = "not converged within max_mvp";
        return rc;
    });
}

int bie_calderon_create(const bie_op *op, void *stream, bie_calderon **out)
{
    return guarded([&]() -> int {
        if (!op || !out) return fail(BIE_EINVAL, "NULL argument");
        *out = nullptr;
        if (op->fast) return fail(BIE_EINVAL, "the Calderon preconditioner needs an operator with a stored matrix");
        *out = bie::calderon_create(op, as_stream(stream));
        return BIE_OK;
    });
}

int bie_calderon_apply(const bie_calderon *pc, const void *X, void *Y, int64_t R, void *stream)
{
    return guarded([&]() -> int {
        if (!pc || !X || !Y) return fail(BIE_EINVAL, "NULL argument");
        if (R < 0 || R > 4096) return fail(BIE_EINVAL, "R out of range (0..4096)");
        if (R == 0) return BIE_OK;
        if (X == Y) return fail(BIE_EINVAL, "X and Y must not alias");
        const bie_calderon_info &info = bie::calderon_info(pc);
        if (R >= 8)   // many vectors: the FP64 matrix cores
            bie::gemm64_product(bie::calderon_view(pc, false, as_stream(stream)), X, info.N, Y, info.N, nullptr, 0, R,
                                nullptr, as_stream(stream));
        else
            bie::calderon_apply(pc, X, info.N, Y, info.N, R, nullptr, 1, as_stream(stream));
        return BIE_OK;
    });
}

int bie_calderon_get_info(const bie_calderon *pc, bie_calderon_info *info)
{
    if (!pc || !info) return fail(BIE_EINVAL, "NULL argument");
    *info = bie::calderon_info(pc);
    return BIE_OK;
}

void bie_calderon_destroy(bie_calderon *pc) { bie::calderon_destroy(pc); }

int bie_batch_apply(const bie_op *const *ops, int64_t nops, const void *const *X, void *const *Y, const int64_t *R,
                    int mat, int unit_tiles, int cols_per_item, void *stream)
{
    return guarded([&]() -> int {
        if (!ops || !X || !Y || !R) return fail(BIE_EINVAL, "NULL argument");
        if (nops < 1 || nops > 4096) return fail(BIE_EINVAL, "nops out of range (1..4096)");
        int64_t total = 0;
        for (int64_t p = 0; p < nops; ++p) {
            if (!ops[p]) return fail(BIE_EINVAL, "NULL operator");
            if (ops[p]->star || ops[p]->fast) return fail(BIE_EINVAL, "grouped products take assembled dense operators");
            if (R[p] < 0 || R[p] > 4096) return fail(BIE_EINVAL, "R out of range (0..4096)");
            if (R[p] > 0 && (!X[p] || !Y[p])) return fail(BIE_EINVAL, "NULL vector pointer");
            total += R[p];
        }
        if (total > 65535) return fail(BIE_EINVAL, "at most 65535 columns per call");
        bie::batch_apply(ops, nops, X, Y, R, mat, unit_tiles, cols_per_item, as_stream(stream));
        return BIE_OK;
    });
}

int bie_batch_solve_pc(const bie_op *const *ops, const bie_calderon *const *pcs, int64_t nops,
                       const void *const *B, void *const *X, const int64_t *R, const bie_solve_opts *opts,
                       bie_solve_stat *stats, void *stream)
{
    return guarded([&]() -> int {
        if (!ops || !B || !X || !R) return fail(BIE_EINVAL, "NULL argument");
        if (nops < 1 || nops > 4096) return fail(BIE_EINVAL, "nops out of range (1..4096)");
        bie_solve_opts o{ BIE_GMRES, 30, 1e-6, 10000, BIE_SCC, 512, 1234, 0, 0, 0.0, 0, 0, 0, 0, nullptr };
        if (opts) o = *opts;
        if (o.method != BIE_GMRES || (o.precision != 0 && o.precision != 1) || o.basis != 0)
            return fail(BIE_EINVAL, "batched solves take GMRES with precision 0 or 1");
        if (o.crit != BIE_SCC && o.crit != BIE_RSCC && o.crit != BIE_CCC) return fail(BIE_EINVAL, "unknown criterion");
        if (o.crit != BIE_SCC && o.rscc_rows < 1) return fail(BIE_EINVAL, "rscc_rows must be >= 1");
        if (o.calderon) return fail(BIE_EINVAL, "batched solves take their preconditioners per operator (pcs)");
        if (o.restart < 1 || o.restart > 64) return fail(BIE_EINVAL, "restart must be 1..64");
        if (!(o.tol > 0.0)) return fail(BIE_EINVAL, "tol must be > 0");
        if (o.max_mvp < 1) return fail(BIE_EINVAL, "max_mvp must be >= 1");
        if (o.use_x0 < 0 || o.use_x0 > 2) return fail(BIE_EINVAL, "use_x0 must be 0, 1 or 2");
        hipStream_t s = as_stream(stream);
        int64_t total = 0;
        for (int64_t p = 0; p < nops; ++p) {
            if (!ops[p]) return fail(BIE_EINVAL, "NULL operator");
            if (ops[p]->star) return fail(BIE_EINVAL, "batched solves take assembled operators");
            if (pcs && !pcs[p]) return fail(BIE_EINVAL, "NULL preconditioner");
            if (pcs && bie::calderon_operator(pcs[p]) != ops[p])
                return fail(BIE_EINVAL, "a preconditioner was built for another operator");
            if (R[p] < 0 || R[p] > 4096) return fail(BIE_EINVAL, "R out of range (0..4096)");
            if (R[p] > 0 && (!B[p] || !X[p])) return fail(BIE_EINVAL, "NULL vector pointer");
            total += R[p];
            const int64_t n2 = 2 * R[p] * ops[p]->mesh.N;
            if (R[p] > 0 && bie::has_nonfinite(B[p], n2, s)) return fail(BIE_ENUMERIC, "non-finite right-hand side");
            if (R[p] > 0 && o.use_x0 && bie::has_nonfinite(X[p], n2, s))
                return fail(BIE_ENUMERIC, "non-finite initial guess");
        }
        if (total == 0) return BIE_OK;
        if (total > 65535) return fail(BIE_EINVAL, "at most 65535 right-hand sides per batch");
        const int rc = bie::solve_batch(ops, pcs, nops, B, X, R, o, stats, s);
        if (rc == BIE_NOT_CONVERGED) g_err = "not converged within max_mvp";
        return rc;
    });
}

int bie_batch_solve(const bie_op *const *ops, int64_t nops, const void *const *B, void *const *X,
                    const int64_t *R, const bie_solve_opts *opts, bie_solve_stat *stats, void *stream)
{
    return bie_batch_solve_pc(ops, nullptr, nops, B, X, R, opts, stats, stream);
}

int bie_batch_config(int unit_tiles, int use_graph, int matrix_cores)
{
    return guarded([&]() -> int {
        if (unit_tiles < -1 || unit_tiles > 64) return fail(BIE_EINVAL, "unit_tiles must be -1..64");
        bie::batch_config(unit_tiles, use_graph != 0, matrix_cores != 0);
        return BIE_OK;
    });
}

int bie_batch_tuned(const bie_op *const *ops, int64_t nops, const int64_t *R)
{
    return guarded([&]() -> int {
        if (!ops || !R || nops < 1) return fail(BIE_EINVAL, "bad arguments");
        return bie::batch_unit_chosen(ops, nops, R);
    });
}

int bie_farfield(const bie_op *op, const void *X, int64_t R, const double *obs, int64_t M, void *F, void *stream)
{
    return guarded([&]() -> int {
        if (!op || !X || !obs || !F) return fail(BIE_EINVAL, "NULL argument");
        if (R < 0 || R > 65535 || M < 0 || M > (int64_t(1) << 31)) return fail(BIE_EINVAL, "size out of range");
        if (R == 0 || M == 0) return BIE_OK;
        bie::farfield(op, X, R, obs, M, F, false, as_stream(stream));
        return BIE_OK;
    });
}

int bie_rcs(const bie_op *op, const void *X, int64_t R, const double *obs, int64_t M, double *sigma, void *stream)
{
    return guarded([&]() -> int {
        if (!op || !X || !obs || !sigma) return fail(BIE_EINVAL, "NULL argument");
        if (R < 0 || R > 65535 || M < 0 || M > (int64_t(1) << 31)) return fail(BIE_EINVAL, "size out of range");
        for (int64_t m = 0; m < M; ++m) {
            const double n2 = obs[3 * m] * obs[3 * m] + obs[3 * m + 1] * obs[3 * m + 1] + obs[3 * m + 2] * obs[3 * m + 2];
            if (!(std::fabs(n2 - 1.0) <= 1e-9)) return fail(BIE_EINVAL, "observation directions must be unit vectors");
        }
        if (R == 0 || M == 0) return BIE_OK;
        bie::farfield(op, X, R, obs, M, sigma, true, as_stream(stream));
        return BIE_OK;
    });
}

int bie_far_create(const bie_op *op, const bie_far_opts *opts, void *stream, bie_far **out)
{
    return guarded([&]() -> int {
        if (!op || !opts || !out) return fail(BIE_EINVAL, "NULL argument");
        *out = nullptr;
        *out = bie::far_create(op, opts->box, opts->s, opts->p, as_stream(stream));
        return BIE_OK;
    });
}

int bie_far_apply(bie_far *far, const void *X, void *Y, int64_t R, void *stream)
{
    return guarded([&]() -> int {
        if (!far || !X || !Y) return fail(BIE_EINVAL, "NULL argument");
        if (R < 0 || R > 64) return fail(BIE_EINVAL, "R out of range (0..64)");
        if (R == 0) return BIE_OK;
        bie::far_apply(far, X, Y, R, as_stream(stream));
        return BIE_OK;
    });
}

int bie_farml_create(const bie_op *op, const bie_farml_opts *opts, void *stream, bie_farml **out)
{
    return guarded([&]() -> int {
        if (!op || !opts || !out) return fail(BIE_EINVAL, "NULL argument");
        *out = nullptr;
        *out = bie::farml_create(op, opts->box, opts->levels, opts->s, opts->p, as_stream(stream));
        return BIE_OK;
    });
}

int bie_farml_apply(bie_farml *f, const void *X, void *Y, int64_t R, void *stream)
{
    return guarded([&]() -> int {
        if (!f || !X || !Y) return fail(BIE_EINVAL, "NULL argument");
        if (R < 0 || R > 64) return fail(BIE_EINVAL, "R out of range (0..64)");
        if (R == 0) return BIE_OK;
        bie::farml_apply(f, X, Y, R, as_stream(stream));
        return BIE_OK;
    });
}

int bie_farml_level_info(const bie_farml *f, int level, bie_far_info *info)
{
    return guarded([&]() -> int {
        if (!f || !info) return fail(BIE_EINVAL, "NULL argument");
        bie::farml_level_info(f, level, info);
        return BIE_OK;
    });
}

void bie_farml_destroy(bie_farml *f) { bie::farml_destroy(f); }

int bie_far_get_info(const bie_far *far, bie_far_info *info)
{
    if (!far || !info) return fail(BIE_EINVAL, "NULL argument");
    bie::far_info(far, info);
    return BIE_OK;
}

int bie_far_boxes(const bie_far *far, int32_t *out)
{
    if (!far || !out) return fail(BIE_EINVAL, "NULL argument");
    bie::far_boxes(far, out);
    return BIE_OK;
}

void bie_far_destroy(bie_far *far)
{
    if (far) bie::far_destroy(far);
}

int bie_ws_train(const bie_op *op, const double *feats, const double *pols, const void *X, int64_t S,
                 const bie_ws_opts *opts, void *stream, bie_ws **out)
{
    return guarded([&]() -> int {
        if (!op || !feats || !X || !out) return fail(BIE_EINVAL, "NULL argument");
        if (op->star) return fail(BIE_EINVAL, "the warm start takes an assembled operator");
        *out = nullptr;
        bie_ws_opts o{ 256, 512, 3000, 256, 1e-3, 1e-5, 555, 32, 2, 0 };
        if (opts) o = *opts;
        if (S < 2 || o.pod_rank < 1 || o.pod_rank > S || o.hidden < 1 || o.hidden > 4096 || o.epochs < 0 ||
            o.batch < 1 || o.oversample < 0 || o.power_iters < 0 || !(o.lr_max > 0.0) || !(o.lr_min >= 0.0) ||
            (o.pol_model != 0 && o.pol_model != 1) || (o.pol_model == 1 && !pols))
            return fail(BIE_EINVAL, "bad warm-start options");
        for (int64_t i = 0; i < 4 * S; ++i)
            if (!std::isfinite(feats[i])) return fail(BIE_ENUMERIC, "non-finite feature");
        *out = bie::ws_train(op, feats, pols, X, S, o, as_stream(stream));
        return BIE_OK;
    });
}

int bie_ws_fit(bie_ws *ws, const double *feats, const double *pols, const float *targets, int64_t S, int epochs,
               int batch, double lr_max, double lr_min, uint64_t seed, double *final_loss, void *stream)
{
    return guarded([&]() -> int {
        if (!ws || !feats || !targets) return fail(BIE_EINVAL, "NULL argument");
        if (S < 1 || S > (int64_t(1) << 31) || epochs < 0 || batch < 1 || !(lr_max > 0.0) || !(lr_min >= 0.0))
            return fail(BIE_EINVAL, "bad training options");
        for (int64_t i = 0; i < 4 * S; ++i)
            if (!std::isfinite(feats[i])) return fail(BIE_ENUMERIC, "non-finite feature");
        const double l = bie::ws_fit(ws, feats, pols, targets, S, epochs, batch, lr_max, lr_min, seed,
                                     as_stream(stream));
        if (final_loss) *final_loss = l;
        return BIE_OK;
    });
}

int bie_ws_predict(bie_ws *ws, const double *feats, const double *pols, int64_t R, const void *B, void *X0,
                   int32_t *used, void *stream)
{
    return guarded([&]() -> int {
        if (!ws || !feats || !X0) return fail(BIE_EINVAL, "NULL argument");
        if (R < 1 || R > 65535) return fail(BIE_EINVAL, "R out of range");
        bie::ws_predict(ws, feats, pols, R, B, X0, used, as_stream(stream));
        return BIE_OK;
    });
}

int bie_ws_info(const bie_ws *ws, int64_t *K, int64_t *H, int64_t *np, double *scale, double *loss, double *sigma)
{
    if (!ws) return fail(BIE_EINVAL, "NULL warm start");
    bie::ws_info(ws, K, H, np, scale, loss, sigma);
    return BIE_OK;
}

int bie_ws_basis(const bie_ws *ws, void *U, void *stream)
{
    return guarded([&]() -> int {
        if (!ws || !U) return fail(BIE_EINVAL, "NULL argument");
        bie::ws_basis(ws, U, as_stream(stream));
        return BIE_OK;
    });
}

int bie_ws_params(bie_ws *ws, float *host, int set)
{
    return guarded([&]() -> int {
        if (!ws || !host) return fail(BIE_EINVAL, "NULL argument");
        bie::ws_params(ws, host, set != 0);
        return BIE_OK;
    });
}

int bie_ws_loss_grad(bie_ws *ws, const double *feats, const double *pols, const float *targets, int64_t R,
                     double *loss, float *grad)
{
    return guarded([&]() -> int {
        if (!ws || !feats || !targets || !loss) return fail(BIE_EINVAL, "NULL argument");
        if (R < 1 || R > 65535) return fail(BIE_EINVAL, "R out of range");
        *loss = bie::ws_loss_grad(ws, feats, pols, targets, R, grad, nullptr);
        return BIE_OK;
    });
}

int bie_ws_forward(bie_ws *ws, const double *feats, int64_t R, float *out)
{
    return guarded([&]() -> int {
        if (!ws || !feats || !out) return fail(BIE_EINVAL, "NULL argument");
        if (R < 1 || R > 65535) return fail(BIE_EINVAL, "R out of range");
        bie::ws_forward(ws, feats, R, out, nullptr);
        return BIE_OK;
    });
}

int bie_ws_create(const bie_op *op, int pod_rank, int hidden, uint64_t seed, int pol_model, bie_ws **out)
{
    return guarded([&]() -> int {
        if (!op || !out) return fail(BIE_EINVAL, "NULL argument");
        if (op->star) return fail(BIE_EINVAL, "the warm start takes an assembled operator");
        if (pod_rank < 1 || hidden < 1 || hidden > 4096) return fail(BIE_EINVAL, "bad sizes");
        if (pol_model != 0 && pol_model != 1) return fail(BIE_EINVAL, "pol_model must be 0 or 1");
        *out = bie::ws_create_untrained(op, pod_rank, hidden, seed, pol_model);
        return BIE_OK;
    });
}

int bie_ws_save(const bie_ws *ws, const char *path)
{
    return guarded([&]() -> int {
        if (!ws || !path) return fail(BIE_EINVAL, "NULL argument");
        bie::ws_save(ws, path);
        return BIE_OK;
    });
}

int bie_ws_load(const bie_op *op, const char *path, bie_ws **out)
{
    return guarded([&]() -> int {
        if (!op || !path || !out) return fail(BIE_EINVAL, "NULL argument");
        if (op->star) return fail(BIE_EINVAL, "the warm start takes an assembled operator");
        *out = bie::ws_load(op, path);
        return BIE_OK;
    });
}

void bie_ws_destroy(bie_ws *ws)
{
    if (ws) bie::ws_destroy(ws);
}

int bie_autotune(int on)
{
    bie::tune_set_enabled(on != 0);
    return BIE_OK;
}

int64_t bie_autotune_report(char *buf, int64_t cap)
{
    const std::string r = bie::tune_report();
    if (buf && cap > 0) {
        const size_t n = std::min<size_t>(r.size(), size_t(cap - 1));
        std::memcpy(buf, r.data(), n);
        buf[n] = 0;
    }
    return int64_t(r.size()) + 1;
}

int bie_prof_enable(int on)
{
    return guarded([&]() -> int {
        bie::prof_enable(on != 0);
        return BIE_OK;
    });
}

int bie_prof_read(int kernel, int64_t *launches, double *total_ms, int64_t *columns)
{
    return guarded([&]() -> int {
        if (!launches || !total_ms) return fail(BIE_EINVAL, "NULL argument");
        bie::prof_read(kernel, launches, total_ms, columns);
        return BIE_OK;
    });
}

int bie_rscc_rows(int64_t N, int64_t S, uint64_t seed, int64_t *out)
{
    return guarded([&]() -> int {
        if (!out || N < 1 || S < 1) return fail(BIE_EINVAL, "bad argument");
        auto v = bie::rscc_rows(N, S, seed);
        std::memcpy(out, v.data(), v.size() * sizeof(int64_t));
        return BIE_OK;
    });
}

}  // extern "C"
