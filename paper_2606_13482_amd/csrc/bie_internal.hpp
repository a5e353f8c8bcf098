// Internal declarations of libbie: operator state, error plumbing, launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
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

}  // namespace bie

struct bie_op {
    int device = 0;
    double k = 0.0;
    int storage = BIE_C128;
    bie::Mesh mesh;
    bie::TriDev tri;
    void *Z64 = nullptr;   // N x N complex128 row-major (storage C128 or keep_fp64)
    void *Z32 = nullptr;   // N x N complex64 row-major (storage C64)
    bie::Workspace *ws = nullptr;
};

namespace bie {

// fill.hip
void upload_triangles(bie_op *op, hipStream_t s);
void fill_matrix(bie_op *op, bool fp64_regular, bool want64, bool want32, hipStream_t s);
void rhs_planewave(const bie_op *op, const double *dirs, const double *pols, int64_t R, void *B,
                   hipStream_t s);
void farfield(const bie_op *op, const void *X, int64_t R, const double *obs, int64_t M, void *F,
              hipStream_t s);

// blas.hip: Y = Z X (R vectors), complex128 or complex64 vectors and matrix.
void gemv_c128(const void *Z, int64_t N, const void *X, void *Y, int64_t R, bool conj, hipStream_t s);
void gemv_c64(const void *Z, int64_t N, const void *X, void *Y, int64_t R, bool conj, hipStream_t s);
void convert_c128_to_c64(const void *src, void *dst, int64_t n, hipStream_t s);
void convert_c64_to_c128(const void *src, void *dst, int64_t n, hipStream_t s);
bool has_nonfinite(const void *x, int64_t n_doubles, hipStream_t s);
void prof_enable(bool enable);
void prof_read(int64_t *launches, double *total_ms);

// krylov.hip
int solve(const bie_op *op, const void *B, void *X, int64_t R, const bie_solve_opts &o,
          bie_solve_stat *stats, hipStream_t s);
void free_workspace(bie_op *op);

}  // namespace bie
