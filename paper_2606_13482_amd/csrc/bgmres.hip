// Restarted block GMRES over groups of right-hand sides: every group of at most
// `block` right-hand sides shares one block Krylov space, and each of its
// columns takes the element of that space that minimises its own residual
// (block GMRES: Vital 1990; Saad, Iterative Methods for Sparse Linear Systems,
// Sec. 6.12).  The paper's acronym list names GMRES only; block GMRES is the
// reading used for its many-right-hand-side runs.
//
// One restart cycle of a group of q columns:
//   R0 (scaled to unit columns) = V_0 S     rank-revealing: pivoted Cholesky of
//                                           the Gram matrix, directions below
//                                           delta are left out (width r <= q)
//   j = 0, 1, ...:
//     W = T V_j                             one block product over the active
//                                           columns of every group
//     C = V^H W; W -= V C; G = W^H W        block classical Gram-Schmidt; with
//                                           the FP64 basis a second pass when a
//                                           column kept less than half of its
//                                           norm squared
//     W^H W = R^H R (Cholesky), V_{j+1} = W R^{-1}
//     Hbar(:, j) = [C; R]; block Householder update of its QR factorisation and
//     of E_1 S; per-column residual estimate from the last r rows
//   the cycle ends when every column meets its target, on a partial breakdown
//   (a Cholesky pivot at or below delta times the largest column norm of T V_j)
//   or after m steps; then Y = argmin ||E_1 S - Hbar Y|| and X += V Y.
//
// Everything after the product runs on the device, with one host
// synchronisation per step (the estimates decide which groups go on).
// Precision 0: FP64 basis, FP64 block products on the matrix cores, target
// tol ||b||.  Precision 1 (iterative refinement): complex64 basis, split-BF16
// block products, one cycle per refinement step to inner_tol relative to the
// FP64 residual, FP64 residuals and criterion outside.
#include "bie_internal.hpp"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <type_traits>
#include <cstring>
#include <memory>
#include <vector>

namespace bie {
namespace {

constexpr int BMAX = 32;    // right-hand sides per group, at most
constexpr int DT = 128;     // basis vectors per tile of the dot kernel
constexpr int DS = 16;      // rows per LDS stage of the dot kernel
constexpr double DELTA = 1e-6;

__device__ inline double2 to_d2(double2 v) { return v; }
__device__ inline double2 to_d2(float2 v) { return make_double2(double(v.x), double(v.y)); }
template <typename T>
__device__ inline T from_d2(double2 v);
template <>
__device__ inline double2 from_d2<double2>(double2 v) { return v; }
template <>
__device__ inline float2 from_d2<float2>(double2 v) { return make_float2(float(v.x), float(v.y)); }
__device__ inline double2 to_d2(c32h v) { return make_double2(double(v.x), double(v.y)); }
template <>
__device__ inline c32h from_d2<c32h>(double2 v) { return c32h{ (_Float16)v.x, (_Float16)v.y }; }
// Basis entries as loaded (raw) and as two floats: complex64, or an FP16 pair
// read as one 4-byte vector.  The loads name the global address space: a
// generic (flat) load also counts against the LDS wait counter, so waiting for
// the LDS fragment reads would wait for the prefetch of the next stage too.
typedef _Float16 h2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef double d2v __attribute__((ext_vector_type(2)));
template <typename V>
__device__ inline V ld_vec(const void *p, int64_t i)
{
    return ((const __attribute__((address_space(1))) V *)p)[i];
}
__device__ inline float2 ld_global(const float2 *p, int64_t i)
{
    const f2v v = ld_vec<f2v>(p, i);
    return make_float2(v[0], v[1]);
}
__device__ inline double2 ld_global(const double2 *p, int64_t i)
{
    const d2v v = ld_vec<d2v>(p, i);
    return make_double2(v[0], v[1]);
}
__device__ inline h2v ld_global(const h2v *p, int64_t i) { return ld_vec<h2v>(p, i); }
typedef float f4v __attribute__((ext_vector_type(4)));
typedef _Float16 h8v __attribute__((ext_vector_type(8)));
// load16: the P16 entries i .. i + P16 - 1 (i a multiple of P16, 16-byte aligned) in one load
template <typename AT> struct BasisRaw;
template <> struct BasisRaw<float2> {
    typedef float2 type;
    static constexpr int P16 = 2;
    static constexpr int MINB = 1;   // workgroups per CU asked of the compiler for the update (more would spill)
    static __device__ inline type load(const void *A, int64_t i) { return ld_global((const float2 *)A, i); }
    static __device__ inline void load16(const void *A, int64_t i, type *o)
    {
        const f4v v = ld_vec<f4v>(A, i >> 1);
        o[0] = make_float2(v[0], v[1]);
        o[1] = make_float2(v[2], v[3]);
    }
    static __device__ inline type zero() { return make_float2(0.f, 0.f); }
    static __device__ inline float2 f2(type v) { return v; }
};
template <> struct BasisRaw<c32h> {
    typedef h2v type;
    static constexpr int MINB = 4;   // the update's 4 waves per SIMD fit in the registers without spills
    static constexpr int P16 = 4;
    static __device__ inline type load(const void *A, int64_t i) { return ld_global((const h2v *)A, i); }
    static __device__ inline void load16(const void *A, int64_t i, type *o)
    {
        const h8v v = ld_vec<h8v>(A, i >> 2);
#pragma unroll
        for (int j = 0; j < 4; ++j) o[j] = h2v{ v[2 * j], v[2 * j + 1] };
    }
    static __device__ inline type zero() { return h2v{ (_Float16)0.f, (_Float16)0.f }; }
    static __device__ inline float2 f2(type v) { return make_float2(float(v[0]), float(v[1])); }
};

__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 cmulc(double2 a, double2 b)   // conj(a) * b
{
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }

// Dot item: dst[(k0 + v) * ld + b] = sum_n conj(A_{k0+v}[n]) B_b[n] for v < kc, b < nb.
// Basis vector k is at A + ((k / ar) * astride + k % ar) * N (blocks of ar
// vectors, astride vectors apart); column b of B at Bm + b * N.
struct DItem {
    const void *A;
    int64_t astride;
    const double2 *Bm;
    double2 *dst;
    const int *flag;   // item runs only if *flag != 0 (null: always)
    int ar, k0, kc, nb, ld, pad;
};

// Combination item: out_b[n] = beta out_b[n] + alpha sum_k A_k[n] C[k * ldc + b]
// for k < K, b < nb; output column b at out + (ocol ? ocol[b] : b) * N.
struct CItem {
    const void *A;
    int64_t astride;
    const double2 *C;
    void *out;
    const int *ocol;
    const int *flag;
    double alpha, beta;
    int ar, K, ldc, nb;
};

// Partial dots over a chunk of L rows, tiles of 32 U basis vectors;
// part[((item * nchunks + chunk) * 32 U + v) * BMAX + b].  Thread (v = t % 32,
// h = t / 32): basis vectors v + 32 u (u < U) of the tile against columns
// h + 8 q (q < NC).
template <typename AT, int NQ, int U>
__global__ __launch_bounds__(256) void k_bdots(const DItem *__restrict__ items, int64_t N, int nchunks, int64_t L,
                                               double2 *__restrict__ part)
{
    constexpr int NC = (NQ + 1) / 2;   // columns per thread: 4 NQ columns over 8 thread groups
    constexpr int TU = 32 * U;         // basis vectors per tile
    const DItem it = items[blockIdx.y];
    if (it.flag && *it.flag == 0) return;
    const int t = threadIdx.x, v = t & 31, h = t >> 5;
    const int64_t n0 = int64_t(blockIdx.x) * L, n1 = min(N, n0 + L);
    __shared__ double2 As[DS][TU + 1];
    __shared__ double2 Bs[BMAX][DS + 1];
    __shared__ int64_t Aoff[TU];
    if (t < TU) {
        const int k = it.k0 + t;
        Aoff[t] = t < it.kc ? (int64_t(k / it.ar) * it.astride + k % it.ar) * N : 0;
    }
    double2 acc[U][NC];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int q = 0; q < NC; ++q) acc[u][q] = make_double2(0.0, 0.0);
    const AT *A = static_cast<const AT *>(it.A);
    for (int64_t ns = n0; ns < n1; ns += DS) {
        __syncthreads();
        for (int e = t; e < TU * DS; e += 256) {
            const int vv = e / DS, rr = e % DS;
            const int64_t n = ns + rr;
            As[rr][vv] = (vv < it.kc && n < n1) ? to_d2(A[Aoff[vv] + n]) : make_double2(0.0, 0.0);
        }
        for (int e = t; e < 8 * NC * DS; e += 256) {
            const int b = e / DS, rr = e % DS;
            const int64_t n = ns + rr;
            Bs[b][rr] = (b < it.nb && n < n1) ? it.Bm[int64_t(b) * N + n] : make_double2(0.0, 0.0);
        }
        __syncthreads();
#pragma unroll 2
        for (int rr = 0; rr < DS; ++rr) {
            double2 a[U];
#pragma unroll
            for (int u = 0; u < U; ++u) a[u] = As[rr][v + 32 * u];
#pragma unroll
            for (int q = 0; q < NC; ++q) {
                const double2 bv = Bs[h + 8 * q][rr];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    acc[u][q].x = fma(a[u].x, bv.x, fma(a[u].y, bv.y, acc[u][q].x));
                    acc[u][q].y = fma(a[u].x, bv.y, fma(-a[u].y, bv.x, acc[u][q].y));
                }
            }
        }
    }
    double2 *o = part + (int64_t(blockIdx.y) * nchunks + blockIdx.x) * TU * BMAX;
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        const int b = h + 8 * q;
        if (b < it.nb)
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (v + 32 * u < it.kc) o[(v + 32 * u) * BMAX + b] = acc[u][q];
    }
}

// Sums the chunk partials in a fixed order: 4 lanes per output, chunks c = lane
// mod 4, then a 4-lane reduction.
__global__ __launch_bounds__(256) void k_bdots_fin(const DItem *__restrict__ items, int nchunks, int tu,
                                                   const double2 *__restrict__ part)
{
    const DItem it = items[blockIdx.x];
    if (it.flag && *it.flag == 0) return;
    const int e = blockIdx.y * 64 + (threadIdx.x >> 2), l = threadIdx.x & 3;
    const bool live = e < it.kc * it.nb;
    const int v = live ? e / it.nb : 0, b = live ? e % it.nb : 0;
    double2 sv = make_double2(0.0, 0.0);
    if (live)
        for (int c = l; c < nchunks; c += 4) sv = cadd(sv, part[((int64_t(blockIdx.x) * nchunks + c) * tu + v) * BMAX + b]);
    for (int o = 1; o < 4; o <<= 1) {
        sv.x += __shfl_xor(sv.x, o, 4);
        sv.y += __shfl_xor(sv.y, o, 4);
    }
    if (live && l == 0) it.dst[int64_t(it.k0 + v) * it.ld + b] = sv;
}

// 128 rows per block; thread (rows v + 32 u, u < 4, with v = t % 32, h = t / 32)
// accumulates columns h, h + 8, ...; 16 basis vectors and their coefficient
// rows staged in LDS per round.
template <typename AT, typename OT, int NB>
__global__ __launch_bounds__(256) void k_bcomb(const CItem *__restrict__ items, int64_t N)
{
    constexpr int NC = (NB + 7) / 8, KS = 16, RT = 128;
    const CItem it = items[blockIdx.y];
    if (it.flag && *it.flag == 0) return;
    const int t = threadIdx.x, v = t & 31, h = t >> 5;
    const int64_t n0 = int64_t(blockIdx.x) * RT;
    __shared__ double2 As[KS][RT + 1];
    __shared__ double2 Cs[KS][8 * NC];
    __shared__ int64_t Aoff[KS];
    double2 acc[4][NC];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < NC; ++q) acc[u][q] = make_double2(0.0, 0.0);
    const AT *A = static_cast<const AT *>(it.A);
    for (int k0 = 0; k0 < it.K; k0 += KS) {
        const int kc = min(KS, it.K - k0);
        __syncthreads();
        if (t < KS) {
            const int k = k0 + t;
            Aoff[t] = t < kc ? (int64_t(k / it.ar) * it.astride + k % it.ar) * N : 0;
        }
        for (int e = t; e < KS * 8 * NC; e += 256) {
            const int kk = e / (8 * NC), b = e % (8 * NC);
            Cs[kk][b] = (kk < kc && b < it.nb) ? it.C[int64_t(k0 + kk) * it.ldc + b] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        for (int e = t; e < KS * RT; e += 256) {
            const int kk = e / RT, rr = e % RT;
            const int64_t nn = n0 + rr;
            As[kk][rr] = (kk < kc && nn < N) ? to_d2(A[Aoff[kk] + nn]) : make_double2(0.0, 0.0);
        }
        __syncthreads();
#pragma unroll 2
        for (int kk = 0; kk < kc; ++kk) {
            double2 a[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) a[u] = As[kk][v + 32 * u];
#pragma unroll
            for (int q = 0; q < NC; ++q) {
                const double2 c = Cs[kk][h + 8 * q];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    acc[u][q].x = fma(a[u].x, c.x, fma(-a[u].y, c.y, acc[u][q].x));
                    acc[u][q].y = fma(a[u].x, c.y, fma(a[u].y, c.x, acc[u][q].y));
                }
            }
        }
    }
    OT *out = static_cast<OT *>(it.out);
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        const int b = h + 8 * q;
        if (b < it.nb) {
            const int64_t col = int64_t(it.ocol ? it.ocol[b] : b) * N;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t n = n0 + v + 32 * u;
                if (n < N) {
                    double2 y = cscale(it.alpha, acc[u][q]);
                    if (it.beta != 0.0) y = cadd(y, cscale(it.beta, to_d2(out[col + n])));
                    out[col + n] = from_d2<OT>(y);
                }
            }
        }
    }
}

// FP32 matrix-core forms of the dots and the update for the complex64 basis of
// the refinement's inner solves (FP32 products, FP32 accumulation; the inner
// tolerance is 1e-3 .. 1e-1).  v_mfma_f32_32x32x2f32: A[i][k] in lane i + 32 k,
// B[k][j] in lane j + 32 k, D value q of lane l at row 8 (q / 4) + 4 (l / 32) +
// q % 4, column l % 32.  Complex products as four real ones.
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ inline f32x16 mfma32(float a, float b, f32x16 c) { return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0); }

// Dots C = V^H W over a chunk of L rows, tiles of 128 basis vectors (one 32 x 32
// output tile per wave) against up to 32 columns; partials as k_bdots with U = 4.
__global__ __launch_bounds__(256) void k_bdots_mf(const DItem *__restrict__ items, int64_t N, int nchunks, int64_t L,
                                                  double2 *__restrict__ part)
{
    constexpr int MS = 32;   // rows per LDS stage
    const DItem it = items[blockIdx.y];
    if (it.flag && *it.flag == 0) return;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t n0 = int64_t(blockIdx.x) * L, n1 = min(N, n0 + L);
    __shared__ float2 As[MS][128 + 1];
    __shared__ float2 Bs[MS][32 + 1];
    __shared__ int64_t Aoff[128];
    if (t < 128) {
        const int k = it.k0 + t;
        Aoff[t] = t < it.kc ? (int64_t(k / it.ar) * it.astride + k % it.ar) * N : 0;
    }
    f32x16 cr, ci;
#pragma unroll
    for (int q = 0; q < 16; ++q) cr[q] = ci[q] = 0.f;
    const float2 *A = static_cast<const float2 *>(it.A);
    // each thread stages 16 basis entries and 4 column entries per stage; the
    // next stage is loaded into registers while the current one is multiplied
    float2 ra[16];
    double2 rb[4];
    auto gload = [&](int64_t ns) {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = t + 256 * u, vv = e / MS, rr = e % MS;
            const int64_t n = ns + rr;
            ra[u] = (vv < it.kc && n < n1) ? A[Aoff[vv] + n] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = t + 256 * u, b = e / MS, rr = e % MS;
            const int64_t n = ns + rr;
            rb[u] = (b < it.nb && n < n1) ? it.Bm[int64_t(b) * N + n] : make_double2(0.0, 0.0);
        }
    };
    __syncthreads();   // Aoff
    if (n0 < n1) gload(n0);
    for (int64_t ns = n0; ns < n1; ns += MS) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = t + 256 * u;
            As[e % MS][e / MS] = ra[u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = t + 256 * u;
            Bs[e % MS][e / MS] = make_float2(float(rb[u].x), float(rb[u].y));
        }
        __syncthreads();
        if (ns + MS < n1) gload(ns + MS);
#pragma unroll 4
        for (int rr = 0; rr < MS; rr += 2) {
            const float2 a = As[rr + (lane >> 5)][32 * w + (lane & 31)];
            const float2 b = Bs[rr + (lane >> 5)][lane & 31];
            cr = mfma32(a.x, b.x, cr);
            cr = mfma32(a.y, b.y, cr);
            ci = mfma32(a.x, b.y, ci);
            ci = mfma32(-a.y, b.x, ci);
        }
    }
    double2 *o = part + (int64_t(blockIdx.y) * nchunks + blockIdx.x) * 128 * BMAX;
    const int col = lane & 31;
    if (col < it.nb) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int v = 32 * w + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
            if (v < it.kc) o[v * BMAX + col] = make_double2(double(cr[q]), double(ci[q]));
        }
    }
}

// Update out_b = beta out_b + alpha (V C)_b on 128 rows per block (one 32 x 32
// output tile per wave), 32 basis vectors per LDS stage.
__global__ __launch_bounds__(256) void k_bcomb_mf(const CItem *__restrict__ items, int64_t N)
{
    constexpr int KS = 32;
    const CItem it = items[blockIdx.y];
    if (it.flag && *it.flag == 0) return;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t n0 = int64_t(blockIdx.x) * 128;
    __shared__ float2 As[KS][128 + 1];
    __shared__ float2 Cs[KS][32 + 1];
    __shared__ int64_t Aoff[KS];
    f32x16 orr, oi;
#pragma unroll
    for (int q = 0; q < 16; ++q) orr[q] = oi[q] = 0.f;
    const float2 *A = static_cast<const float2 *>(it.A);
    // 16 basis entries and 4 coefficients per thread and stage; the next stage
    // is loaded into registers while the current one is multiplied
    float2 ra[16];
    double2 rc[4];
    auto offs = [&](int k0) {
        if (t < KS) {
            const int k = k0 + t;
            Aoff[t] = k < it.K ? (int64_t(k / it.ar) * it.astride + k % it.ar) * N : 0;
        }
    };
    auto gload = [&](int k0) {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = t + 256 * u, kk = e / 128, rr = e % 128;
            const int64_t nn = n0 + rr;
            ra[u] = (k0 + kk < it.K && nn < N) ? A[Aoff[kk] + nn] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = t + 256 * u, kk = e / 32, b = e % 32;
            rc[u] = (k0 + kk < it.K && b < it.nb) ? it.C[int64_t(k0 + kk) * it.ldc + b] : make_double2(0.0, 0.0);
        }
    };
    offs(0);
    __syncthreads();
    gload(0);
    for (int k0 = 0; k0 < it.K; k0 += KS) {
        __syncthreads();   // previous stage's LDS reads and Aoff reads done
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = t + 256 * u;
            As[e / 128][e % 128] = ra[u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = t + 256 * u;
            Cs[e / 32][e % 32] = make_float2(float(rc[u].x), float(rc[u].y));
        }
        offs(k0 + KS);
        __syncthreads();
        if (k0 + KS < it.K) gload(k0 + KS);
#pragma unroll 4
        for (int kk = 0; kk < KS; kk += 2) {
            const float2 a = As[kk + (lane >> 5)][32 * w + (lane & 31)];
            const float2 c = Cs[kk + (lane >> 5)][lane & 31];
            orr = mfma32(a.x, c.x, orr);
            orr = mfma32(-a.y, c.y, orr);
            oi = mfma32(a.x, c.y, oi);
            oi = mfma32(a.y, c.x, oi);
        }
    }
    const int col = lane & 31;
    if (col >= it.nb) return;
    double2 *out = static_cast<double2 *>(it.out);
    const int64_t ob = int64_t(it.ocol ? it.ocol[col] : col) * N;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int64_t n = n0 + 32 * w + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
        if (n < N) {
            double2 y = make_double2(it.alpha * double(orr[q]), it.alpha * double(oi[q]));
            if (it.beta != 0.0) y = cadd(y, cscale(it.beta, out[ob + n]));
            out[ob + n] = y;
        }
    }
}

// BF16 matrix-core forms of the same dots and update: every FP32 operand value
// v is split into hi = rne_bf16(v) and lo = rne_bf16(v - hi), and each real
// product is taken as hi*hi + hi*lo + lo*hi (about 16 significant bits, FP32
// accumulation) with v_mfma_f32_32x32x16_bf16, whose rate is 16 times that of
// the FP32 matrix-core instruction: the complex64 basis is then read at the
// memory rate instead of the FP32 matrix cores' rate.  The complex products
// are real GEMMs with re/im interleaved along K (K' = 2 k + part).
// Fragment layout of the instruction: A[i][k] is element k % 8 of lane
// i + 32 (k / 8), B[k][j] element k % 8 of lane j + 32 (k / 8); the output as
// for the FP32 instruction.  LDS planes hold rows of 64 K' values (one stage,
// 4 instruction K steps) with a stride of 72 (16-byte fragment reads of 16
// consecutive rows start in 16 distinct 4-bank groups).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
constexpr int SPL = 72;

__device__ inline f32x16 mfma_bf(bf16x8 a, bf16x8 b, f32x16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ inline void split_bf(float v, __bf16 &hi, __bf16 &lo)
{
    hi = (__bf16)v;
    lo = (__bf16)(v - (float)hi);
}

// Dots C = V^H W over a chunk of L rows as k_bdots_mf (128 basis vectors per
// block, one 32 x 32 output tile per wave, up to 32 columns, the same partials):
// A[v][2 n + p] = (Re, Im) V_v[n], B_re[2 n + p][b] = (Re, Im) W_b[n] (C_re),
// B_im[2 n + p][b] = (Im, -Re) W_b[n] (C_im); 32 complex rows per stage.
template <typename AT>
__global__ __launch_bounds__(256) void k_bdots_bf(const DItem *__restrict__ items, int64_t N, int nchunks, int64_t L,
                                                  double2 *__restrict__ part)
{
    constexpr int MS = 32;
    const DItem it = items[blockIdx.y];
    if (it.flag && *it.flag == 0) return;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t n0 = int64_t(blockIdx.x) * L, n1 = min(N, n0 + L);
    __shared__ __attribute__((aligned(16))) __bf16 Ah[128 * SPL], Al[128 * SPL];
    __shared__ __attribute__((aligned(16))) __bf16 Bh[2][32 * SPL], Bl[2][32 * SPL];
    __shared__ int64_t Aoff[128];
    if (t < 128) {
        const int k = it.k0 + t;
        Aoff[t] = t < it.kc ? (int64_t(k / it.ar) * it.astride + k % it.ar) * N : 0;
    }
    f32x16 cr, ci;
#pragma unroll
    for (int q = 0; q < 16; ++q) cr[q] = ci[q] = 0.f;
    typedef BasisRaw<AT> BR;
    // staging: thread t takes rows 2 (t % 16) and 2 (t % 16) + 1 of basis
    // vectors t / 16 + 16 u (u < 8), and rows 4 (t % 8) .. + 3 of column t / 8
    const int ar = 2 * (t & 15), av = t >> 4, bc = t >> 3, br = 4 * (t & 7);
    typename BR::type ra[16];   // raw: converted when written to LDS, so the prefetch stays in flight
    double2 rb[4];
    int64_t ao[8];              // offsets of the thread's 8 basis vectors
    auto gload = [&](int64_t ns) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int v = av + 16 * u;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int64_t n = ns + ar + e;
                ra[2 * u + e] = (v < it.kc && n < n1) ? BR::load(it.A, ao[u] + n) : BR::zero();
            }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t n = ns + br + e;
            rb[e] = (bc < it.nb && n < n1) ? ld_global(it.Bm, int64_t(bc) * N + n) : make_double2(0.0, 0.0);
        }
    };
    __syncthreads();   // Aoff
#pragma unroll
    for (int u = 0; u < 8; ++u) ao[u] = Aoff[av + 16 * u];
    if (n0 < n1) gload(n0);
    for (int64_t ns = n0; ns < n1; ns += MS) {
        __syncthreads();   // the previous stage's fragment reads are done
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            bf16x4 h, l;
            const float2 f0 = BR::f2(ra[2 * u]), f1 = BR::f2(ra[2 * u + 1]);
            const float f[4] = { f0.x, f0.y, f1.x, f1.y };
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                __bf16 hh, ll;
                split_bf(f[e], hh, ll);
                h[e] = hh;
                l[e] = ll;
            }
            const int o = (av + 16 * u) * SPL + 2 * ar;
            *reinterpret_cast<bf16x4 *>(&Ah[o]) = h;
            *reinterpret_cast<bf16x4 *>(&Al[o]) = l;
        }
        {
            bf16x8 rh, rl, ih, il;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                __bf16 hr, lr, hi, li;
                split_bf(float(rb[e].x), hr, lr);
                split_bf(float(rb[e].y), hi, li);
                rh[2 * e] = hr;
                rh[2 * e + 1] = hi;
                rl[2 * e] = lr;
                rl[2 * e + 1] = li;
                ih[2 * e] = hi;
                ih[2 * e + 1] = -hr;
                il[2 * e] = li;
                il[2 * e + 1] = -lr;
            }
            const int o = bc * SPL + 2 * br;
            *reinterpret_cast<bf16x8 *>(&Bh[0][o]) = rh;
            *reinterpret_cast<bf16x8 *>(&Bl[0][o]) = rl;
            *reinterpret_cast<bf16x8 *>(&Bh[1][o]) = ih;
            *reinterpret_cast<bf16x8 *>(&Bl[1][o]) = il;
        }
        __syncthreads();
        if (ns + MS < n1) gload(ns + MS);
        const int fa = (32 * w + (lane & 31)) * SPL + 8 * (lane >> 5), fb = (lane & 31) * SPL + 8 * (lane >> 5);
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const bf16x8 ah = *reinterpret_cast<const bf16x8 *>(&Ah[fa + 16 * ks]);
            const bf16x8 al = *reinterpret_cast<const bf16x8 *>(&Al[fa + 16 * ks]);
            const bf16x8 brh = *reinterpret_cast<const bf16x8 *>(&Bh[0][fb + 16 * ks]);
            const bf16x8 brl = *reinterpret_cast<const bf16x8 *>(&Bl[0][fb + 16 * ks]);
            const bf16x8 bih = *reinterpret_cast<const bf16x8 *>(&Bh[1][fb + 16 * ks]);
            const bf16x8 bil = *reinterpret_cast<const bf16x8 *>(&Bl[1][fb + 16 * ks]);
            cr = mfma_bf(ah, brh, cr);
            ci = mfma_bf(ah, bih, ci);
            cr = mfma_bf(ah, brl, cr);
            ci = mfma_bf(ah, bil, ci);
            cr = mfma_bf(al, brh, cr);
            ci = mfma_bf(al, bih, ci);
        }
    }
    double2 *o = part + (int64_t(blockIdx.y) * nchunks + blockIdx.x) * 128 * BMAX;
    const int col = lane & 31;
    if (col < it.nb) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int v = 32 * w + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
            if (v < it.kc) o[v * BMAX + col] = make_double2(double(cr[q]), double(ci[q]));
        }
    }
}

// Update out_b = beta out_b + alpha (V C)_b as k_bcomb_mf (128 rows per block,
// one 32 x 32 output tile per wave, 32 basis vectors per stage):
// A[n][2 k + p] = (Re, Im) V_k[n], B_re[2 k + p][b] = (Re, -Im) C[k][b],
// B_im[2 k + p][b] = (Im, Re) C[k][b].
template <typename AT>
__global__ __launch_bounds__(256) void k_bcomb_bf(const CItem *__restrict__ items, int64_t N)
{
    constexpr int KS = 32;
    const CItem it = items[blockIdx.y];
    if (it.flag && *it.flag == 0) return;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t n0 = int64_t(blockIdx.x) * 128;
    __shared__ __attribute__((aligned(16))) __bf16 Ah[128 * SPL], Al[128 * SPL];
    __shared__ __attribute__((aligned(16))) __bf16 Bh[2][32 * SPL], Bl[2][32 * SPL];
    __shared__ int64_t Aoff[KS];
    f32x16 orr, oi;
#pragma unroll
    for (int q = 0; q < 16; ++q) orr[q] = oi[q] = 0.f;
    typedef BasisRaw<AT> BR;
    // staging: thread t takes row t % 128 of basis vectors 16 (t / 128) .. + 15,
    // and coefficients k = 4 (t / 32) .. + 3 of column t % 32
    const int an = t & 127, ak = 16 * (t >> 7), cb = t & 31, ck = 4 * (t >> 5);
    typename BR::type ra[16];   // raw: converted when written to LDS
    double2 rc[4];
    auto offs = [&](int k0) {
        if (t < KS) {
            const int k = k0 + t;
            Aoff[t] = k < it.K ? (int64_t(k / it.ar) * it.astride + k % it.ar) * N : 0;
        }
    };
    auto gload = [&](int k0) {
        const int64_t nn = n0 + an;
        int64_t ao[16];   // the stage's offsets read from LDS first, then all loads issued
#pragma unroll
        for (int u = 0; u < 16; ++u) ao[u] = Aoff[ak + u];
#pragma unroll
        for (int u = 0; u < 16; ++u)
            ra[u] = (k0 + ak + u < it.K && nn < N) ? BR::load(it.A, ao[u] + nn) : BR::zero();
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + ck + u;
            rc[u] = (k < it.K && cb < it.nb) ? ld_global(it.C, int64_t(k) * it.ldc + cb) : make_double2(0.0, 0.0);
        }
    };
    offs(0);
    __syncthreads();
    gload(0);
    for (int k0 = 0; k0 < it.K; k0 += KS) {
        __syncthreads();   // previous stage's fragment reads and Aoff reads done
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            bf16x8 h, l;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                __bf16 hr, lr, hi, li;
                const float2 f = BR::f2(ra[4 * g + e]);
                split_bf(f.x, hr, lr);
                split_bf(f.y, hi, li);
                h[2 * e] = hr;
                h[2 * e + 1] = hi;
                l[2 * e] = lr;
                l[2 * e + 1] = li;
            }
            const int o = an * SPL + 2 * (ak + 4 * g);
            *reinterpret_cast<bf16x8 *>(&Ah[o]) = h;
            *reinterpret_cast<bf16x8 *>(&Al[o]) = l;
        }
        {
            bf16x8 rh, rl, ih, il;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                __bf16 hr, lr, hi, li;
                split_bf(float(rc[e].x), hr, lr);
                split_bf(float(rc[e].y), hi, li);
                rh[2 * e] = hr;
                rh[2 * e + 1] = -hi;
                rl[2 * e] = lr;
                rl[2 * e + 1] = -li;
                ih[2 * e] = hi;
                ih[2 * e + 1] = hr;
                il[2 * e] = li;
                il[2 * e + 1] = lr;
            }
            const int o = cb * SPL + 2 * ck;
            *reinterpret_cast<bf16x8 *>(&Bh[0][o]) = rh;
            *reinterpret_cast<bf16x8 *>(&Bl[0][o]) = rl;
            *reinterpret_cast<bf16x8 *>(&Bh[1][o]) = ih;
            *reinterpret_cast<bf16x8 *>(&Bl[1][o]) = il;
        }
        offs(k0 + KS);
        __syncthreads();
        if (k0 + KS < it.K) gload(k0 + KS);
        const int fa = (32 * w + (lane & 31)) * SPL + 8 * (lane >> 5), fb = (lane & 31) * SPL + 8 * (lane >> 5);
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const bf16x8 ah = *reinterpret_cast<const bf16x8 *>(&Ah[fa + 16 * ks]);
            const bf16x8 al = *reinterpret_cast<const bf16x8 *>(&Al[fa + 16 * ks]);
            const bf16x8 brh = *reinterpret_cast<const bf16x8 *>(&Bh[0][fb + 16 * ks]);
            const bf16x8 brl = *reinterpret_cast<const bf16x8 *>(&Bl[0][fb + 16 * ks]);
            const bf16x8 bih = *reinterpret_cast<const bf16x8 *>(&Bh[1][fb + 16 * ks]);
            const bf16x8 bil = *reinterpret_cast<const bf16x8 *>(&Bl[1][fb + 16 * ks]);
            orr = mfma_bf(ah, brh, orr);
            oi = mfma_bf(ah, bih, oi);
            orr = mfma_bf(ah, brl, orr);
            oi = mfma_bf(ah, bil, oi);
            orr = mfma_bf(al, brh, orr);
            oi = mfma_bf(al, bih, oi);
        }
    }
    const int col = lane & 31;
    if (col >= it.nb) return;
    double2 *out = static_cast<double2 *>(it.out);
    const int64_t ob = int64_t(it.ocol ? it.ocol[col] : col) * N;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int64_t n = n0 + 32 * w + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
        if (n < N) {
            double2 y = make_double2(it.alpha * double(orr[q]), it.alpha * double(oi[q]));
            if (it.beta != 0.0) y = cadd(y, cscale(it.beta, out[ob + n]));
            out[ob + n] = y;
        }
    }
}

// The same dots with the basis read straight into the matrix-core operands
// (no LDS for it): the order of the real K values is permuted (any order
// serves, as long as both operands take the same one) so that in a stage of 32
// rows lane l of a wave holds rows 16 (l / 32) .. + 15 of its basis vector, read
// as 16-byte loads, and instruction K step ks takes its rows 4 ks .. 4 ks + 3.
// The columns W stay in LDS in natural order (K' = 2 row + part), where the
// fragment of (ks, l / 32) is the 8 values at 32 (l / 32) + 8 ks.  Needs
// N % 4 == 0 (16-byte alignment of every lane's rows).
template <typename AT>
__global__ __launch_bounds__(256) void k_bdots_bd(const DItem *__restrict__ items, int64_t N, int nchunks, int64_t L,
                                                  double2 *__restrict__ part, int xcd)
{
    constexpr int MS = 32;
    typedef BasisRaw<AT> BR;
    int chunk = blockIdx.x, item = blockIdx.y;
    if (xcd) {
        // workgroups go to the 8 XCDs in turn: give each XCD a contiguous run of
        // (chunk, item) pairs, items fastest, so that the tiles of one group on
        // one chunk of rows follow each other on one XCD and its L2 keeps the
        // chunk of the columns W they all read
        const int total = gridDim.x * gridDim.y, lin = blockIdx.x + gridDim.x * blockIdx.y;
        const int x = lin & 7, per = total >> 3, extra = total & 7;
        const int wi = x * per + min(x, extra) + (lin >> 3);
        chunk = wi / gridDim.y;
        item = wi % gridDim.y;
    }
    const DItem it = items[item];
    if (it.flag && *it.flag == 0) return;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, h = lane >> 5;
    const int64_t n0 = int64_t(chunk) * L, n1 = min(N, n0 + L);
    __shared__ __attribute__((aligned(16))) __bf16 Bh[2][32 * SPL], Bl[2][32 * SPL];
    const int v = 32 * w + (lane & 31);
    const bool vlive = v < it.kc;
    const int64_t aoff = vlive ? (int64_t((it.k0 + v) / it.ar) * it.astride + (it.k0 + v) % it.ar) * N : 0;
    f32x16 cr, ci;
#pragma unroll
    for (int q = 0; q < 16; ++q) cr[q] = ci[q] = 0.f;
    // column staging: rows 4 (t % 8) .. + 3 of column t / 8
    const int bc = t >> 3, br = 4 * (t & 7);
    typename BR::type ra[16];   // the lane's 16 rows, raw
    double2 rb[4];
    auto gload = [&](int64_t ns) {
        const int64_t r0 = ns + 16 * h;
        if (ns + MS <= n1) {
#pragma unroll
            for (int c = 0; c < 16 / BR::P16; ++c) {
                if (vlive) BR::load16(it.A, aoff + r0 + BR::P16 * c, &ra[BR::P16 * c]);
                else
#pragma unroll
                    for (int j = 0; j < BR::P16; ++j) ra[BR::P16 * c + j] = BR::zero();
            }
        } else {
#pragma unroll
            for (int e = 0; e < 16; ++e) ra[e] = (vlive && r0 + e < n1) ? BR::load(it.A, aoff + r0 + e) : BR::zero();
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t n = ns + br + e;
            rb[e] = (bc < it.nb && n < n1) ? ld_global(it.Bm, int64_t(bc) * N + n) : make_double2(0.0, 0.0);
        }
    };
    if (n0 < n1) gload(n0);
    for (int64_t ns = n0; ns < n1; ns += MS) {
        __syncthreads();   // the previous stage's fragment reads are done
        {
            bf16x8 rh, rl, ih, il;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                __bf16 hr, lr, hi, li;
                split_bf(float(rb[e].x), hr, lr);
                split_bf(float(rb[e].y), hi, li);
                rh[2 * e] = hr;
                rh[2 * e + 1] = hi;
                rl[2 * e] = lr;
                rl[2 * e + 1] = li;
                ih[2 * e] = hi;
                ih[2 * e + 1] = -hr;
                il[2 * e] = li;
                il[2 * e + 1] = -lr;
            }
            const int o = bc * SPL + 2 * br;
            *reinterpret_cast<bf16x8 *>(&Bh[0][o]) = rh;
            *reinterpret_cast<bf16x8 *>(&Bl[0][o]) = rl;
            *reinterpret_cast<bf16x8 *>(&Bh[1][o]) = ih;
            *reinterpret_cast<bf16x8 *>(&Bl[1][o]) = il;
        }
        // the lane's basis fragments of the 4 K steps, split into BF16 hi / lo
        bf16x8 fh[4], fl[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float2 f = BR::f2(ra[4 * ks + e]);
                __bf16 a, b, c, d;
                split_bf(f.x, a, b);
                split_bf(f.y, c, d);
                fh[ks][2 * e] = a;
                fl[ks][2 * e] = b;
                fh[ks][2 * e + 1] = c;
                fl[ks][2 * e + 1] = d;
            }
        __syncthreads();
        if (ns + MS < n1) gload(ns + MS);
        const int fb = (lane & 31) * SPL + 32 * h;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const bf16x8 brh = *reinterpret_cast<const bf16x8 *>(&Bh[0][fb + 8 * ks]);
            const bf16x8 brl = *reinterpret_cast<const bf16x8 *>(&Bl[0][fb + 8 * ks]);
            const bf16x8 bih = *reinterpret_cast<const bf16x8 *>(&Bh[1][fb + 8 * ks]);
            const bf16x8 bil = *reinterpret_cast<const bf16x8 *>(&Bl[1][fb + 8 * ks]);
            cr = mfma_bf(fh[ks], brh, cr);
            ci = mfma_bf(fh[ks], bih, ci);
            cr = mfma_bf(fh[ks], brl, cr);
            ci = mfma_bf(fh[ks], bil, ci);
            cr = mfma_bf(fl[ks], brh, cr);
            ci = mfma_bf(fl[ks], bih, ci);
        }
    }
    double2 *o = part + (int64_t(item) * nchunks + chunk) * 128 * BMAX;
    const int col = lane & 31;
    if (col < it.nb) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int vv = 32 * w + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
            if (vv < it.kc) o[vv * BMAX + col] = make_double2(double(cr[q]), double(ci[q]));
        }
    }
}

// The update with the basis read straight into the matrix-core operands: the
// transposed product out^T = C^T V^T, whose right operand is V (column n of a
// wave's 32 rows, K' = 2 k + part along the basis index k), so that lane l reads
// entry n of 4 basis vectors per instruction K step (the lanes of a half-wave:
// 32 consecutive entries of one vector), and whose left operand C^T (the
// coefficients, as the planes of k_bcomb_bf) comes from LDS.  Output value q of
// lane l: column b = 8 (q / 4) + 4 (l / 32) + q % 4, row n = l % 32 of the wave.
template <typename AT>
__global__ __launch_bounds__(256, BasisRaw<AT>::MINB) void k_bcomb_bd(const CItem *__restrict__ items, int64_t N)
{
    constexpr int KS = 32;
    typedef BasisRaw<AT> BR;
    const CItem it = items[blockIdx.y];
    if (it.flag && *it.flag == 0) return;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, h = lane >> 5;
    const int64_t nn = int64_t(blockIdx.x) * 128 + 32 * w + (lane & 31);
    const bool nlive = nn < N;
    __shared__ __attribute__((aligned(16))) __bf16 Ch[2][32 * SPL], Cl[2][32 * SPL];
    __shared__ int64_t Aoff[KS];
    f32x16 orr, oi;
#pragma unroll
    for (int q = 0; q < 16; ++q) orr[q] = oi[q] = 0.f;
    // coefficient staging: k = 4 (t / 32) .. + 3 of column t % 32
    const int cb = t & 31, ck = 4 * (t >> 5);
    typename BR::type ra[16];   // entry nn of basis vectors 8 ks + 4 h + j (ks, j < 4), raw
    double2 rc[4];
    auto offs = [&](int k0) {
        if (t < KS) {
            const int k = k0 + t;
            Aoff[t] = k < it.K ? (int64_t(k / it.ar) * it.astride + k % it.ar) * N : 0;
        }
    };
    auto gload = [&](int k0) {
        int64_t ao[16];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
#pragma unroll
            for (int j = 0; j < 4; ++j) ao[4 * ks + j] = Aoff[8 * ks + 4 * h + j];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = k0 + 8 * ks + 4 * h + j;
                ra[4 * ks + j] = (k < it.K && nlive) ? BR::load(it.A, ao[4 * ks + j] + nn) : BR::zero();
            }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + ck + u;
            rc[u] = (k < it.K && cb < it.nb) ? ld_global(it.C, int64_t(k) * it.ldc + cb) : make_double2(0.0, 0.0);
        }
    };
    offs(0);
    __syncthreads();
    gload(0);
    for (int k0 = 0; k0 < it.K; k0 += KS) {
        __syncthreads();   // previous stage's fragment reads and Aoff reads done
        {
            bf16x8 rh, rl, ih, il;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                __bf16 hr, lr, hi, li;
                split_bf(float(rc[e].x), hr, lr);
                split_bf(float(rc[e].y), hi, li);
                rh[2 * e] = hr;
                rh[2 * e + 1] = -hi;
                rl[2 * e] = lr;
                rl[2 * e + 1] = -li;
                ih[2 * e] = hi;
                ih[2 * e + 1] = hr;
                il[2 * e] = li;
                il[2 * e + 1] = lr;
            }
            const int o = cb * SPL + 2 * ck;
            *reinterpret_cast<bf16x8 *>(&Ch[0][o]) = rh;
            *reinterpret_cast<bf16x8 *>(&Cl[0][o]) = rl;
            *reinterpret_cast<bf16x8 *>(&Ch[1][o]) = ih;
            *reinterpret_cast<bf16x8 *>(&Cl[1][o]) = il;
        }
        bf16x8 fh[4], fl[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float2 f = BR::f2(ra[4 * ks + j]);
                __bf16 a, b, c, d;
                split_bf(f.x, a, b);
                split_bf(f.y, c, d);
                fh[ks][2 * j] = a;
                fl[ks][2 * j] = b;
                fh[ks][2 * j + 1] = c;
                fl[ks][2 * j + 1] = d;
            }
        offs(k0 + KS);
        __syncthreads();
        if (k0 + KS < it.K) gload(k0 + KS);
        const int fa = (lane & 31) * SPL + 8 * h;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const bf16x8 arh = *reinterpret_cast<const bf16x8 *>(&Ch[0][fa + 16 * ks]);
            const bf16x8 arl = *reinterpret_cast<const bf16x8 *>(&Cl[0][fa + 16 * ks]);
            const bf16x8 aih = *reinterpret_cast<const bf16x8 *>(&Ch[1][fa + 16 * ks]);
            const bf16x8 ail = *reinterpret_cast<const bf16x8 *>(&Cl[1][fa + 16 * ks]);
            orr = mfma_bf(arh, fh[ks], orr);
            oi = mfma_bf(aih, fh[ks], oi);
            orr = mfma_bf(arh, fl[ks], orr);
            oi = mfma_bf(aih, fl[ks], oi);
            orr = mfma_bf(arl, fh[ks], orr);
            oi = mfma_bf(ail, fh[ks], oi);
        }
    }
    if (!nlive) return;
    double2 *out = static_cast<double2 *>(it.out);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int b = 8 * (q >> 2) + 4 * h + (q & 3);
        if (b < it.nb) {
            const int64_t ob = int64_t(it.ocol ? it.ocol[b] : b) * N;
            double2 y = make_double2(it.alpha * double(orr[q]), it.alpha * double(oi[q]));
            if (it.beta != 0.0) y = cadd(y, cscale(it.beta, out[ob + nn]));
            out[ob + nn] = y;
        }
    }
}

// The update of an item whose K <= 32 vectors are FP64 (the scaling of a new
// block, V_{j+1} = W T^{-1}, and the first block of a cycle) on the FP64 matrix
// cores: v_mfma_f64_16x16x4f64 (A[i][k] in lane i + 16 k, B[k][j] in lane j + 16
// k, output value q of lane l at row l / 16 + 4 q, column l % 16), complex
// products as four real ones, exact FP64 products with FP64 accumulation.  Wave
// w of a workgroup takes rows 16 w .. + 15 of its 64 and all 32 columns (two
// tiles of 16); lane l reads entry n of vector k = 4 ks + l / 16 straight into
// the operand, and the coefficients from global memory (one small matrix per
// item, cached); no LDS and no barriers.  UPPER: every coefficient matrix
// is upper triangular (C[k][b] = 0 for k > b), so columns 0 .. 15 take only
// vectors 0 .. 15 (the products skipped are exact zeros).
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename OT, bool UPPER>
__global__ __launch_bounds__(256) void k_bcomb64(const CItem *__restrict__ items, int64_t N)
{
    const CItem it = items[blockIdx.y];
    if (it.flag && *it.flag == 0) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
    const int64_t nrow = int64_t(blockIdx.x) * 64 + 16 * w + li;   // the row this lane reads
    const double2 *A = static_cast<const double2 *>(it.A);
    f64x4 orr[2], oi[2];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int q = 0; q < 4; ++q) orr[c][q] = oi[c][q] = 0.0;
    double2 a[8], b[8][2];
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {   // all operands of the item's K <= 32 issued first
        const int k = 4 * ks + lk;
        const bool kl = k < it.K;
        a[ks] = (kl && nrow < N) ? ld_global(A, (int64_t(k / it.ar) * it.astride + k % it.ar) * N + nrow)
                                 : make_double2(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int col = 16 * c + li;
            b[ks][c] = (kl && col < it.nb && !(UPPER && c == 0 && ks >= 4)) ? ld_global(it.C, int64_t(k) * it.ldc + col)
                                                                             : make_double2(0.0, 0.0);
        }
    }
#pragma unroll
    for (int ks = 0; ks < 8; ++ks)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            if (UPPER && c == 0 && ks >= 4) continue;
            orr[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks].x, b[ks][c].x, orr[c], 0, 0, 0);
            orr[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[ks].y, b[ks][c].y, orr[c], 0, 0, 0);
            oi[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks].x, b[ks][c].y, oi[c], 0, 0, 0);
            oi[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks].y, b[ks][c].x, oi[c], 0, 0, 0);
        }
    OT *out = static_cast<OT *>(it.out);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int col = 16 * c + li;
        if (col >= it.nb) continue;
        const int64_t ob = int64_t(it.ocol ? it.ocol[col] : col) * N;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t n = int64_t(blockIdx.x) * 64 + 16 * w + lk + 4 * q;
            if (n < N) {
                double2 y = make_double2(it.alpha * orr[c][q], it.alpha * oi[c][q]);
                if (it.beta != 0.0) y = cadd(y, cscale(it.beta, to_d2(out[ob + n])));
                out[ob + n] = from_d2<OT>(y);
            }
        }
    }
}

// Gram matrix G = W^H W of an item's r <= 32 FP64 columns (A and Bm the same
// vectors) over a chunk of L rows on the FP64 matrix cores, partial sums laid
// out as k_bdots' with 32 vectors per tile (summed by k_bdots_fin).  Lane l
// reads entry n = ns + l / 16 of column l % 16 (and of column 16 + l % 16): the
// same register is the A operand (conj(W) as rows) and the B operand (W as
// columns), so one load feeds both.  Tiles (0,0), (0,1), (1,1) of 16 x 16 are
// formed (the last two only when r > 16), (1,0) is written as the conjugate
// transpose of (0,1).  Wave w takes every fourth step of 4 rows; the waves'
// sums are added through LDS in a fixed order.
__global__ __launch_bounds__(256) void k_bgram64(const DItem *__restrict__ items, int64_t N, int nchunks, int64_t L,
                                                 double2 *__restrict__ part)
{
    const DItem it = items[blockIdx.y];
    if (it.flag && *it.flag == 0) return;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, li = lane & 15, lk = lane >> 4;
    const int r = it.kc;
    const bool two = r > 16;
    const int64_t n0 = int64_t(blockIdx.x) * L, n1 = min(N, n0 + L);
    const double2 *A = static_cast<const double2 *>(it.A);
    auto voff = [&](int v) { return (int64_t((it.k0 + v) / it.ar) * it.astride + (it.k0 + v) % it.ar) * N; };
    const bool l0 = li < r, l1 = 16 + li < r;
    const int64_t o0 = l0 ? voff(li) : 0, o1 = l1 ? voff(16 + li) : 0;
    f64x4 g[6];   // (0,0) re, im; (0,1) re, im; (1,1) re, im
#pragma unroll
    for (int e = 0; e < 6; ++e)
#pragma unroll
        for (int q = 0; q < 4; ++q) g[e][q] = 0.0;
    auto step = [&](double2 x0, double2 x1) {
        // conj(a) b: re = a.x b.x + a.y b.y, im = a.x b.y - a.y b.x
        g[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0.x, x0.x, g[0], 0, 0, 0);
        g[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0.y, x0.y, g[0], 0, 0, 0);
        g[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0.x, x0.y, g[1], 0, 0, 0);
        g[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(-x0.y, x0.x, g[1], 0, 0, 0);
        if (two) {
            g[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0.x, x1.x, g[2], 0, 0, 0);
            g[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0.y, x1.y, g[2], 0, 0, 0);
            g[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0.x, x1.y, g[3], 0, 0, 0);
            g[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(-x0.y, x1.x, g[3], 0, 0, 0);
            g[4] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1.x, x1.x, g[4], 0, 0, 0);
            g[4] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1.y, x1.y, g[4], 0, 0, 0);
            g[5] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1.x, x1.y, g[5], 0, 0, 0);
            g[5] = __builtin_amdgcn_mfma_f64_16x16x4f64(-x1.y, x1.x, g[5], 0, 0, 0);
        }
    };
    const double2 z = make_double2(0.0, 0.0);
    int64_t ns = n0 + 4 * w;
    for (; ns + 52 <= n1; ns += 64) {   // four whole steps per trip (rows up to ns + 51), loads first
        double2 x0[4], x1[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t n = ns + 16 * u + lk;
            x0[u] = l0 ? ld_global(A, o0 + n) : z;
            x1[u] = (two && l1) ? ld_global(A, o1 + n) : z;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) step(x0[u], x1[u]);
    }
    for (; ns < n1; ns += 16) {
        const int64_t n = ns + lk;
        const bool nl = n < n1;
        step((nl && l0) ? ld_global(A, o0 + n) : z, (nl && two && l1) ? ld_global(A, o1 + n) : z);
    }
    __shared__ double red[3][24][64];
    if (w > 0)
#pragma unroll
        for (int e = 0; e < 6; ++e)
#pragma unroll
            for (int q = 0; q < 4; ++q) red[w - 1][4 * e + q][lane] = g[e][q];
    __syncthreads();
    if (w > 0) return;
#pragma unroll 1
    for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int e = 0; e < 6; ++e)
#pragma unroll
            for (int q = 0; q < 4; ++q) g[e][q] += red[v][4 * e + q][lane];
    double2 *o = part + (int64_t(blockIdx.y) * nchunks + blockIdx.x) * 32 * BMAX;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int v = lk + 4 * q;   // output row of value q, column li
        if (v < r && l0) o[v * BMAX + li] = make_double2(g[0][q], g[1][q]);
        if (two && v < r && l1) {
            o[v * BMAX + 16 + li] = make_double2(g[2][q], g[3][q]);
            o[(16 + li) * BMAX + v] = make_double2(g[2][q], -g[3][q]);
        }
        if (two && 16 + v < r && l1) o[(16 + v) * BMAX + 16 + li] = make_double2(g[4][q], g[5][q]);
    }
}

// dst[i * N + n] = src[cols[i] * N + n]
__global__ __launch_bounds__(256) void k_bgather(int64_t N, const double2 *__restrict__ src, const int *__restrict__ cols,
                                                 double2 *__restrict__ dst)
{
    const int i = blockIdx.y;
    const double2 *a = src + int64_t(cols[i]) * N;
    double2 *b = dst + int64_t(i) * N;
    for (int64_t n = int64_t(blockIdx.x) * 256 + threadIdx.x; n < N; n += int64_t(gridDim.x) * 256) b[n] = a[n];
}

// squared norms of columns cols[i] of src, partial over row chunks, then summed
// in a fixed order
__global__ __launch_bounds__(256) void k_bnorm_part(int64_t N, const double2 *__restrict__ src,
                                                    const int *__restrict__ cols, double *__restrict__ part)
{
    const int i = blockIdx.y;
    const double2 *a = src + int64_t(cols[i]) * N;
    double s = 0.0;
    for (int64_t n = int64_t(blockIdx.x) * 256 + threadIdx.x; n < N; n += int64_t(gridDim.x) * 256)
        s = fma(a[n].x, a[n].x, fma(a[n].y, a[n].y, s));
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[int64_t(i) * gridDim.x + blockIdx.x] = red[0];
}
__global__ void k_bnorm_fin(int nparts, int count, const double *__restrict__ part, double *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    double s = 0.0;
    for (int c = 0; c < nparts; ++c) s += part[int64_t(i) * nparts + c];
    out[i] = std::sqrt(s);
}

// Device state of one group (fixed regions sized for r, q <= BMAX and m steps).
struct GDev {
    double2 *C2;        // projection coefficients of the second pass, ((m+1) r) x r (the first
                        // pass writes its own into Hbar)
    double2 *G1, *G2;   // Gram matrices of T V_j before the passes and of W after the last one, r x r
    double2 *Rt;        // block column j at Rt + j * (m+1) r r: rows 0 .. (j+2) r of Hbar, reduced in place
    double2 *U;         // Householder vectors of block column j: 2r x r at U + j * 2 r r
    double2 *T;         // triangular factor of those reflectors (Q = I - U T U^H): r x r at T + j r r
    double2 *Mw;        // M = U T^H of block column j (Q^H x = x - M U^H x): 2r x r at Mw + j * 2 r r
    double2 *Tinv;      // R^{-1} of the current step, r x r
    double2 *Gv;        // E_1 S with the reflectors applied, ((m+1) r) x q
    double2 *Y;         // least-squares solution times the column scales, (m r) x q
    double *est;        // per-column residual estimate (scaled units)
    double *scale;      // per-column residual norm at the start of the cycle
    int *flag;          // [0] second Gram-Schmidt pass needed, [2 + (j & 1)] partial breakdown at step j
    int r, q;
};

// The Gram matrix after the first update (G2) against the one before (G1)
// decides whether a second pass runs: any column that kept less than `keep`
// of its norm squared (0: never).
__global__ __launch_bounds__(64) void k_bflag(GDev *__restrict__ gd, const int *__restrict__ gids, double keep)
{
    GDev g = gd[gids[blockIdx.x]];
    const int r = g.r, a = threadIdx.x;
    const bool lost = keep > 0.0 && a < r && g.G2[a * r + a].x < keep * g.G1[a * r + a].x;
    const unsigned long long any = __ballot(lost);
    if (a == 0) g.flag[0] = any != 0ull;
}

// Complete Hbar(:, j) = [C1 + C2; R] (C1 already in place) with R^H R = G2 (Cholesky of the Gram
// matrix of W after the last pass), and R^{-1} for the next basis block.  A
// pivot at or below delta^2 times the largest squared column norm of T V_j
// (G2_aa + sum_k |H_ka|^2: the part removed plus the part kept) marks a partial
// breakdown; that direction gets a zero row in R.
__global__ __launch_bounds__(256) void k_bchol(GDev *__restrict__ gd, const int *__restrict__ gids, int j, int m,
                                               double delta)
{
    GDev g = gd[gids[blockIdx.x]];
    const int r = g.r, K = (j + 1) * r, t = threadIdx.x;
    const bool two = g.flag[0] != 0;
    __shared__ double2 Gs[BMAX][BMAX + 1];
    __shared__ double2 L[BMAX][BMAX + 1];
    __shared__ double2 Ti[BMAX][BMAX + 1];
    __shared__ double gmax;
    __shared__ int brk;
    double2 *H = g.Rt + int64_t(j) * (m + 1) * r * r;   // ((m+1) r) x r, row-major
    if (two)   // the first pass wrote its coefficients into H directly
        for (int e = t; e < K * r; e += 256) H[e] = cadd(H[e], g.C2[e]);
    __shared__ double cn[8][BMAX];
    __syncthreads();
    {   // squared column norms of H(0 : K, :), 8 partial sums per column
        const int a = t & 31, part = t >> 5;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        if (a < r) {
            int k = part;
            for (; k + 120 < K; k += 128) {   // 16 rows per trip, all loads issued first
                double2 h[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) h[u] = H[int64_t(k + 8 * u) * r + a];
#pragma unroll
                for (int u = 0; u < 16; u += 4) {
                    s0 += h[u].x * h[u].x + h[u].y * h[u].y;
                    s1 += h[u + 1].x * h[u + 1].x + h[u + 1].y * h[u + 1].y;
                    s2 += h[u + 2].x * h[u + 2].x + h[u + 2].y * h[u + 2].y;
                    s3 += h[u + 3].x * h[u + 3].x + h[u + 3].y * h[u + 3].y;
                }
            }
            for (; k + 24 < K; k += 32) {
                const double2 h0 = H[int64_t(k) * r + a], h1 = H[int64_t(k + 8) * r + a];
                const double2 h2 = H[int64_t(k + 16) * r + a], h3 = H[int64_t(k + 24) * r + a];
                s0 += h0.x * h0.x + h0.y * h0.y;
                s1 += h1.x * h1.x + h1.y * h1.y;
                s2 += h2.x * h2.x + h2.y * h2.y;
                s3 += h3.x * h3.x + h3.y * h3.y;
            }
            for (; k < K; k += 8) {
                const double2 h = H[int64_t(k) * r + a];
                s0 += h.x * h.x + h.y * h.y;
            }
        }
        cn[part][a] = (s0 + s1) + (s2 + s3);
    }
    for (int e = t; e < BMAX * (BMAX + 1); e += 256) {
        (&L[0][0])[e] = make_double2(0.0, 0.0);
        (&Ti[0][0])[e] = make_double2(0.0, 0.0);
    }
    for (int e = t; e < r * r; e += 256) Gs[e / r][e % r] = g.G2[e];
    __syncthreads();
    if (t == 0) {
        double mx = 0.0;
        for (int a = 0; a < r; ++a) {
            double sv = Gs[a][a].x;
            for (int q = 0; q < 8; ++q) sv += cn[q][a];
            mx = fmax(mx, sv);
        }
        gmax = mx;
        brk = 0;
    }
    __syncthreads();
    // right-looking Cholesky of the lower triangle of Gs (G2 = L L^H), one
    // barrier per column: every thread reads the pivot, column k of L and the
    // trailing update G(i, l) -= G(i, k) conj(G(l, k)) / G(k, k) (l > k, the
    // columns the update writes) come from column k of Gs in the same phase
    for (int k = 0; k < r; ++k) {
        const double p = Gs[k][k].x;
        const bool ok = p > delta * delta * gmax;
        const double d = ok ? std::sqrt(p) : 0.0;
        if (t == 0 && !ok) brk = 1;
        if (t >= k && t < r)
            L[t][k] = t == k ? make_double2(d, 0.0) : (ok ? cscale(1.0 / d, Gs[t][k]) : make_double2(0.0, 0.0));
        if (ok) {
            const double ip = 1.0 / p;
            for (int e = t; e < r * r; e += 256) {
                const int i = e / r, l = e % r;
                if (l > k && l <= i)
                    Gs[i][l] = csub(Gs[i][l], cscale(ip, cmul(Gs[i][k], make_double2(Gs[l][k].x, -Gs[l][k].y))));
            }
        }
        __syncthreads();
    }
    // R = L^H into rows K .. K + r of H
    for (int e = t; e < r * r; e += 256) {
        const int a = e / r, b = e % r;
        const double2 v = b >= a ? make_double2(L[b][a].x, -L[b][a].y) : make_double2(0.0, 0.0);
        H[int64_t(K + a) * r + b] = v;
    }
    // L^{-1} by forward substitution, row i at a time, 8 lanes per column c <= i
    // (Gs is free now and holds it); R^{-1} = (L^{-1})^H; zero for broken pivots
    for (int i = 0; i < r; ++i) {
        const int c = t >> 3, part = t & 7;
        double2 sv = make_double2(0.0, 0.0);
        if (c <= i && c < r)
            for (int l = c + part; l < i; l += 8) sv = cadd(sv, cmul(L[i][l], Gs[l][c]));
        for (int o = 4; o > 0; o >>= 1) {
            sv.x += __shfl_xor(sv.x, o, 8);
            sv.y += __shfl_xor(sv.y, o, 8);
        }
        if (part == 0 && c <= i && c < r) {
            const double lii = L[i][i].x;
            const double2 rhs = c == i ? make_double2(1.0, 0.0) : make_double2(0.0, 0.0);
            Gs[i][c] = lii > 0.0 ? cscale(1.0 / lii, csub(rhs, sv)) : make_double2(0.0, 0.0);
        }
        __syncthreads();
    }
    for (int e = t; e < r * r; e += 256) {
        const int a = e / r, b = e % r;
        Ti[a][b] = b >= a ? make_double2(Gs[b][a].x, -Gs[b][a].y) : make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int e = t; e < r * r; e += 256) g.Tinv[e] = Ti[e / r][e % r];
    if (t == 0) g.flag[2 + (j & 1)] = brk;
}

// Apply Q^H = I - U T^H U^H (U: 2r x r, T: r x r upper) to X (2r x nc) in LDS.
// All 256 threads take part; W1, W2 are r x nc scratch.
template <int XC>
__device__ void wy_apply(double2 (*X)[XC], double2 (*Us)[BMAX + 1], double2 (*Ts)[BMAX + 1], double2 (*W1)[XC],
                         double2 (*W2)[XC], int r, int nc)
{
    const int t = threadIdx.x;
    for (int e = t; e < r * nc; e += 256) {   // W1 = U^H X
        const int a = e / nc, c = e % nc;
        double2 sv = make_double2(0.0, 0.0);
        for (int i = a; i < 2 * r; ++i) sv = cadd(sv, cmulc(Us[i][a], X[i][c]));
        W1[a][c] = sv;
    }
    __syncthreads();
    for (int e = t; e < r * nc; e += 256) {   // W2 = T^H W1
        const int a = e / nc, c = e % nc;
        double2 sv = make_double2(0.0, 0.0);
        for (int b = 0; b <= a; ++b) sv = cadd(sv, cmulc(Ts[b][a], W1[b][c]));
        W2[a][c] = sv;
    }
    __syncthreads();
    for (int e = t; e < 2 * r * nc; e += 256) {   // X -= U W2
        const int i = e / nc, c = e % nc;
        double2 sv = X[i][c];
        const int amax = min(i, r - 1);
        for (int a = 0; a <= amax; ++a) sv = csub(sv, cmul(Us[i][a], W2[a][c]));
        X[i][c] = sv;
    }
    __syncthreads();
}

constexpr int CS = 8;   // columns of the new block column per workgroup of k_bls_apply
static_assert(BMAX * CS <= 256, "k_bls_apply keeps one entry of the r x CS row window per thread");

// The reflectors of block columns 0 .. j-1 applied, in order, to the new block
// column of Hbar as x -= M_i (U_i^H x); the columns are independent, CS of them
// per workgroup.  Block i works on rows ir .. ir + 2r: its upper half is final
// afterwards and is written back, its lower half stays in LDS as the next
// block's upper half; U and M of the next block are loaded into registers
// while the current block is applied.
__global__ __launch_bounds__(256) void k_bls_apply(GDev *__restrict__ gd, const int *__restrict__ gids, int j, int m)
{
    GDev g = gd[gids[blockIdx.x]];
    const int r = g.r, c0 = blockIdx.y * CS, nc = min(CS, r - c0), t = threadIdx.x;
    if (nc <= 0 || j == 0) return;
    __shared__ double2 X[2 * BMAX][CS + 1];
    __shared__ double2 Us[2 * BMAX][BMAX + 1];
    __shared__ double2 Ms[2 * BMAX][BMAX + 1];
    __shared__ double2 W1[BMAX][CS + 1];
    double2 *H = g.Rt + int64_t(j) * (m + 1) * r * r;
    const int nu = 2 * r * r;   // entries of U (and of M) per block column, <= 2048
    double2 pu[8], pm[8];
    double2 ph = make_double2(0.0, 0.0);   // the row entry t of the next lower half (r nc <= 256 entries)
    auto fetch = [&](int i) {
        const double2 *Ui = g.U + int64_t(i) * nu, *Mi = g.Mw + int64_t(i) * nu;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = t + 256 * u;
            pu[u] = e < nu ? Ui[e] : make_double2(0.0, 0.0);
            pm[u] = e < nu ? Mi[e] : make_double2(0.0, 0.0);
        }
        // rows (i + 1) r .. + r of the column block, the lower half of block i's window
        // (untouched until then: this workgroup writes only rows below the window)
        if (i + 1 <= j && t < r * nc) ph = H[int64_t((i + 1) * r + t / nc) * r + c0 + t % nc];
    };
    fetch(0);
    for (int e = t; e < 2 * r * nc; e += 256) X[e / nc][e % nc] = H[int64_t(e / nc) * r + c0 + e % nc];
    for (int i = 0; i < j; ++i) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = t + 256 * u;
            if (e < nu) {
                Us[e / r][e % r] = pu[u];
                Ms[e / r][e % r] = pm[u];
            }
        }
        __syncthreads();
        if (i + 1 < j) fetch(i + 1);
        for (int e = t; e < r * nc; e += 256) {   // W1 = U^H X, four independent partial sums
            const int a = e / nc, c = e % nc;
            double2 s0 = make_double2(0.0, 0.0), s1 = s0, s2 = s0, s3 = s0;
            int row = a;
            for (; row + 3 < 2 * r; row += 4) {
                s0 = cadd(s0, cmulc(Us[row][a], X[row][c]));
                s1 = cadd(s1, cmulc(Us[row + 1][a], X[row + 1][c]));
                s2 = cadd(s2, cmulc(Us[row + 2][a], X[row + 2][c]));
                s3 = cadd(s3, cmulc(Us[row + 3][a], X[row + 3][c]));
            }
            for (; row < 2 * r; ++row) s0 = cadd(s0, cmulc(Us[row][a], X[row][c]));
            W1[a][c] = cadd(cadd(s0, s1), cadd(s2, s3));
        }
        __syncthreads();
        for (int e = t; e < 2 * r * nc; e += 256) {   // X -= M W1, four independent partial sums
            const int row = e / nc, c = e % nc;
            const int amax = min(row, r - 1);
            double2 s0 = make_double2(0.0, 0.0), s1 = s0, s2 = s0, s3 = s0;
            int a = 0;
            for (; a + 3 <= amax; a += 4) {
                s0 = cadd(s0, cmul(Ms[row][a], W1[a][c]));
                s1 = cadd(s1, cmul(Ms[row][a + 1], W1[a + 1][c]));
                s2 = cadd(s2, cmul(Ms[row][a + 2], W1[a + 2][c]));
                s3 = cadd(s3, cmul(Ms[row][a + 3], W1[a + 3][c]));
            }
            for (; a <= amax; ++a) s0 = cadd(s0, cmul(Ms[row][a], W1[a][c]));
            X[row][c] = csub(X[row][c], cadd(cadd(s0, s1), cadd(s2, s3)));
        }
        __syncthreads();
        // rows ir .. ir + r are final; shift the lower half up and take the next rows
        // (fetched with block i + 1's reflectors)
        if (i + 1 < j) {
            if (t < r * nc) {
                const int row = t / nc, c = t % nc;
                H[int64_t(i * r + row) * r + c0 + c] = X[row][c];
                X[row][c] = X[r + row][c];
                X[r + row][c] = ph;
            }
        } else {
            for (int e = t; e < 2 * r * nc; e += 256) H[int64_t(i * r + e / nc) * r + c0 + e % nc] = X[e / nc][e % nc];
        }
    }
}

// New reflectors for rows jr .. jr + 2r of the new block column of Hbar (the
// earlier ones already applied), their triangular factor, the same applied to
// E_1 S, and the residual estimates.  One workgroup per group.
__global__ __launch_bounds__(256) void k_bls_qr(GDev *__restrict__ gd, const int *__restrict__ gids, int j, int m)
{
    GDev g = gd[gids[blockIdx.x]];
    const int r = g.r, q = g.q, t = threadIdx.x;
    __shared__ double2 X[2 * BMAX][BMAX + 1];
    __shared__ double2 Us[2 * BMAX][BMAX + 1];
    __shared__ double2 Ts[BMAX][BMAX + 1];
    __shared__ double2 W1[BMAX][BMAX + 1];
    __shared__ double2 W2[BMAX][BMAX + 1];
    __shared__ double2 alpha_s;
    __shared__ double beta_s;
    double2 *H = g.Rt + int64_t(j) * (m + 1) * r * r;
    // Householder QR of rows jr .. jr + 2r
    for (int e = t; e < 2 * r * r; e += 256) {
        X[e / r][e % r] = H[int64_t(j) * r * r + e];
        Us[e / r][e % r] = make_double2(0.0, 0.0);
    }
    for (int e = t; e < r * r; e += 256) Ts[e / r][e % r] = make_double2(0.0, 0.0);
    __syncthreads();
    for (int k = 0; k < r; ++k) {
        if (t < 64) {   // one wave: the reflector of column k
            double s = 0.0;
            for (int i = k + t; i < 2 * r; i += 64) s += X[i][k].x * X[i][k].x + X[i][k].y * X[i][k].y;
            for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
            const double nx = std::sqrt(s);
            const double2 x0 = X[k][k];
            const double ax0 = std::sqrt(x0.x * x0.x + x0.y * x0.y);
            const double2 ph = ax0 > 0.0 ? make_double2(x0.x / ax0, x0.y / ax0) : make_double2(1.0, 0.0);
            const double2 al = make_double2(-ph.x * nx, -ph.y * nx);
            // v = x - alpha e_1; |v|^2 = |x|^2 - 2 Re(conj(alpha) x0) + |alpha|^2 = 2 nx (nx + |x0|)
            const double vv = 2.0 * nx * (nx + ax0);
            for (int i = k + t; i < 2 * r; i += 64) Us[i][k] = i == k ? csub(X[k][k], al) : X[i][k];
            if (t == 0) {
                alpha_s = al;
                beta_s = vv > 0.0 ? 2.0 / vv : 0.0;
                Ts[k][k] = make_double2(vv > 0.0 ? 2.0 / vv : 0.0, 0.0);
            }
        }
        __syncthreads();
        const double beta = beta_s;
        // apply to columns k+1 .. r-1: x -= beta v (v^H x), one column per thread group of 8
        for (int c = k + 1 + (t >> 3); c < r; c += 32) {
            const int l = t & 7;
            double2 s = make_double2(0.0, 0.0);
            for (int i = k + l; i < 2 * r; i += 8) s = cadd(s, cmulc(Us[i][k], X[i][c]));
            for (int o = 4; o > 0; o >>= 1) {
                s.x += __shfl_xor(s.x, o, 8);
                s.y += __shfl_xor(s.y, o, 8);
            }
            for (int i = k + l; i < 2 * r; i += 8) X[i][c] = csub(X[i][c], cscale(beta, cmul(Us[i][k], s)));
        }
        __syncthreads();
        if (t == 0) X[k][k] = alpha_s;
        for (int i = k + 1 + t; i < 2 * r; i += 256) X[i][k] = make_double2(0.0, 0.0);
        __syncthreads();
    }
    // T of the new reflectors: T(0:k, k) = -beta_k T(0:k, 0:k) (U(:, 0:k)^H u_k)
    for (int e = t; e < r * r; e += 256) {   // W1 = U^H U (upper part used)
        const int a = e / r, b = e % r;
        double2 s = make_double2(0.0, 0.0);
        if (a < b)
            for (int i = b; i < 2 * r; ++i) s = cadd(s, cmulc(Us[i][a], Us[i][b]));
        W1[a][b] = s;
    }
    __syncthreads();
    for (int k = 1; k < r; ++k) {
        if (t < k) {
            double2 s = make_double2(0.0, 0.0);
            for (int l = t; l < k; ++l) s = cadd(s, cmul(Ts[t][l], W1[l][k]));
            W2[t][0] = cscale(-Ts[k][k].x, s);
        }
        __syncthreads();
        if (t < k) Ts[t][k] = W2[t][0];
        __syncthreads();
    }
    double2 *Uj = g.U + int64_t(j) * 2 * r * r, *Tj = g.T + int64_t(j) * r * r, *Mj = g.Mw + int64_t(j) * 2 * r * r;
    for (int e = t; e < 2 * r * r; e += 256) {
        H[int64_t(j) * r * r + e] = X[e / r][e % r];
        Uj[e] = Us[e / r][e % r];
        const int row = e / r, a = e % r;   // M = U T^H: sum over b >= a, b <= row
        double2 sv = make_double2(0.0, 0.0);
        const int bmax = min(row, r - 1);
        for (int b = a; b <= bmax; ++b) sv = cadd(sv, cmul(Us[row][b], make_double2(Ts[a][b].x, -Ts[a][b].y)));
        Mj[e] = sv;
    }
    for (int e = t; e < r * r; e += 256) Tj[e] = Ts[e / r][e % r];
    __syncthreads();
    // E_1 S rows jr .. jr + 2r, q columns
    for (int e = t; e < 2 * r * q; e += 256) X[e / q][e % q] = g.Gv[int64_t(j) * r * q + e];
    __syncthreads();
    wy_apply<BMAX + 1>(X, Us, Ts, W1, W2, r, q);
    for (int e = t; e < 2 * r * q; e += 256) g.Gv[int64_t(j) * r * q + e] = X[e / q][e % q];
    if (t < q) {
        double s = 0.0;
        for (int i = r; i < 2 * r; ++i) s += X[i][t].x * X[i][t].x + X[i][t].y * X[i][t].y;
        g.est[t] = std::sqrt(s);
    }
}

// Y = R^{-1} Gv(0 : J r, :) by right-looking block back substitution (R upper
// triangular, block column b of R at Rt + b (m+1) r r), one launch per block
// row I from the last: workgroup b (block row b <= I) takes R(b, I+1) Y_{I+1}
// off its rows of Gv, and the workgroup of block row I then solves
// R_II Y_I = Gv_I.  Y holds the solution times the column scales; Gv is consumed.
__global__ __launch_bounds__(256) void k_bls_back(GDev *__restrict__ gd, const int *__restrict__ gids,
                                                  const int *__restrict__ steps, int I, int m)
{
    const int gid = gids[blockIdx.x];
    GDev g = gd[gid];
    const int r = g.r, q = g.q, t = threadIdx.x, b = blockIdx.y, J = steps[gid];
    if (I >= J || b > I) return;
    const int64_t bs = int64_t(m + 1) * r * r;
    __shared__ double2 Ys[BMAX][BMAX + 1];
    __shared__ double2 S[BMAX][BMAX + 1];
    __shared__ double2 D[BMAX][BMAX + 1];
    if (I + 1 < J) {   // Y_{I+1} without the column scales
        for (int e = t; e < r * q; e += 256) {
            const int c = e % q;
            const double sc = g.scale[c];
            const double2 y = g.Y[int64_t((I + 1) * r + e / q) * q + c];
            Ys[e / q][c] = sc > 0.0 ? cscale(1.0 / sc, y) : make_double2(0.0, 0.0);
        }
        __syncthreads();
        const double2 *Rb = g.Rt + (I + 1) * bs;
        for (int e = t; e < r * q; e += 256) {
            const int row = b * r + e / q, c = e % q;
            double2 sv = g.Gv[int64_t(row) * q + c];
            const double2 *Rr = Rb + int64_t(row) * r;
            for (int k = 0; k < r; ++k) sv = csub(sv, cmul(Rr[k], Ys[k][c]));
            g.Gv[int64_t(row) * q + c] = sv;
        }
    }
    if (b != I) return;
    __syncthreads();
    const double2 *Rb = g.Rt + I * bs;
    for (int e = t; e < r * r; e += 256) D[e / r][e % r] = Rb[int64_t(I * r + e / r) * r + e % r];
    for (int e = t; e < r * q; e += 256) S[e / q][e % q] = g.Gv[int64_t(I * r + e / q) * q + e % q];
    __syncthreads();
    if (t < q) {
        for (int a = r - 1; a >= 0; --a) {
            double2 sv = S[a][t];
            for (int c = a + 1; c < r; ++c) sv = csub(sv, cmul(D[a][c], S[c][t]));
            const double2 d = D[a][a];
            const double dd = d.x * d.x + d.y * d.y;
            S[a][t] = dd > 0.0 ? make_double2((sv.x * d.x + sv.y * d.y) / dd, (sv.y * d.x - sv.x * d.y) / dd)
                               : make_double2(0.0, 0.0);
        }
    }
    __syncthreads();
    for (int e = t; e < r * q; e += 256) g.Y[int64_t(I * r + e / q) * q + e % q] = cscale(g.scale[e % q], S[e / q][e % q]);
}

// Start-of-cycle uploads of every group in one launch: dst[0 .. n) = src, then
// zeros up to nzero (doubles).
struct SItem {
    const double *src;
    double *dst;
    int64_t n, nzero;
};

__global__ __launch_bounds__(256) void k_bscatter(const SItem *__restrict__ items)
{
    const SItem t = items[blockIdx.x];
    for (int64_t i = threadIdx.x; i < t.nzero; i += 256) t.dst[i] = i < t.n ? t.src[i] : 0.0;
}

using cd = std::complex<double>;

// Small per-launch tables: staged in pinned host memory and copied to a device
// mirror on the stream, all tables staged since the last copy in one transfer
// (flush).  Space is reused only after a stream synchronisation, when every
// copy and every kernel reading the tables has finished.
struct Arena {
    char *h = nullptr, *d = nullptr;
    size_t cap = 0, used = 0, flushed = 0;
    explicit Arena(size_t n) : cap(n)
    {
        BIE_HIP(hipHostMalloc(reinterpret_cast<void **>(&h), n));
        BIE_HIP(hipMalloc(reinterpret_cast<void **>(&d), n));
    }
    ~Arena()
    {
        if (h) (void)hipHostFree(h);
        if (d) (void)hipFree(d);
    }
    size_t stage(const void *src, size_t bytes)
    {
        const size_t off = (used + 255) & ~size_t(255);
        if (off + bytes > cap) throw Error(BIE_ENOMEM, "block GMRES: table space exhausted");
        std::memcpy(h + off, src, bytes);
        used = off + bytes;
        return off;
    }
    // device address of a staged copy of v (valid after the next flush)
    template <typename T>
    T *put(const std::vector<T> &v)
    {
        return reinterpret_cast<T *>(d + stage(v.data(), v.size() * sizeof(T)));
    }
    void flush(hipStream_t s)
    {
        if (used > flushed)
            BIE_HIP(hipMemcpyAsync(d + flushed, h + flushed, used - flushed, hipMemcpyHostToDevice, s));
        flushed = used;
    }
    // staged copy to another device buffer
    template <typename T>
    void copy_to(T *dst, const T *src, size_t count, hipStream_t s)
    {
        flush(s);
        const size_t off = stage(src, count * sizeof(T));
        BIE_HIP(hipMemcpyAsync(dst, h + off, count * sizeof(T), hipMemcpyHostToDevice, s));
        flushed = used;
    }
    void reset() { used = flushed = 0; }
};

struct HGroup {
    std::vector<int> rhs;          // chunk-local right-hand sides of the columns
    std::vector<double> scale, target;
    int q = 0, r = 0, c0 = 0, qoff = 0, cap = 0, steps = 0;
    bool active = false;
};

int pick_nb(int n) { return n <= 4 ? 4 : n <= 8 ? 8 : n <= 16 ? 16 : 32; }

// U = 4: tiles of 128 basis vectors (basis dots); U = 1: tiles of 32 (Gram matrices)
template <typename AT, int U = 4>
void launch_dots(const DItem *d, size_t ni, int64_t N, double2 *part, int nbmax, hipStream_t s)
{
    if (ni == 0) return;
    const int64_t nch = std::max<int64_t>(1, std::min<int64_t>((1024 + int64_t(ni) - 1) / int64_t(ni), (N + 127) / 128));
    const int64_t L = ((N + nch - 1) / nch + DS - 1) / DS * DS;
    const int nchunks = int((N + L - 1) / L);
    const dim3 grid{ unsigned(nchunks), unsigned(ni) };
    const int nq = (nbmax + 3) / 4;
    if (nq <= 1) hipLaunchKernelGGL((k_bdots<AT, 1, U>), grid, dim3(256), 0, s, d, N, nchunks, L, part);
    else if (nq <= 2) hipLaunchKernelGGL((k_bdots<AT, 2, U>), grid, dim3(256), 0, s, d, N, nchunks, L, part);
    else if (nq <= 4) hipLaunchKernelGGL((k_bdots<AT, 4, U>), grid, dim3(256), 0, s, d, N, nchunks, L, part);
    else hipLaunchKernelGGL((k_bdots<AT, 8, U>), grid, dim3(256), 0, s, d, N, nchunks, L, part);
    hipLaunchKernelGGL(k_bdots_fin, dim3(unsigned(ni), unsigned((32 * U * BMAX) / 64)), dim3(256), 0, s, d, nchunks,
                       32 * U, (const double2 *)part);
    BIE_HIP(hipGetLastError());
}

template <typename AT, typename OT>
void launch_comb(const CItem *d, size_t ni, int64_t N, int nbmax, hipStream_t s)
{
    if (ni == 0) return;
    const dim3 grid{ unsigned((N + 127) / 128), unsigned(ni) };
    switch (pick_nb(nbmax)) {
    case 4: hipLaunchKernelGGL((k_bcomb<AT, OT, 4>), grid, dim3(256), 0, s, d, N); break;
    case 8: hipLaunchKernelGGL((k_bcomb<AT, OT, 8>), grid, dim3(256), 0, s, d, N); break;
    case 16: hipLaunchKernelGGL((k_bcomb<AT, OT, 16>), grid, dim3(256), 0, s, d, N); break;
    default: hipLaunchKernelGGL((k_bcomb<AT, OT, 32>), grid, dim3(256), 0, s, d, N); break;
    }
    BIE_HIP(hipGetLastError());
}

// Gram matrices W^H W of FP64 columns (items with A == Bm, kc == nb <= 32): the
// FP64 matrix cores, or the vector ALUs with BIE_COMB64=valu (for comparison)
void launch_gram64(const DItem *d, size_t ni, int64_t N, double2 *part, int nbmax, hipStream_t s)
{
    static const bool valu = [] {
        const char *e = getenv("BIE_COMB64");
        return e && std::strcmp(e, "valu") == 0;
    }();
    if (ni == 0) return;
    if (valu) return launch_dots<double2, 1>(d, ni, N, part, nbmax, s);
    const int64_t nch = std::max<int64_t>(1, std::min<int64_t>((N + 63) / 64, (768 + int64_t(ni) - 1) / int64_t(ni)));
    const int64_t L = ((N + nch - 1) / nch + 15) / 16 * 16;
    const int nchunks = int((N + L - 1) / L);
    hipLaunchKernelGGL(k_bgram64, dim3(unsigned(nchunks), unsigned(ni)), dim3(256), 0, s, d, N, nchunks, L, part);
    hipLaunchKernelGGL(k_bdots_fin, dim3(unsigned(ni), unsigned((32 * BMAX) / 64)), dim3(256), 0, s, d, nchunks, 32,
                       (const double2 *)part);
    BIE_HIP(hipGetLastError());
}

// Update whose vectors are FP64 and whose items have K <= 32 (every item of the
// block solver's scalings): the FP64 matrix cores, or the vector ALUs with
// BIE_COMB64=valu (for comparison)
template <typename OT>
void launch_comb64(const CItem *d, size_t ni, int64_t N, int nbmax, hipStream_t s, bool upper)
{
    static const bool valu = [] {
        const char *e = getenv("BIE_COMB64");
        return e && std::strcmp(e, "valu") == 0;
    }();
    if (ni == 0) return;
    if (valu) return launch_comb<double2, OT>(d, ni, N, nbmax, s);
    const dim3 grid{ unsigned((N + 63) / 64), unsigned(ni) };
    if (upper) hipLaunchKernelGGL((k_bcomb64<OT, true>), grid, dim3(256), 0, s, d, N);
    else hipLaunchKernelGGL((k_bcomb64<OT, false>), grid, dim3(256), 0, s, d, N);
    BIE_HIP(hipGetLastError());
}

// the basis kernels: BF16 three-term splits with the basis read straight into
// the operands (default), the same with the basis staged in LDS
// (BIE_BASIS_MFMA=lds, and the dots whenever N % 4 != 0), or the FP32 matrix
// cores (BIE_BASIS_MFMA=fp32, complex64 basis); the choices for comparison
enum { BASIS_DIRECT = 0, BASIS_LDS = 1, BASIS_FP32 = 2 };
int basis_mode()
{
    static const int v = [] {
        const char *e = getenv("BIE_BASIS_MFMA");
        if (e && std::strcmp(e, "fp32") == 0) return int(BASIS_FP32);
        if (e && std::strcmp(e, "lds") == 0) return int(BASIS_LDS);
        return int(BASIS_DIRECT);
    }();
    return v;
}

// XCD-aware order of the basis dots' workgroups (BIE_BDOTS_XCD=0 keeps the
// launch order, for comparison)
int bdots_xcd()
{
    static const int v = [] {
        const char *e = getenv("BIE_BDOTS_XCD");
        return (e && std::strcmp(e, "0") == 0) ? 0 : 1;
    }();
    return v;
}

// workgroups of the direct basis dots resident on the whole GPU at once
// (one device type per process)
template <typename VT>
int64_t bdots_slots()
{
    static const int64_t v = [] {
        int dev = 0, cus = 0, nb = 0;
        BIE_HIP(hipGetDevice(&dev));
        BIE_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        BIE_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_bdots_bd<VT>, 256, 0));
        return std::max<int64_t>(1, int64_t(cus) * std::max(nb, 1));
    }();
    return v;
}

// Row chunks per basis-dots item: every workgroup does the same work, so the
// count of workgroups is chosen to fill whole rounds of the resident slots
// (the last round of a plain count can run nearly empty); among counts of at
// least the slots' worth of workgroups (or all 128-row chunks) and at most
// twice it, the one with the best filled fraction, then the fewest chunks;
// one chunk when the items alone exceed that.  ni * chunks <= ni + 2 slots
// (the partial sums' buffer is sized for that).
int64_t dots_chunks(int64_t ni, int64_t N, int64_t slots)
{
    const int64_t maxch = std::max<int64_t>(1, (N + 127) / 128);
    const int64_t need = std::min(slots, ni * maxch);
    int64_t best = 1;
    double beff = -1.0;
    for (int64_t c = 1; c <= maxch && ni * c <= 2 * slots; ++c) {
        const int64_t tot = ni * c;
        if (tot < need) continue;
        const double eff = double(tot) / double(((tot + slots - 1) / slots) * slots);
        if (eff > beff + 1e-9) {
            beff = eff;
            best = c;
        }
    }
    return best;
}

template <typename VT>
void launch_dots_mf(const DItem *d, size_t ni, int64_t N, double2 *part, hipStream_t s)
{
    if (ni == 0) return;
    const bool direct = basis_mode() == BASIS_DIRECT && N % 4 == 0;
    int64_t nch = std::max<int64_t>(1, std::min<int64_t>((1024 + int64_t(ni) - 1) / int64_t(ni), (N + 127) / 128));
    if (direct) nch = dots_chunks(int64_t(ni), N, bdots_slots<VT>());
    const int64_t L = ((N + nch - 1) / nch + 31) / 32 * 32;
    const int nchunks = int((N + L - 1) / L);
    const dim3 grid{ unsigned(nchunks), unsigned(ni) };
    if (std::is_same<VT, float2>::value && basis_mode() == BASIS_FP32)
        hipLaunchKernelGGL(k_bdots_mf, grid, dim3(256), 0, s, d, N, nchunks, L, part);
    else if (direct)
        hipLaunchKernelGGL(k_bdots_bd<VT>, grid, dim3(256), 0, s, d, N, nchunks, L, part, bdots_xcd());
    else hipLaunchKernelGGL(k_bdots_bf<VT>, grid, dim3(256), 0, s, d, N, nchunks, L, part);
    hipLaunchKernelGGL(k_bdots_fin, dim3(unsigned(ni), unsigned((128 * BMAX) / 64)), dim3(256), 0, s, d, nchunks, 128,
                       (const double2 *)part);
    BIE_HIP(hipGetLastError());
}

template <typename VT>
void launch_comb_mf(const CItem *d, size_t ni, int64_t N, hipStream_t s)
{
    if (ni == 0) return;
    const dim3 grid{ unsigned((N + 127) / 128), unsigned(ni) };
    if (std::is_same<VT, float2>::value && basis_mode() == BASIS_FP32)
        hipLaunchKernelGGL(k_bcomb_mf, grid, dim3(256), 0, s, d, N);
    else if (basis_mode() == BASIS_DIRECT) hipLaunchKernelGGL(k_bcomb_bd<VT>, grid, dim3(256), 0, s, d, N);
    else hipLaunchKernelGGL(k_bcomb_bf<VT>, grid, dim3(256), 0, s, d, N);
    BIE_HIP(hipGetLastError());
}

// basis dots and updates: matrix cores (BF16 splits) for the complex64 and the
// FP16-pair bases, FP64 vector ALUs for the FP64 basis
template <typename VT>
void basis_dots(const DItem *d, size_t ni, int64_t N, double2 *part, int nbmax, hipStream_t s)
{
    if constexpr (std::is_same<VT, double2>::value) launch_dots<VT>(d, ni, N, part, nbmax, s);
    else launch_dots_mf<VT>(d, ni, N, part, s);
}
template <typename VT>
void basis_comb(const CItem *d, size_t ni, int64_t N, int nbmax, hipStream_t s)
{
    if constexpr (std::is_same<VT, double2>::value) launch_comb<VT, double2>(d, ni, N, nbmax, s);
    else launch_comb_mf<VT>(d, ni, N, s);
}

// Rank-revealing orthonormalisation of the unit-scaled residual block from its
// Gram matrix G (q x q, row-major): pivoted Cholesky P^T Gs P = L L^H stopped at
// pivots <= delta^2.  Returns r; T0 (q x r) maps the unscaled residual columns
// to V_0, S (r x q) gives the scaled residuals as V_0 S.
int rank_revealing(const std::vector<cd> &G, int q, const std::vector<double> &scale, std::vector<cd> &T0,
                   std::vector<cd> &S)
{
    std::vector<cd> A(size_t(q) * q), L(size_t(q) * q, cd(0.0));
    for (int a = 0; a < q; ++a)
        for (int b = 0; b < q; ++b) A[a * q + b] = G[a * q + b] / (scale[a] * scale[b]);
    std::vector<int> perm(q);
    for (int i = 0; i < q; ++i) perm[i] = i;
    int r = 0;
    for (int k = 0; k < q; ++k) {
        int p = k;
        for (int i = k + 1; i < q; ++i)
            if (A[i * q + i].real() > A[p * q + p].real()) p = i;
        if (!(A[p * q + p].real() > DELTA * DELTA)) break;
        if (p != k) {
            for (int i = 0; i < q; ++i) std::swap(A[k * q + i], A[p * q + i]);
            for (int i = 0; i < q; ++i) std::swap(A[i * q + k], A[i * q + p]);
            for (int i = 0; i < k; ++i) std::swap(L[k * q + i], L[p * q + i]);
            std::swap(perm[k], perm[p]);
        }
        const double d = std::sqrt(A[k * q + k].real());
        L[k * q + k] = d;
        for (int i = k + 1; i < q; ++i) L[i * q + k] = A[i * q + k] / d;
        for (int i = k + 1; i < q; ++i)
            for (int l = k + 1; l < q; ++l) A[i * q + l] -= L[i * q + k] * std::conj(L[l * q + k]);
        r = k + 1;
    }
    // Li = L11^{-1} (lower), V_0 = R0s(:, perm[0..r)) Li^H
    std::vector<cd> Li(size_t(r) * r, cd(0.0));
    for (int c = 0; c < r; ++c) {
        Li[c * r + c] = 1.0 / L[c * q + c];
        for (int i = c + 1; i < r; ++i) {
            cd s = 0.0;
            for (int l = c; l < i; ++l) s += L[i * q + l] * Li[l * r + c];
            Li[i * r + c] = -s / L[i * q + i];
        }
    }
    T0.assign(size_t(q) * r, cd(0.0));
    for (int i = 0; i < r; ++i)
        for (int c = 0; c < r; ++c) T0[perm[i] * r + c] = std::conj(Li[c * r + i]) / scale[perm[i]];
    S.assign(size_t(r) * q, cd(0.0));
    for (int i = 0; i < q; ++i)
        for (int a = 0; a < std::min(r, i + 1); ++a) S[a * q + perm[i]] = std::conj(L[i * q + a]);
    return r;
}

// Second and third streams (least-squares updates; end-of-cycle solutions),
// events and pinned buffers of one solve, released at scope exit.
struct Aux {
    hipStream_t s2 = nullptr, s3 = nullptr;
    hipEvent_t ev[7] = {};
    Aux()
    {
        BIE_HIP(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
        BIE_HIP(hipStreamCreateWithFlags(&s3, hipStreamNonBlocking));
        for (auto &e : ev) BIE_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    ~Aux()
    {
        if (s2) (void)hipStreamSynchronize(s2);
        if (s3) (void)hipStreamSynchronize(s3);
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
        if (s2) (void)hipStreamDestroy(s2);
        if (s3) (void)hipStreamDestroy(s3);
    }
};

// Device and pinned buffers, table arenas and side streams of the block solver,
// kept by the operator between calls: a solve takes its buffers in a fixed order
// and reuses the one in the same place when it is large enough (else it is
// replaced).  A solve returns with its streams synchronised, so the next may reuse
// everything; after a solve that ended in an error the device is synchronised
// first.  Solves on one operator from several threads at once are not supported.
struct BlockCache {
    std::vector<std::pair<void *, size_t>> dev, pin;
    size_t nd = 0, np = 0;
    std::unique_ptr<Arena> ar[3];
    std::unique_ptr<Aux> aux;
    bool dirty = false;
    void begin()
    {
        if (dirty) (void)hipDeviceSynchronize();
        dirty = true;
        nd = np = 0;
        for (auto &a : ar) {
            if (!a) a = std::make_unique<Arena>(size_t(8) << 20);
            a->reset();
        }
        if (!aux) aux = std::make_unique<Aux>();
    }
    template <typename T>
    T *get(size_t n)
    {
        const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
        if (nd == dev.size()) dev.emplace_back(nullptr, 0);
        auto &slot = dev[nd++];
        if (slot.second < bytes) {
            if (slot.first) (void)hipFree(slot.first);
            slot = { nullptr, 0 };
            BIE_HIP(hipMalloc(&slot.first, bytes));
            slot.second = bytes;
        }
        return static_cast<T *>(slot.first);
    }
    template <typename T>
    T *pinned(size_t n)
    {
        const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
        if (np == pin.size()) pin.emplace_back(nullptr, 0);
        auto &slot = pin[np++];
        if (slot.second < bytes) {
            if (slot.first) (void)hipHostFree(slot.first);
            slot = { nullptr, 0 };
            BIE_HIP(hipHostMalloc(&slot.first, bytes));
            slot.second = bytes;
        }
        return static_cast<T *>(slot.first);
    }
    ~BlockCache()
    {
        aux.reset();
        for (auto &d : dev)
            if (d.first) (void)hipFree(d.first);
        for (auto &h : pin)
            if (h.first) (void)hipHostFree(h.first);
    }
};

// element type of a basis block as the right-hand block of a split-BF16 product
template <typename VT>
constexpr int vec_type()
{
    return std::is_same<VT, c32h>::value ? VEC_F16 : std::is_same<VT, float2>::value ? VEC_C64 : VEC_C128;
}

template <typename VT>
int solve_chunk(bie_op *op, const double2 *B, double2 *X, int64_t R, const bie_solve_opts &o, bie_solve_stat *hs,
                hipStream_t s)
{
    const int64_t N = op->mesh.N;
    const int m = o.restart;
    const int p = o.block > 0 ? o.block : 32;
    const bool mixed = o.precision == 1;
    const int terms = o.inner_terms ? o.inner_terms : 3;
    const double itol = std::max(o.inner_tol > 0.0 ? o.inner_tol : 1e-3, terms == 2 ? 1e-2 : 0.0);
    const int64_t Gmax = (R + p - 1) / p;
    // second Gram-Schmidt pass when a column keeps less than half its norm
    // squared; none with the complex64 basis of the refinement's inner solves,
    // whose storage already bounds orthogonality near 1e-7 against their
    // tolerance of 1e-3 .. 1e-1
    const double reorth = mixed ? 0.0 : 0.5;
    // Calderon preconditioner on the right: each step forms T (M V_j); a cycle's
    // solution U of T M U = residual gathers in Ux and X += M U ends the cycle
    const bie_calderon *pcd = o.calderon;
    bie_op *pview = pcd ? calderon_view(pcd, mixed, s) : nullptr;
    bie_op *ptm = pcd && mixed ? calderon_tm(pcd, s) : nullptr;   // T M as one split-BF16 operand

    if (!op->bcache) op->bcache = new BlockCache();
    BlockCache &db = *static_cast<BlockCache *>(op->bcache);
    db.begin();
    double2 *Rres = db.get<double2>(size_t(R) * N);
    double2 *Wb = db.get<double2>(size_t(R) * N);
    double2 *Wt = pcd && !mixed ? db.get<double2>(size_t(R) * N) : nullptr;   // M V_j (FP64 form)
    double2 *Ux = pcd ? db.get<double2>(size_t(R) * N) : nullptr;
    double2 *Du = pcd ? db.get<double2>(size_t(R) * N) : nullptr;   // M U
    VT *V = db.get<VT>(size_t(m + 1) * R * N);
    const int64_t tiles = ((m + 1) * p + DT - 1) / DT + 1;   // basis tiles per group, and its Gram item
    int64_t slack = 1024;   // workgroups of a basis-dots launch beyond one per item
    if constexpr (!std::is_same<VT, double2>::value) slack = std::max<int64_t>(slack, 2 * bdots_slots<VT>());
    double2 *part = db.get<double2>(size_t(Gmax * tiles + slack) * DT * BMAX);
    const int nparts = int(std::min<int64_t>(64, (N + 255) / 256));
    double *npart = db.get<double>(size_t(R) * nparts);
    double *nrm = db.get<double>(size_t(R));
    // group regions
    const size_t p2 = size_t(p) * p;
    const size_t per = (m + 1) * p2 + 2 * p2 + size_t(m) * (m + 1) * p2 + 4 * size_t(m) * p2 + size_t(m) * p2 + p2 +
                       (m + 1) * p2 + size_t(m) * p2;
    double2 *greg = db.get<double2>(per * Gmax);
    double *gest = db.get<double>(size_t(Gmax) * BMAX);
    double *gscale = db.get<double>(size_t(Gmax) * BMAX);
    int *gflag = db.get<int>(size_t(Gmax) * 4);
    GDev *gd = db.get<GDev>(size_t(Gmax));
    std::vector<GDev> hg(Gmax);
    for (int64_t g = 0; g < Gmax; ++g) {
        double2 *b = greg + per * g;
        GDev &d = hg[g];
        d.C2 = b; b += (m + 1) * p2;
        d.G1 = b; b += p2;
        d.G2 = b; b += p2;
        d.Rt = b; b += size_t(m) * (m + 1) * p2;
        d.U = b; b += 2 * size_t(m) * p2;
        d.T = b; b += size_t(m) * p2;
        d.Mw = b; b += 2 * size_t(m) * p2;
        d.Tinv = b; b += p2;
        d.Gv = b; b += (m + 1) * p2;
        d.Y = b;
        d.est = gest + g * BMAX;
        d.scale = gscale + g * BMAX;
        d.flag = gflag + 4 * g;
    }
    Arena &ar = *db.ar[0];
    Arena *arena[2] = { db.ar[1].get(), db.ar[2].get() };
    Aux &aux = *db.aux;
    hipStream_t s2 = aux.s2, s3 = aux.s3;
    hipEvent_t ev_prod = aux.ev[0], ev_ls[2] = { aux.ev[1], aux.ev[2] }, ev_arena[2] = { aux.ev[3], aux.ev[4] };
    hipEvent_t ev_s3[2] = { aux.ev[5], aux.ev[6] };
    BIE_HIP(hipEventRecord(ev_arena[0], s));
    BIE_HIP(hipEventRecord(ev_arena[1], s));
    BIE_HIP(hipEventRecord(ev_s3[0], s3));
    BIE_HIP(hipEventRecord(ev_s3[1], s3));
    double *hest[2];
    int *hfl[2];
    for (int i = 0; i < 2; ++i) {
        hest[i] = db.pinned<double>(size_t(Gmax) * BMAX);
        hfl[i] = db.pinned<int>(size_t(Gmax) * 4);
    }
    int *gsteps = db.get<int>(size_t(Gmax));
    double2 *gG = db.get<double2>(size_t(Gmax) * p2);   // Gram matrices of the start blocks, gathered
    double2 *hGpin = db.pinned<double2>(size_t(Gmax) * p2);
    std::vector<int> hsteps(Gmax, 0);
    auto sync = [&]() {
        BIE_HIP(hipStreamSynchronize(s));
        ar.reset();
    };
    auto norms = [&](const double2 *src, const std::vector<int> &cols, std::vector<double> &out) {
        const int *dc = ar.put(cols);
        ar.flush(s);
        hipLaunchKernelGGL(k_bnorm_part, dim3(unsigned(nparts), unsigned(cols.size())), dim3(256), 0, s, N, src, dc,
                           npart);
        hipLaunchKernelGGL(k_bnorm_fin, dim3(unsigned((cols.size() + 63) / 64)), dim3(64), 0, s, nparts,
                           int(cols.size()), (const double *)npart, nrm);
        BIE_HIP(hipGetLastError());
        out.resize(cols.size());
        BIE_HIP(hipMemcpyAsync(out.data(), nrm, cols.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        sync();
    };

    std::vector<int> all(R);
    for (int64_t i = 0; i < R; ++i) all[i] = int(i);
    std::vector<double> bn;
    norms(B, all, bn);
    for (int64_t i = 0; i < R; ++i) hs[i] = bie_solve_stat{ 0, 0, NAN, NAN, 0, 0, o.use_x0 ? 1 : 0 };
    if (!o.use_x0) BIE_HIP(hipMemsetAsync(X, 0, size_t(R) * N * sizeof(double2), s));
    std::vector<int> live;
    for (int64_t i = 0; i < R; ++i) {
        if (bn[i] == 0.0) {
            BIE_HIP(hipMemsetAsync(X + i * N, 0, N * sizeof(double2), s));
            hs[i].converged = 1;
            hs[i].relres_est = hs[i].relres_true = 0.0;
        } else {
            live.push_back(int(i));
        }
    }
    bool first = true;
    std::vector<double> rn;
    std::vector<HGroup> grp;
    while (!live.empty()) {
        // (1) FP64 residuals and the standard criterion.  In refinement a residual
        // far from convergence only starts the next correction: every residual is
        // taken with the 3-term split-BF16 product (relative error near 1e-5), and
        // every right-hand side it puts within that product's reach of convergence
        // (at or below max(tol, 1e-3)) is taken again in FP64, which decides
        const bool guess_low = mixed && !(first && !o.use_x0);
        if (first && !o.use_x0) {
            BIE_HIP(hipMemcpyAsync(Rres, B, size_t(R) * N * sizeof(double2), hipMemcpyDeviceToDevice, s));
        } else {
            const int *dl = ar.put(live);
            ar.flush(s);
            if (guess_low) gemm_product(op, X, N, VEC_C128, Rres, N, B, N, int64_t(live.size()), dl, s, 3);
            else gemm64_product(op, X, N, Rres, N, B, N, int64_t(live.size()), dl, s);
        }
        norms(Rres, live, rn);
        if (guess_low) {
            std::vector<int> conf;
            for (size_t a = 0; a < live.size(); ++a)
                if (rn[a] <= std::max(o.tol, 1e-3) * bn[live[a]]) conf.push_back(live[a]);
            if (!conf.empty()) {
                const int *dc = ar.put(conf);
                ar.flush(s);
                gemm64_product(op, X, N, Rres, N, B, N, int64_t(conf.size()), dc, s);
                norms(Rres, live, rn);
            }
        }
        std::vector<int> keep;
        std::vector<double> krn;
        for (size_t a = 0; a < live.size(); ++a) {
            const int i = live[a];
            bie_solve_stat &st = hs[i];
            if (!(first && !o.use_x0)) st.mvps += 1;
            st.checks += 1;
            double rel = rn[a] / bn[i];
            if (first && o.use_x0 == 2 && !(rel < 1.0)) {   // a guess no better than zero is replaced by zero
                st.x0_kept = 0;
                BIE_HIP(hipMemsetAsync(X + int64_t(i) * N, 0, N * sizeof(double2), s));
                BIE_HIP(hipMemcpyAsync(Rres + int64_t(i) * N, B + int64_t(i) * N, N * sizeof(double2),
                                       hipMemcpyDeviceToDevice, s));
                rn[a] = bn[i];
                rel = 1.0;
            }
            st.relres_true = rel;
            if (rel <= o.tol) st.converged = 1;
            else if (st.mvps < o.max_mvp) {
                keep.push_back(i);
                krn.push_back(rn[a]);
            }
        }
        first = false;
        live = keep;
        if (live.empty()) break;
        // (2) groups of consecutive live right-hand sides; their residuals
        // gathered into Wb, Gram matrices, rank-revealing start blocks
        grp.clear();
        for (size_t g0 = 0; g0 < live.size(); g0 += p) {
            HGroup h;
            h.q = int(std::min<size_t>(p, live.size() - g0));
            h.qoff = int(g0);
            h.rhs.assign(live.begin() + g0, live.begin() + g0 + h.q);
            grp.push_back(h);
        }
        const int ng = int(grp.size());
        {
            const int *dl = ar.put(live);
            std::vector<DItem> it;
            for (int g = 0; g < ng; ++g) {
                const HGroup &h = grp[g];
                it.push_back(DItem{ Wb + int64_t(h.qoff) * N, 0, Wb + int64_t(h.qoff) * N, hg[g].G1, nullptr, h.q, 0,
                                    h.q, h.q, h.q, 0 });
            }
            const DItem *di = ar.put(it);
            ar.flush(s);
            hipLaunchKernelGGL(k_bgather, dim3(unsigned(std::min<int64_t>((N + 255) / 256, 64)), unsigned(live.size())),
                               dim3(256), 0, s, N, (const double2 *)Rres, dl, Wb);
            launch_dots<double2, 1>(di, it.size(), N, part, p, s);
        }
        // the Gram matrices of all groups gathered on the device, then one copy to pinned memory
        {
            std::vector<SItem> gi;
            for (int g = 0; g < ng; ++g) {
                const int64_t n = 2 * int64_t(grp[g].q) * grp[g].q;
                gi.push_back(SItem{ reinterpret_cast<const double *>(hg[g].G1),
                                    reinterpret_cast<double *>(gG + size_t(g) * p2), n, n });
            }
            const SItem *dgi = ar.put(gi);
            ar.flush(s);
            hipLaunchKernelGGL(k_bscatter, dim3(unsigned(ng)), dim3(256), 0, s, dgi);
            BIE_HIP(hipGetLastError());
            BIE_HIP(hipMemcpyAsync(hGpin, gG, size_t(ng) * p2 * sizeof(double2), hipMemcpyDeviceToHost, s));
        }
        sync();
        std::vector<std::vector<cd>> hG(ng);
        for (int g = 0; g < ng; ++g) {
            const cd *src = reinterpret_cast<const cd *>(hGpin) + size_t(g) * p2;
            hG[g].assign(src, src + size_t(grp[g].q) * grp[g].q);
        }
        int Wc = 0;
        std::vector<std::vector<cd>> T0(ng), S(ng);
        for (int g = 0; g < ng; ++g) {
            HGroup &h = grp[g];
            h.scale.resize(h.q);
            for (int a = 0; a < h.q; ++a) h.scale[a] = std::sqrt(std::max(hG[g][a * h.q + a].real(), 0.0));
            h.r = rank_revealing(hG[g], h.q, h.scale, T0[g], S[g]);
            if (h.r < 1) throw Error(BIE_ENUMERIC, "block GMRES: start block of rank 0 for unconverged right-hand sides");
            h.c0 = Wc;
            Wc += h.r;
            h.target.resize(h.q);
            int64_t used = 0;
            for (int a = 0; a < h.q; ++a) {
                h.target[a] = mixed ? itol : o.tol * bn[h.rhs[a]] / h.scale[a];
                used = std::max<int64_t>(used, hs[h.rhs[a]].mvps);
            }
            h.cap = int(std::min<int64_t>(m, std::max<int64_t>(1, o.max_mvp - used)));
            h.steps = 0;
            h.active = true;
            hg[g].r = h.r;
            hg[g].q = h.q;
        }
        ar.copy_to(gd, hg.data(), size_t(ng), s);
        {
            std::vector<CItem> it;
            std::vector<SItem> up;
            for (int g = 0; g < ng; ++g) {
                const HGroup &h = grp[g];
                std::vector<double2> t0(T0[g].size());
                for (size_t e = 0; e < t0.size(); ++e) t0[e] = make_double2(T0[g][e].real(), T0[g][e].imag());
                const double2 *dT = ar.put(t0);
                it.push_back(CItem{ Wb + int64_t(h.qoff) * N, 0, dT, V + int64_t(h.c0) * N, nullptr, nullptr, 1.0, 0.0,
                                    h.q, h.q, h.r, h.r });
                // E_1 S into Gv (rows 0 .. r), zeros below; column scales
                std::vector<double2> sv(S[g].size());
                for (size_t e = 0; e < sv.size(); ++e) sv[e] = make_double2(S[g][e].real(), S[g][e].imag());
                const double2 *dS = ar.put(sv);
                const double *dsc = ar.put(h.scale);
                up.push_back(SItem{ reinterpret_cast<const double *>(dS), reinterpret_cast<double *>(hg[g].Gv),
                                    2 * int64_t(sv.size()), 2 * int64_t(m + 1) * h.r * h.q });
                up.push_back(SItem{ dsc, hg[g].scale, int64_t(h.q), int64_t(h.q) });
            }
            const CItem *ci = ar.put(it);
            const SItem *dup = ar.put(up);
            ar.flush(s);
            hipLaunchKernelGGL(k_bscatter, dim3(unsigned(up.size())), dim3(256), 0, s, dup);
            BIE_HIP(hipGetLastError());
            if constexpr (std::is_same<VT, double2>::value) launch_comb<double2, VT>(ci, it.size(), N, p, s);
            else launch_comb64<VT>(ci, it.size(), N, p, s, false);   // K = q <= 32
        }
        if (pcd) zero_into(R * N, Ux, s);
        // (3) block Arnoldi steps; every active group advances together.  The
        // least-squares update of step j runs on the second stream beside the
        // orthogonalisation of step j + 1; its estimates are read one step late,
        // so a group that has met its targets runs at most one step more
        // (discarded: its solution uses the steps up to the decision).
        int prev = -1;
        std::vector<int> prev_act;
        for (int j = 0; j <= m; ++j) {
            std::vector<int> act, cols;
            if (j < m)
                for (int g = 0; g < ng; ++g)
                    if (grp[g].active && j < grp[g].cap) {
                        act.push_back(g);
                        for (int a = 0; a < grp[g].r; ++a) cols.push_back(grp[g].c0 + a);
                    }
            if (act.empty() && prev < 0) break;
            Arena &A = *arena[j & 1];
            BIE_HIP(hipEventSynchronize(ev_arena[j & 1]));
            BIE_HIP(hipEventSynchronize(ev_s3[j & 1]));
            A.reset();
            // least-squares update of step prev on the second stream, queued after
            // this step's product so that it shares the GPU with the smaller
            // kernels of the step instead of with the product's workgroups
            bool ls_queued = false;
            auto launch_ls = [&]() {
                if (prev < 0 || ls_queued) return;
                ls_queued = true;
                std::vector<int> lsg;
                for (int g : prev_act)
                    if (grp[g].active) lsg.push_back(g);
                if (!lsg.empty()) {
                    const int *dls = A.put(lsg);
                    A.flush(s);
                    BIE_HIP(hipEventRecord(ev_prod, s));
                    BIE_HIP(hipStreamWaitEvent(s2, ev_prod, 0));
                    hipLaunchKernelGGL(k_bls_apply, dim3(unsigned(lsg.size()), unsigned((p + CS - 1) / CS)), dim3(256), 0,
                                       s2, gd, dls, prev, m);
                    hipLaunchKernelGGL(k_bls_qr, dim3(unsigned(lsg.size())), dim3(256), 0, s2, gd, dls, prev, m);
                    BIE_HIP(hipGetLastError());
                }
                BIE_HIP(hipMemcpyAsync(hest[prev & 1], gest, size_t(ng) * BMAX * sizeof(double), hipMemcpyDeviceToHost,
                                       s2));
                BIE_HIP(hipMemcpyAsync(hfl[prev & 1], gflag, size_t(ng) * 4 * sizeof(int), hipMemcpyDeviceToHost, s2));
                BIE_HIP(hipEventRecord(ev_ls[prev & 1], s2));
            };
            if (!act.empty()) {
                const int na = int(act.size());
                // tables of the step: pass 1 basis dots, Gram before and after,
                // updates; pass 2 the same for flagged groups; basis scaling
                std::vector<DItem> dv[2], dpre, dpost[2];
                std::vector<CItem> ci[2], cs;
                for (int g : act) {
                    const HGroup &h = grp[g];
                    const int K = (j + 1) * h.r;
                    double2 *Wg = Wb + int64_t(h.c0) * N;
                    for (int pass = 0; pass < 2; ++pass) {
                        const int *fl = pass ? hg[g].flag : nullptr;
                        // first-pass coefficients straight into column block j of Hbar
                        double2 *Cd = pass ? hg[g].C2 : hg[g].Rt + int64_t(j) * (m + 1) * h.r * h.r;
                        for (int k0 = 0; k0 < K; k0 += DT)
                            dv[pass].push_back(DItem{ V + int64_t(h.c0) * N, Wc, Wg, Cd, fl, h.r, k0, std::min(DT, K - k0),
                                                      h.r, h.r, 0 });
                        dpost[pass].push_back(DItem{ Wg, 0, Wg, hg[g].G2, fl, h.r, 0, h.r, h.r, h.r, 0 });
                        ci[pass].push_back(CItem{ V + int64_t(h.c0) * N, Wc, Cd, Wg, nullptr, fl, -1.0, 1.0, h.r, K, h.r,
                                                  h.r });
                    }
                    dpre.push_back(DItem{ Wg, 0, Wg, hg[g].G1, nullptr, h.r, 0, h.r, h.r, h.r, 0 });
                    cs.push_back(CItem{ Wg, 0, hg[g].Tinv, V + (int64_t(j + 1) * Wc + h.c0) * N, nullptr, nullptr, 1.0,
                                        0.0, h.r, h.r, h.r, h.r });
                }
                const int *dg = A.put(act), *dc = A.put(cols);
                const DItem *pv0 = A.put(dv[0]), *pv1 = A.put(dv[1]), *ppre = A.put(dpre), *pp0 = A.put(dpost[0]),
                            *pp1 = A.put(dpost[1]);
                const CItem *pc0 = A.put(ci[0]), *pc1 = A.put(ci[1]), *pcs = A.put(cs);
                A.flush(s);
                const VT *Vj = V + int64_t(j) * Wc * N;
                const int64_t nc = int64_t(cols.size());
                if (pcd && mixed) {
                    gemm_product(ptm, Vj, N, vec_type<VT>(), Wb, N, nullptr, 0, nc, dc, s, terms);
                } else if (pcd) {
                    gemm64_product(pview, Vj, N, Wt, N, nullptr, 0, nc, dc, s);
                    gemm64_product(op, Wt, N, Wb, N, nullptr, 0, nc, dc, s);
                } else if (mixed) {
                    gemm_product(op, Vj, N, vec_type<VT>(), Wb, N, nullptr, 0, nc, dc, s, terms);
                } else {
                    gemm64_product(op, Vj, N, Wb, N, nullptr, 0, nc, dc, s);
                }
                launch_ls();
                // Gram matrices of W: FP64 matrix cores in the mixed forms
                auto gram = [&](const DItem *gi, size_t n) {
                    if constexpr (std::is_same<VT, double2>::value) launch_dots<double2, 1>(gi, n, N, part, p, s);
                    else launch_gram64(gi, n, N, part, p, s);
                };
                int64_t pairs = 0, vecs = 0;   // basis vector x column pairs, basis vectors of the first pass
                for (int g : act) {
                    pairs += int64_t(j + 1) * grp[g].r * grp[g].r;
                    vecs += int64_t(j + 1) * grp[g].r;
                }
                prof_begin(4, s, pairs);
                basis_dots<VT>(pv0, dv[0].size(), N, part, p, s);
                prof_end(4, s);
                if (reorth > 0.0) gram(ppre, dpre.size());   // G1 for the second-pass test
                prof_begin(5, s, vecs);
                basis_comb<VT>(pc0, ci[0].size(), N, p, s);
                prof_end(5, s);
                gram(pp0, dpost[0].size());
                hipLaunchKernelGGL(k_bflag, dim3(unsigned(na)), dim3(64), 0, s, gd, dg, reorth);
                if (reorth > 0.0) {
                    basis_dots<VT>(pv1, dv[1].size(), N, part, p, s);
                    basis_comb<VT>(pc1, ci[1].size(), N, p, s);
                    gram(pp1, dpost[1].size());
                }
                hipLaunchKernelGGL(k_bchol, dim3(unsigned(na)), dim3(256), 0, s, gd, dg, j, m, DELTA);
                if constexpr (std::is_same<VT, double2>::value) launch_comb<double2, VT>(pcs, cs.size(), N, p, s);
                else launch_comb64<VT>(pcs, cs.size(), N, p, s, true);   // K = r <= 32, R^{-1} upper triangular
            }
            launch_ls();   // no step j: the update of step prev right away
            if (prev >= 0) {
                BIE_HIP(hipEventSynchronize(ev_ls[prev & 1]));
                const double *est = hest[prev & 1];
                const int *fl = hfl[prev & 1];
                std::vector<int> ended;
                for (int g : prev_act) {
                    HGroup &h = grp[g];
                    if (!h.active) continue;
                    h.steps = prev + 1;
                    bool met = true;
                    for (int a = 0; a < h.q; ++a) {
                        const double e = est[size_t(g) * BMAX + a];
                        bie_solve_stat &st = hs[h.rhs[a]];
                        st.iters += 1;
                        st.mvps += 1;
                        st.relres_est = e * h.scale[a] / bn[h.rhs[a]];
                        if (!(e <= h.target[a])) met = false;
                    }
                    if (met || fl[4 * g + 2 + (prev & 1)] || h.steps >= h.cap) {
                        h.active = false;
                        hsteps[g] = h.steps;
                        ended.push_back(g);
                    }
                }
                if (!ended.empty()) {
                    // Y = R^{-1} (E_1 S) and X += V Y for the groups that ended at step prev,
                    // on the third stream beside the next steps (after their tables and the
                    // least-squares update of step prev)
                    std::vector<CItem> it;
                    std::vector<const int *> oc;
                    const int *de = A.put(ended);
                    for (int g : ended) oc.push_back(A.put(grp[g].rhs));
                    for (size_t e = 0; e < ended.size(); ++e) {
                        const HGroup &h = grp[ended[e]];
                        it.push_back(CItem{ V + int64_t(h.c0) * N, Wc, hg[ended[e]].Y, pcd ? Ux : X, oc[e], nullptr, 1.0,
                                            1.0, h.r, h.steps * h.r, h.q, h.q });
                    }
                    const CItem *pit = A.put(it);
                    A.copy_to(gsteps, hsteps.data(), size_t(ng), s3);   // also uploads the tables above
                    BIE_HIP(hipStreamWaitEvent(s3, ev_ls[prev & 1], 0));
                    int jmax = 0;
                    for (int g : ended) jmax = std::max(jmax, grp[g].steps);
                    for (int I = jmax - 1; I >= 0; --I)
                        hipLaunchKernelGGL(k_bls_back, dim3(unsigned(ended.size()), unsigned(I + 1)), dim3(256), 0, s3,
                                           gd, de, gsteps, I, m);
                    BIE_HIP(hipGetLastError());
                    basis_comb<VT>(pit, it.size(), N, p, s3);
                }
                BIE_HIP(hipEventRecord(ev_s3[j & 1], s3));
            }
            BIE_HIP(hipEventRecord(ev_arena[j & 1], s));
            prev = act.empty() ? -1 : j;
            prev_act = act;
        }
        BIE_HIP(hipStreamSynchronize(s2));
        BIE_HIP(hipStreamSynchronize(s3));
        if (pcd) {   // X += M U (zero for the columns outside this cycle), on the matrix cores: split-BF16
                     // with 3 terms in the refinement (its 1e-5 error is far below the inner tolerance), else FP64
            if (mixed) gemm_product(pview, Ux, N, VEC_C128, Du, N, nullptr, 0, R, nullptr, s, 3);
            else gemm64_product(pview, Ux, N, Du, N, nullptr, 0, R, nullptr, s);
            add_into(R * N, Du, X, s);
        }
    }
    sync();
    BIE_HIP(hipStreamSynchronize(s2));
    BIE_HIP(hipStreamSynchronize(s3));
    db.dirty = false;
    int status = BIE_OK;
    for (int64_t i = 0; i < R; ++i)
        if (!hs[i].converged) status = BIE_NOT_CONVERGED;
    return status;
}

}  // namespace

void free_block_cache(bie_op *op)
{
    delete static_cast<BlockCache *>(op->bcache);
    op->bcache = nullptr;
}

// Block GMRES for R right-hand sides, in consecutive chunks of `slots` (all R
// when 0), each chunk solved to the end before the next.
int solve_block(const bie_op *opc, const void *Bv, void *Xv, int64_t R, const bie_solve_opts &o,
                bie_solve_stat *stats, hipStream_t s)
{
    bie_op *op = const_cast<bie_op *>(opc);
    const int64_t N = op->mesh.N;
    const int64_t W = o.slots > 0 ? std::min<int64_t>(o.slots, R) : R;
    const double2 *B = static_cast<const double2 *>(Bv);
    double2 *X = static_cast<double2 *>(Xv);
    std::vector<bie_solve_stat> hs(R);
    int status = BIE_OK;
    for (int64_t c0 = 0; c0 < R; c0 += W) {
        const int64_t n = std::min(W, R - c0);
        const int rc = o.precision != 1 ? solve_chunk<double2>(op, B + c0 * N, X + c0 * N, n, o, hs.data() + c0, s)
                       : o.basis == 1   ? solve_chunk<c32h>(op, B + c0 * N, X + c0 * N, n, o, hs.data() + c0, s)
                                        : solve_chunk<float2>(op, B + c0 * N, X + c0 * N, n, o, hs.data() + c0, s);
        if (rc != BIE_OK) status = rc;
    }
    if (stats)
        for (int64_t i = 0; i < R; ++i) stats[i] = hs[i];
    return status;
}

}  // namespace bie
