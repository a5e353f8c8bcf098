// Krylov solvers on the device: restarted GMRES(m) and CGNR, with the
// standard and random-sampling convergence criteria.
//
// The paper solves eq:discretizedEFIE "using an iterative solver" (Sec. II)
// and names GMRES, CG and the two criteria only in its acronym list; the
// readings implemented:
//   GMRES(m): Arnoldi with classical Gram-Schmidt and selective
//     reorthogonalisation (DGKS), complex Givens rotations kept in FP64 on the
//     device, tolerance relative
//     to ||b||; a cycle ends when |g_{j+1}|/||b|| <= tol, on breakdown, or at
//     j = m; the criterion is then evaluated on the true residual, and the
//     method restarts from the true residual if it fails.
//   CGNR: CG on T^H T x = T^H b (CGLS recurrences), stopping on the recursive
//     ||r||/||b|| confirmed by the criterion on the true residual.
//   SCC:  ||b - T x|| / ||b|| <= tol.
//   RSCC: sqrt((N/S) sum_{i in S} |b_i - (T x)_i|^2) / ||b|| <= tol.
//
// R right-hand sides advance together: one product kernel per iteration
// serves all active columns, each column keeps its own Krylov basis,
// Hessenberg matrix and Givens rotations.  Every kernel of a GMRES cycle is
// enqueued without host synchronisation; columns whose cycle has ended are
// skipped on the device.  The host reads a 96-byte status record per column
// once per cycle.
//
// Reductions are deterministic: every block writes partial sums, the last
// block to finish (agent-scope fence + counter) adds them in block order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "bie_internal.hpp"

// No automatic fusion of multiplies and adds in this file: the rounding of
// every result follows the source expression, so kernels instantiated with
// different element counts per thread, or different column counts, give
// bitwise identical columns.  Fused multiply-adds are written out as fma().
#pragma clang fp contract(off)

namespace bie {


namespace {

constexpr int BT = 256;          // threads per block
constexpr int EPT = 4;           // elements per thread in vector kernels
constexpr int BE = BT * EPT;     // elements per block
constexpr int MAXM = 64;         // largest restart length

struct ColStat {
    double bnorm;    // ||b||
    double est;      // recursive residual estimate / ||b||
    double wnorm0;   // ||w|| before orthogonalisation (breakdown test)
    double hn;       // h_{j+1,j}
    double rnorm;    // ||b - T x|| (full residual)
    double rsum;     // sampled squared residual sum (RSCC)
    double cg_zz;    // CGNR: ||z||^2
    double cg_a;     // CGNR: alpha or beta
    int done;        // cycle ended (GMRES) / iteration stopped (CGNR)
    int jend;        // iterations in the current cycle
    int jcap;        // iteration cap for the current cycle
    int brk;         // breakdown
    int active;      // column still solving
    int check;       // CGNR: recursive estimate met the tolerance
    int reorth;      // GMRES: second Gram-Schmidt pass taken in this iteration
    int pad;
};
static_assert(sizeof(ColStat) == 96, "ColStat layout");

// Where the vectors of column r live.  One problem (uniform): length N, basis
// at r (m+1) N, vectors at r N, chunk partials at r nc(N).  Several problems
// of different sizes (batched solves): per-column tables of length and
// offsets, so that one launch serves columns of every problem.
struct Cols {
    const int64_t *n = nullptr;      // length of column r (null: N)
    const int64_t *voff = nullptr;   // offset of its Krylov basis (elements)
    const int64_t *woff = nullptr;   // offset of its vectors (W, residual, solution)
    const int64_t *poff = nullptr;   // offset of its chunk partial sums
    int64_t N = 0;
    int m = 0;
    __device__ int64_t len(int r) const { return n ? n[r] : N; }
    __device__ int64_t vo(int r) const { return voff ? voff[r] : int64_t(r) * (m + 1) * N; }
    __device__ int64_t wo(int r) const { return woff ? woff[r] : int64_t(r) * N; }
    __device__ int64_t po(int r) const;
};

__device__ inline double2 cmul(double2 a, double2 b)
{
    return make_double2(fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x));
}
__device__ inline double2 cmulc(double2 a, double2 b)   // conj(a) * b
{
    return make_double2(fma(a.x, b.x, a.y * b.y), fma(a.x, b.y, -(a.y * b.x)));
}

// Basis vectors are stored as complex128 or complex64 (VT); arithmetic is FP64.
__device__ inline double2 ld2(const double2 &v) { return v; }
__device__ inline double2 ld2(const float2 &v) { return make_double2(double(v.x), double(v.y)); }
__device__ inline double2 ld2(const c32h &v) { return make_double2(double(v.x), double(v.y)); }
template <typename VT> __device__ inline VT st2(double2 v);
template <> __device__ inline double2 st2<double2>(double2 v) { return v; }
template <> __device__ inline float2 st2<float2>(double2 v) { return make_float2(float(v.x), float(v.y)); }
template <> __device__ inline c32h st2<c32h>(double2 v) { return c32h{ (_Float16)v.x, (_Float16)v.y }; }

__device__ inline double wsum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sums 8 complex values p[0..7] over the 64 lanes of a wave at once.  Each
// exchange step halves the number of values a lane carries (it keeps one half,
// sends the other to its partner), so 8 sums cost 4+2+1+3 exchanges instead of
// 8x6.  On return p[0] of lane L holds the total of value (L >> 3) & 7.
__device__ inline void wave_sum8(double2 p[8])
{
    const int lane = threadIdx.x & 63;
    {
        const bool b = lane & 32;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double2 snd = b ? p[i] : p[i + 4];
            const double2 kp = b ? p[i + 4] : p[i];
            p[i] = make_double2(kp.x + __shfl_xor(snd.x, 32, 64), kp.y + __shfl_xor(snd.y, 32, 64));
        }
    }
    {
        const bool b = lane & 16;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const double2 snd = b ? p[i] : p[i + 2];
            const double2 kp = b ? p[i + 2] : p[i];
            p[i] = make_double2(kp.x + __shfl_xor(snd.x, 16, 64), kp.y + __shfl_xor(snd.y, 16, 64));
        }
    }
    {
        const bool b = lane & 8;
        const double2 snd = b ? p[0] : p[1];
        const double2 kp = b ? p[1] : p[0];
        p[0] = make_double2(kp.x + __shfl_xor(snd.x, 8, 64), kp.y + __shfl_xor(snd.y, 8, 64));
    }
#pragma unroll
    for (int o = 4; o > 0; o >>= 1) {
        p[0].x += __shfl_xor(p[0].x, o, 64);
        p[0].y += __shfl_xor(p[0].y, o, 64);
    }
}

// Chunk partials of conj(V[k][e]) * w[e] for k = 0..nk-1: element q of this
// thread belongs to chunk q of the block; written to red[q][k][wave].  Wave
// sums use wave_sum8 over groups of 8 k.
template <typename VT, int EPT>
__device__ inline void block_dots(const VT *__restrict__ V, int64_t N, const int64_t *e, const double2 *w, int nk,
                                  double2 (*red)[MAXM + 1][4])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < EPT; ++q)
        for (int k0 = 0; k0 < nk; k0 += 8) {
            double2 p[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int k = k0 + i;
                p[i] = make_double2(0.0, 0.0);
                if (e[q] < N && k < nk) p[i] = cmulc(ld2(V[int64_t(k) * N + e[q]]), w[q]);
            }
            wave_sum8(p);
            const int kk = k0 + ((lane >> 3) & 7);
            if ((lane & 7) == 0 && kk < nk) red[q][kk][wave] = p[0];
        }
}

// Last-block election: returns true in every thread of the block that
// finished last; resets the counter for the next launch.
__device__ inline bool last_block(unsigned *counter, unsigned nblk)
{
    __shared__ int is_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned prev = atomicAdd(counter, 1u);
        is_last = (prev == nblk - 1);
        if (is_last) atomicExch(counter, 0u);
    }
    __syncthreads();
    if (is_last) __threadfence();
    return is_last != 0;
}

// Wave-per-k dot products of the chunk held in LDS against V rows 0..nk-1:
// part[k] = sum_e conj(V[k][e]) w[e].
__device__ inline void chunk_dots(const double2 *__restrict__ V, int64_t N, int64_t e0, int nk,
                                  const double2 *sw, double2 *__restrict__ part)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = wave; k < nk; k += BT / 64) {
        double ar = 0.0, ai = 0.0;
        for (int t = lane; t < BE; t += 64) {
            const int64_t e = e0 + t;
            if (e < N) {
                const double2 v = V[int64_t(k) * N + e];
                const double2 p = cmulc(v, sw[t]);
                ar += p.x;
                ai += p.y;
            }
        }
        ar = wsum(ar);
        ai = wsum(ai);
        if (lane == 0) part[k] = make_double2(ar, ai);
    }
}

// ---------------------------------------------------------------------------
// Arnoldi step j: classical Gram-Schmidt with selective reorthogonalisation
// (Daniel, Gragg, Kaufman & Stewart, Math. Comp. 30, 1976): after the first
// pass w' = w - V h1, a second pass is made only if ||w'||^2 < ||w||^2 / 2,
// judged from ||w||^2 - ||h1||^2 (accurate whenever the test passes).  Every
// block evaluates the test from the same sums in the same order, so all blocks
// agree.  Partial sums are kept per chunk of AB consecutive elements and the
// next launch adds the partials of all chunks itself, in chunk order (no
// atomics).  A thread handles EPT elements, one in each of EPT chunks of its
// block; the chunk partials do not depend on EPT, so neither do the results.
//   pass1:  P1 = partial V_{0..j}^H w (2-D grid: 8 basis vectors per block
//           column), ||w||^2 partials
//   pass2:  h1 = sum P1; w' = w - V h1; PN = partial ||w'||^2; if the test
//           fails also P2 = partial V^H w'
//   pass3:  only after a failed test: h2 = sum P2; w'' = w' - V h2; PN again
//   finish: h_{j+1,j} = sqrt(sum PN); v_{j+1} = w / h_{j+1,j}; Givens update
//           and the cycle test (block 0).
constexpr int AB = 256;   // elements (threads) per block in the Arnoldi kernels
constexpr int KG = 8;     // basis vectors per block in the first pass

__device__ inline int64_t Cols::po(int r) const { return poff ? poff[r] : int64_t(r) * ((N + AB - 1) / AB); }

// element q of thread t in block b (coalesced): (b EPT + q) AB + t
template <int EPT>
__device__ inline int64_t elem(int q)
{
    return (int64_t(blockIdx.x) * EPT + q) * AB + threadIdx.x;
}

template <typename VT, int EPT>
__global__ __launch_bounds__(AB) void k_cgs_pass1(Cols cl, int m, int j, const VT *__restrict__ Vall,
                                                  const double2 *__restrict__ Wall, double2 *__restrict__ P1all,
                                                  double *__restrict__ PWall, const ColStat *__restrict__ st)
{
    const int r = blockIdx.z;
    if (st[r].done) return;
    const int k0 = blockIdx.y * KG;
    if (k0 > j) return;
    const int64_t N = cl.len(r);
    if (int64_t(blockIdx.x) * EPT * AB >= N) return;   // beyond this column
    const int nc = int((N + AB - 1) / AB);   // chunks of AB elements
    const VT *V = Vall + cl.vo(r);
    Wall += cl.wo(r);
    P1all += cl.po(r) * (m + 1);
    PWall += cl.po(r);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __shared__ double2 red[EPT][KG][AB / 64];
    __shared__ double rn[EPT][AB / 64];
    // all loads first (KG basis vectors x EPT elements), then one wave_sum8 per element
    double2 w[EPT], vv[EPT][KG];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        const int64_t e = elem<EPT>(q);
        w[q] = e < N ? Wall[e] : make_double2(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < KG; ++i)
            vv[q][i] = (e < N && k0 + i <= j) ? ld2(V[int64_t(k0 + i) * N + e]) : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        double2 p[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) p[i] = cmulc(vv[q][i], w[q]);
        wave_sum8(p);
        if ((lane & 7) == 0) red[q][lane >> 3][wave] = p[0];
        if (blockIdx.y == 0) {
            const double nn = wsum(w[q].x * w[q].x + w[q].y * w[q].y);
            if (lane == 0) rn[q][wave] = nn;
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        const int c = int(blockIdx.x) * EPT + q;
        if (c >= nc) break;
        double2 *P1 = P1all + int64_t(c) * (m + 1);
        if (threadIdx.x < KG && k0 + int(threadIdx.x) <= j) {
            double2 a = red[q][threadIdx.x][0];
            for (int u = 1; u < AB / 64; ++u) { a.x += red[q][threadIdx.x][u].x; a.y += red[q][threadIdx.x][u].y; }
            P1[k0 + threadIdx.x] = a;
        }
        if (blockIdx.y == 0 && threadIdx.x == 0) PWall[c] = rn[q][0] + rn[q][1] + rn[q][2] + rn[q][3];
    }
}

// First pass with every basis vector in one block (one element per thread):
// w is read once per chunk and the loads of NG groups of 8 basis vectors are in
// flight together.  Same sums in the same order as k_cgs_pass1 (bitwise equal).
template <typename VT, int NG>
__global__ __launch_bounds__(AB) void k_cgs_dots(Cols cl, int m, int j, const VT *__restrict__ Vall,
                                                 const double2 *__restrict__ Wall, double2 *__restrict__ P1all,
                                                 double *__restrict__ PWall, const ColStat *__restrict__ st)
{
    const int r = blockIdx.y;
    if (st[r].done) return;
    const int64_t N = cl.len(r);
    if (int64_t(blockIdx.x) * AB >= N) return;   // beyond this column
    const VT *V = Vall + cl.vo(r);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t e = int64_t(blockIdx.x) * AB + threadIdx.x;
    const double2 w = e < N ? Wall[cl.wo(r) + e] : make_double2(0.0, 0.0);
    __shared__ double2 red[MAXM + 8][AB / 64];
    __shared__ double rn[AB / 64];
    const double nn = wsum(w.x * w.x + w.y * w.y);
    if (lane == 0) rn[wave] = nn;
    for (int k0 = 0; k0 <= j; k0 += 8 * NG) {
        VT vv[NG][8];
#pragma unroll
        for (int g = 0; g < NG; ++g)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int k = k0 + 8 * g + i;
                vv[g][i] = (e < N && k <= j) ? V[int64_t(k) * N + e] : VT{};
            }
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            if (k0 + 8 * g > j) break;
            double2 p[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) p[i] = cmulc(ld2(vv[g][i]), w);
            wave_sum8(p);
            if ((lane & 7) == 0) red[k0 + 8 * g + (lane >> 3)][wave] = p[0];
        }
    }
    __syncthreads();
    double2 *P1 = P1all + (cl.po(r) + int64_t(blockIdx.x)) * (m + 1);
    for (int t = threadIdx.x; t <= j; t += AB) {
        double2 a = red[t][0];
        for (int u = 1; u < AB / 64; ++u) { a.x += red[t][u].x; a.y += red[t][u].y; }
        P1[t] = a;
    }
    if (threadIdx.x == 0) PWall[cl.po(r) + blockIdx.x] = rn[0] + rn[1] + rn[2] + rn[3];
}

// h[k] = sum over blocks of P[b][k], k <= kmax, into LDS (block order)
__device__ inline void sum_partials(const double2 *__restrict__ P, int nb, int stride, int kmax, double2 *h)
{
    for (int k = threadIdx.x; k <= kmax; k += AB) {
        double ar = 0.0, ai = 0.0;
#pragma unroll 8
        for (int b = 0; b < nb; ++b) {
            const double2 v = P[int64_t(b) * stride + k];
            ar += v.x;
            ai += v.y;
        }
        h[k] = make_double2(ar, ai);
    }
}

// sum over blocks of real partials, by wave 0 (lanes load in parallel, fixed tree)
__device__ inline double sum_real_partials(const double *__restrict__ P, int nb)
{
    double a = 0.0;
    for (int b = threadIdx.x & 63; b < nb; b += 64) a += P[b];
    return wsum(a);
}

// w[q] -= V_{0..j} h for the EPT elements e[q] of this thread (h in LDS).
// Loads are batched over 8 / EPT basis vectors and all EPT elements; every
// element subtracts its terms in ascending k whatever EPT is.
template <typename VT, int EPT>
__device__ inline void cgs_update(const VT *__restrict__ V, int64_t N, const int64_t *e, int j, double2 *w,
                                  const double2 *h)
{
    constexpr int KB = 8 / EPT;
    for (int k0 = 0; k0 <= j; k0 += KB) {
        double2 vv[KB][EPT];
#pragma unroll
        for (int i = 0; i < KB; ++i)
#pragma unroll
            for (int q = 0; q < EPT; ++q)
                vv[i][q] = (k0 + i <= j && e[q] < N) ? ld2(V[int64_t(k0 + i) * N + e[q]]) : make_double2(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < KB; ++i) {
            if (k0 + i > j) break;
#pragma unroll
            for (int q = 0; q < EPT; ++q) {
                const double2 p = cmul(vv[i][q], h[k0 + i]);
                w[q].x -= p.x;
                w[q].y -= p.y;
            }
        }
    }
}

template <typename VT, int EPT>
__global__ __launch_bounds__(AB) void k_cgs_pass2(Cols cl, int m, int j, const VT *__restrict__ Vall,
                                                  double2 *__restrict__ Wall, const double2 *__restrict__ P1all,
                                                  const double *__restrict__ PWall, double2 *__restrict__ P2all,
                                                  double *__restrict__ PNall, double2 *__restrict__ Hall,
                                                  ColStat *__restrict__ st)
{
    const int r = blockIdx.y;
    if (st[r].done) return;
    const int64_t N = cl.len(r);
    if (int64_t(blockIdx.x) * EPT * AB >= N) return;   // beyond this column
    const int nc = int((N + AB - 1) / AB);
    Wall += cl.wo(r);
    P1all += cl.po(r) * (m + 1);
    P2all += cl.po(r) * (m + 1);
    PWall += cl.po(r);
    PNall += cl.po(r);
    __shared__ double2 h[MAXM + 1];
    __shared__ int s_reorth;
    __shared__ double s_w2;
    sum_partials(P1all, nc, m + 1, j, h);
    if (threadIdx.x < 64) {
        const double w2 = sum_real_partials(PWall, nc);
        if (threadIdx.x == 0) s_w2 = w2;
    }
    __syncthreads();
    // DGKS test from ||w||^2 and ||h1||^2 (same sums, same order in every block)
    if (threadIdx.x == 0) {
        double h2 = 0.0;
        for (int k = 0; k <= j; ++k) h2 += h[k].x * h[k].x + h[k].y * h[k].y;
        s_reorth = (s_w2 - h2) < 0.5 * s_w2;
    }
    __syncthreads();
    const bool reorth = s_reorth != 0;
    if (blockIdx.x == 0) {
        for (int k = threadIdx.x; k <= j; k += AB) Hall[(int64_t(r) * m + j) * (m + 1) + k] = h[k];
        if (threadIdx.x == 0) st[r].reorth = reorth;
    }
    const VT *V = Vall + cl.vo(r);
    int64_t e[EPT];
    double2 w[EPT];
    __shared__ double rn[EPT][AB / 64];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        e[q] = elem<EPT>(q);
        w[q] = e[q] < N ? Wall[e[q]] : make_double2(0.0, 0.0);
    }
    cgs_update<VT, EPT>(V, N, e, j, w, h);
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        if (e[q] < N) Wall[e[q]] = w[q];
        const double nn = wsum(w[q].x * w[q].x + w[q].y * w[q].y);
        if ((threadIdx.x & 63) == 0) rn[q][threadIdx.x >> 6] = nn;
    }
    if (reorth) {
        __shared__ double2 red[EPT][MAXM + 1][AB / 64];
        block_dots<VT, EPT>(V, N, e, w, j + 1, red);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int c = int(blockIdx.x) * EPT + q;
            if (c >= nc) break;
            double2 *P2 = P2all + int64_t(c) * (m + 1);
            for (int k = threadIdx.x; k <= j; k += AB) {
                double2 a = red[q][k][0];
                for (int u = 1; u < AB / 64; ++u) { a.x += red[q][k][u].x; a.y += red[q][k][u].y; }
                P2[k] = a;
            }
        }
    } else {
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int c = int(blockIdx.x) * EPT + q;
            if (c < nc) PNall[c] = rn[q][0] + rn[q][1] + rn[q][2] + rn[q][3];
        }
}

template <typename VT, int EPT>
__global__ __launch_bounds__(AB) void k_cgs_pass3(Cols cl, int m, int j, const VT *__restrict__ Vall,
                                                  double2 *__restrict__ Wall, const double2 *__restrict__ P2all,
                                                  double *__restrict__ PNall, double2 *__restrict__ Hall,
                                                  const ColStat *__restrict__ st)
{
    const int r = blockIdx.y;
    if (st[r].done || !st[r].reorth) return;
    const int64_t N = cl.len(r);
    if (int64_t(blockIdx.x) * EPT * AB >= N) return;   // beyond this column
    const int nc = int((N + AB - 1) / AB);
    Wall += cl.wo(r);
    P2all += cl.po(r) * (m + 1);
    PNall += cl.po(r);
    __shared__ double2 h[MAXM + 1];
    sum_partials(P2all, nc, m + 1, j, h);
    __syncthreads();
    if (blockIdx.x == 0)
        for (int k = threadIdx.x; k <= j; k += AB) {
            double2 *hc = Hall + (int64_t(r) * m + j) * (m + 1) + k;
            const double2 a = *hc;
            *hc = make_double2(a.x + h[k].x, a.y + h[k].y);
        }
    const VT *V = Vall + cl.vo(r);
    __shared__ double red[EPT][AB / 64];
    int64_t e[EPT];
    double2 w[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        e[q] = elem<EPT>(q);
        w[q] = e[q] < N ? Wall[e[q]] : make_double2(0.0, 0.0);
    }
    cgs_update<VT, EPT>(V, N, e, j, w, h);
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        double nn = 0.0;
        if (e[q] < N) {
            Wall[e[q]] = w[q];
            nn = w[q].x * w[q].x + w[q].y * w[q].y;
        }
        nn = wsum(nn);
        if ((threadIdx.x & 63) == 0) red[q][threadIdx.x >> 6] = nn;
    }
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int c = int(blockIdx.x) * EPT + q;
            if (c < nc) PNall[c] = red[q][0] + red[q][1] + red[q][2] + red[q][3];
        }
}

// Givens rotation [c s; -conj(s) c], c real, mapping (a, b) to (rho, 0).
__device__ inline void givens(double2 a, double2 b, double &c, double2 &s)
{
    const double aa = hypot(a.x, a.y), bb = hypot(b.x, b.y);
    if (bb == 0.0) { c = 1.0; s = make_double2(0.0, 0.0); return; }
    if (aa == 0.0) { c = 0.0; s = make_double2(1.0, 0.0); return; }
    const double t = hypot(aa, bb);
    c = aa / t;
    const double2 ph = make_double2(a.x / aa, a.y / aa);
    s = make_double2((ph.x * b.x + ph.y * b.y) / t, (ph.y * b.x - ph.x * b.y) / t);   // (a/|a|) conj(b) / t
}

template <typename VT, int EPT>
__global__ __launch_bounds__(AB) void k_cgs_finish(Cols cl, int m, int j, double tol, VT *__restrict__ Vall,
                                                   const double2 *__restrict__ Wall, const double *__restrict__ PNall,
                                                   const double *__restrict__ PWall, double2 *__restrict__ Hall,
                                                   double *__restrict__ csall, double2 *__restrict__ snall,
                                                   double2 *__restrict__ gall, ColStat *__restrict__ st)
{
    const int r = blockIdx.y;
    if (st[r].done) return;
    const int64_t N = cl.len(r);
    if (int64_t(blockIdx.x) * EPT * AB >= N) return;   // beyond this column (block 0 never is)
    const int nc = int((N + AB - 1) / AB);
    Wall += cl.wo(r);
    PNall += cl.po(r);
    PWall += cl.po(r);
    __shared__ double s_hn, s_w2;
    __shared__ double2 Hc[MAXM + 2], sn[MAXM];
    __shared__ double cs[MAXM];
    if (threadIdx.x < 64) {
        const double a = sum_real_partials(PNall, nc);
        const double b = sum_real_partials(PWall, nc);
        if (threadIdx.x == 0) { s_hn = sqrt(a); s_w2 = b; }
    }
    if (blockIdx.x == 0) {
        for (int k = threadIdx.x; k <= j; k += AB) Hc[k] = Hall[(int64_t(r) * m + j) * (m + 1) + k];
        for (int k = threadIdx.x; k < j; k += AB) {
            cs[k] = csall[int64_t(r) * m + k];
            sn[k] = snall[int64_t(r) * m + k];
        }
    }
    __syncthreads();
    const double hn = s_hn;
    if (hn > 0.0) {
        const double inv = 1.0 / hn;
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int64_t e = elem<EPT>(q);
            if (e < N) {
                const double2 w = Wall[e];
                Vall[cl.vo(r) + int64_t(j + 1) * N + e] = st2<VT>(make_double2(w.x * inv, w.y * inv));
            }
        }
    }
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    ColStat &S = st[r];
    S.hn = hn;
    S.wnorm0 = sqrt(s_w2);
    Hc[j + 1] = make_double2(hn, 0.0);
    for (int i = 0; i < j; ++i) {
        const double2 a = Hc[i], b = Hc[i + 1];
        const double2 sb = cmul(sn[i], b);
        const double2 csa = cmul(make_double2(sn[i].x, -sn[i].y), a);
        Hc[i] = make_double2(cs[i] * a.x + sb.x, cs[i] * a.y + sb.y);
        Hc[i + 1] = make_double2(-csa.x + cs[i] * b.x, -csa.y + cs[i] * b.y);
    }
    double c;
    double2 s;
    givens(Hc[j], Hc[j + 1], c, s);
    const double2 sb = cmul(s, Hc[j + 1]);
    Hc[j] = make_double2(c * Hc[j].x + sb.x, c * Hc[j].y + sb.y);
    Hc[j + 1] = make_double2(0.0, 0.0);
    double2 *H = Hall + (int64_t(r) * m + j) * (m + 1);
    for (int i = 0; i <= j + 1; ++i) H[i] = Hc[i];
    csall[int64_t(r) * m + j] = c;
    snall[int64_t(r) * m + j] = s;
    double2 *g = gall + int64_t(r) * (m + 1);
    const double2 gj = g[j];
    const double2 t = cmul(make_double2(s.x, -s.y), gj);
    g[j + 1] = make_double2(-t.x, -t.y);
    g[j] = make_double2(c * gj.x, c * gj.y);
    S.est = hypot(t.x, t.y) / S.bnorm;
    const bool brk = hn <= 64.0 * 2.220446049250313e-16 * S.wnorm0;
    S.jend = j + 1;
    if (brk) S.brk = 1;
    if (S.est <= tol || brk || j + 1 >= S.jcap) S.done = 1;
}

// Upper-triangular solve H y = g for the iterations of the cycle: one block
// per column, H and g staged in LDS, column-oriented back substitution.
__global__ __launch_bounds__(64) void k_lsq(int m, const double2 *__restrict__ Hall, const double2 *__restrict__ gall,
                                            double2 *__restrict__ yall, const ColStat *__restrict__ st)
{
    const int r = blockIdx.x;
    if (!st[r].active) return;
    const int je = st[r].jend;
    extern __shared__ double2 Hs[];          // Hs[k*m + i] = H(i, k), upper part, m*m entries
    __shared__ double2 g[MAXM + 1];
    for (int idx = threadIdx.x; idx < je * je; idx += 64) {
        const int k = idx / je, i = idx % je;
        if (i <= k) Hs[k * m + i] = Hall[(int64_t(r) * m + k) * (m + 1) + i];
    }
    for (int i = threadIdx.x; i < je; i += 64) g[i] = gall[int64_t(r) * (m + 1) + i];
    __syncthreads();
    for (int i = je - 1; i >= 0; --i) {
        __shared__ double2 yi;
        if (threadIdx.x == 0) {
            const double2 d = Hs[i * m + i], a = g[i];
            const double dd = d.x * d.x + d.y * d.y;
            yi = make_double2((a.x * d.x + a.y * d.y) / dd, (a.y * d.x - a.x * d.y) / dd);
            yall[int64_t(r) * m + i] = yi;
        }
        __syncthreads();
        for (int q = threadIdx.x; q < i; q += 64) {
            const double2 p = cmul(Hs[i * m + q], yi);
            g[q].x -= p.x;
            g[q].y -= p.y;
        }
        __syncthreads();
    }
}

// x += V_{0..jend-1} y
template <typename VT>
__global__ __launch_bounds__(BT) void k_xupd(Cols cl, int m, const VT *__restrict__ Vall,
                                             const double2 *__restrict__ yall, double2 *__restrict__ X,
                                             const ColStat *__restrict__ st)
{
    const int r = blockIdx.y;
    if (!st[r].active) return;
    const int64_t N = cl.len(r);
    X += cl.wo(r);
    const int je = st[r].jend;
    __shared__ double2 sy[MAXM];
    if (threadIdx.x < je) sy[threadIdx.x] = yall[int64_t(r) * m + threadIdx.x];
    __syncthreads();
    const VT *V = Vall + cl.vo(r);
    for (int64_t e = int64_t(blockIdx.x) * BT + threadIdx.x; e < N; e += int64_t(gridDim.x) * BT) {
        double2 x = X[e];
        for (int k = 0; k < je; ++k) {
            const double2 p = cmul(ld2(V[int64_t(k) * N + e]), sy[k]);
            x.x += p.x;
            x.y += p.y;
        }
        X[e] = x;
    }
}

// X += Z for the active columns (the preconditioned update x += M (V y)).
__global__ __launch_bounds__(BT) void k_add_active(Cols cl, const double2 *__restrict__ Z, double2 *__restrict__ X,
                                                   const ColStat *__restrict__ st)
{
    const int r = blockIdx.y;
    if (!st[r].active) return;
    const int64_t N = cl.len(r), o = cl.wo(r);
    for (int64_t e = int64_t(blockIdx.x) * BT + threadIdx.x; e < N; e += int64_t(gridDim.x) * BT) {
        const double2 z = Z[o + e];
        double2 x = X[o + e];
        x.x += z.x;
        x.y += z.y;
        X[o + e] = x;
    }
}

// ||v||^2 per column with last-block finish; writes sqrt into the field at `off`.
__global__ __launch_bounds__(BT) void k_norm(Cols cl, const double2 *__restrict__ Vb, double *__restrict__ part,
                                             unsigned *__restrict__ counters, ColStat *__restrict__ st, int field,
                                             const int *__restrict__ mask)
{
    const int r = blockIdx.y;
    if (mask && !mask[r]) return;
    const unsigned nblk = gridDim.x;
    const int64_t N = cl.len(r);
    const double2 *v = Vb + cl.wo(r);
    double nn = 0.0;
    for (int t = threadIdx.x; t < BE; t += BT) {
        const int64_t e = int64_t(blockIdx.x) * BE + t;
        if (e < N) nn += v[e].x * v[e].x + v[e].y * v[e].y;
    }
    __shared__ double red[BT / 64];
    nn = wsum(nn);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nn;
    __syncthreads();
    if (threadIdx.x == 0) part[int64_t(r) * nblk + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    if (!last_block(counters + r, nblk)) return;
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (unsigned b = 0; b < nblk; ++b) s += part[int64_t(r) * nblk + b];
    double *f = reinterpret_cast<double *>(&st[r]);
    f[field] = sqrt(s);
}

// Start a cycle from the residual: v0 = res/||res||, g = (||res||, 0, ...).
template <typename VT>
__global__ __launch_bounds__(BT) void k_restart(Cols cl, int m, const double2 *__restrict__ Res,
                                                VT *__restrict__ Vall, double2 *__restrict__ gall,
                                                ColStat *__restrict__ st, const int *__restrict__ mask)
{
    const int r = blockIdx.y;
    if (!mask[r]) return;
    const double beta = st[r].rnorm;
    const double inv = 1.0 / beta;
    const int64_t N = cl.len(r);
    VT *v = Vall + cl.vo(r);
    Res += cl.wo(r);
    for (int64_t e = int64_t(blockIdx.x) * BT + threadIdx.x; e < N; e += int64_t(gridDim.x) * BT) {
        const double2 w = Res[e];
        v[e] = st2<VT>(make_double2(w.x * inv, w.y * inv));
    }
    if (blockIdx.x == 0 && threadIdx.x <= m)
        gall[int64_t(r) * (m + 1) + threadIdx.x] = make_double2(threadIdx.x == 0 ? beta : 0.0, 0.0);
}

// ----------------------------------------------------------------------------- CGNR
// alpha = zz / ||w||^2 (last block), then x += alpha p, r -= alpha w, est = ||r||/||b||.
__global__ __launch_bounds__(BT) void k_cg_alpha(int64_t N, const double2 *__restrict__ Wv, double *__restrict__ part,
                                                 unsigned *__restrict__ counters, ColStat *__restrict__ st)
{
    const int r = blockIdx.y;
    if (st[r].done) return;
    const unsigned nblk = gridDim.x;
    const double2 *w = Wv + int64_t(r) * N;
    double nn = 0.0;
    for (int t = threadIdx.x; t < BE; t += BT) {
        const int64_t e = int64_t(blockIdx.x) * BE + t;
        if (e < N) nn += w[e].x * w[e].x + w[e].y * w[e].y;
    }
    __shared__ double red[BT / 64];
    nn = wsum(nn);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nn;
    __syncthreads();
    if (threadIdx.x == 0) part[int64_t(r) * nblk + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    if (!last_block(counters + r, nblk)) return;
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (unsigned b = 0; b < nblk; ++b) s += part[int64_t(r) * nblk + b];
    st[r].cg_a = s > 0.0 ? st[r].cg_zz / s : 0.0;
    if (!(s > 0.0)) st[r].done = 1;
}

__global__ __launch_bounds__(BT) void k_cg_step(int64_t N, double tol, const double2 *__restrict__ P,
                                                const double2 *__restrict__ Wv, double2 *__restrict__ X,
                                                double2 *__restrict__ Rv, double *__restrict__ part,
                                                unsigned *__restrict__ counters, ColStat *__restrict__ st,
                                                int64_t *__restrict__ iters)
{
    const int r = blockIdx.y;
    if (st[r].done) return;
    const unsigned nblk = gridDim.x;
    const double a = st[r].cg_a;
    double nn = 0.0;
    for (int t = threadIdx.x; t < BE; t += BT) {
        const int64_t e = int64_t(blockIdx.x) * BE + t;
        if (e < N) {
            const int64_t o = int64_t(r) * N + e;
            const double2 p = P[o], w = Wv[o];
            double2 x = X[o], rr = Rv[o];
            x.x += a * p.x; x.y += a * p.y;
            rr.x -= a * w.x; rr.y -= a * w.y;
            X[o] = x;
            Rv[o] = rr;
            nn += rr.x * rr.x + rr.y * rr.y;
        }
    }
    __shared__ double red[BT / 64];
    nn = wsum(nn);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nn;
    __syncthreads();
    if (threadIdx.x == 0) part[int64_t(r) * nblk + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    if (!last_block(counters + r, nblk)) return;
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (unsigned b = 0; b < nblk; ++b) s += part[int64_t(r) * nblk + b];
    ColStat &S = st[r];
    S.est = sqrt(s) / S.bnorm;
    iters[r] += 1;
    if (S.est <= tol) { S.check = 1; S.done = 1; }
    if (iters[r] >= S.jcap) S.done = 1;
}

// beta = ||z_new||^2 / ||z||^2 (last block), stored in cg_a; zz updated.
// init: start of a (re)started recurrence, beta = 0.  A column is processed if
// mask[r] (when given) or else if it is not done.
__global__ __launch_bounds__(BT) void k_cg_beta(int64_t N, const double2 *__restrict__ Zv, double *__restrict__ part,
                                                unsigned *__restrict__ counters, ColStat *__restrict__ st, int init,
                                                const int *__restrict__ mask)
{
    const int r = blockIdx.y;
    if (mask ? !mask[r] : st[r].done) return;
    const unsigned nblk = gridDim.x;
    const double2 *z = Zv + int64_t(r) * N;
    double nn = 0.0;
    for (int t = threadIdx.x; t < BE; t += BT) {
        const int64_t e = int64_t(blockIdx.x) * BE + t;
        if (e < N) nn += z[e].x * z[e].x + z[e].y * z[e].y;
    }
    __shared__ double red[BT / 64];
    nn = wsum(nn);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nn;
    __syncthreads();
    if (threadIdx.x == 0) part[int64_t(r) * nblk + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    if (!last_block(counters + r, nblk)) return;
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (unsigned b = 0; b < nblk; ++b) s += part[int64_t(r) * nblk + b];
    ColStat &S = st[r];
    S.cg_a = init ? 0.0 : s / S.cg_zz;
    S.cg_zz = s;
}

// p = z + beta p, or p = z at the start of a recurrence (mask given).
__global__ __launch_bounds__(BT) void k_cg_dir(int64_t N, const double2 *__restrict__ Zv, double2 *__restrict__ P,
                                               const ColStat *__restrict__ st, const int *__restrict__ mask)
{
    const int r = blockIdx.y;
    if (mask ? !mask[r] : st[r].done) return;
    const double b = st[r].cg_a;
    for (int64_t e = int64_t(blockIdx.x) * BT + threadIdx.x; e < N; e += int64_t(gridDim.x) * BT) {
        const int64_t o = int64_t(r) * N + e;
        const double2 z = Zv[o];
        if (mask) {
            P[o] = z;
        } else {
            const double2 p = P[o];
            P[o] = make_double2(z.x + b * p.x, z.y + b * p.y);
        }
    }
}

__global__ void k_copy(int64_t n, const double2 *__restrict__ a, double2 *__restrict__ b)
{
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        b[i] = a[i];
}

__global__ void k_zero(int64_t n, double2 *__restrict__ a)
{
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        a[i] = make_double2(0.0, 0.0);
}

}  // namespace

// ----------------------------------------------------------------------------- host side

struct Workspace {
    int64_t N = 0, R = 0;
    int m = 0;
    unsigned nblk = 0;
    double2 *V = nullptr, *W = nullptr, *Res = nullptr, *H = nullptr, *sn = nullptr, *g = nullptr, *y = nullptr;
    double2 *h1 = nullptr, *h2 = nullptr, *part = nullptr, *P1 = nullptr, *P2 = nullptr;
    double *PN = nullptr, *PW = nullptr;
    double *cs = nullptr, *dpart = nullptr, *rs = nullptr;
    unsigned *counters = nullptr;
    ColStat *st = nullptr;
    int *mask = nullptr;
    int64_t *rows = nullptr, *iters = nullptr;
    std::vector<void *> all;

    template <typename T>
    T *alloc(size_t n)
    {
        void *p = nullptr;
        BIE_HIP(hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)));
        all.push_back(p);
        return static_cast<T *>(p);
    }
    ~Workspace()
    {
        for (void *p : all) (void)hipFree(p);
    }
};

// One Arnoldi step j for R columns after the product w = T v_j: CGS with
// selective reorthogonalisation, normalisation and the Givens update.  One
// element per thread: on 256 columns of 7680 unknowns this beat 2 and 4
// elements per thread (fewer loads in flight across the chip), although those
// add 2-4x fewer partial sums per block; the results are the same bitwise.
// Nmax: the longest column (grid size; shorter columns leave their extra
// blocks at once).
template <typename VT, int EPT>
static void arnoldi_launch(Workspace *w, const Cols &cl, int64_t Nmax, VT *V, int m, int j, double tol, int64_t R,
                           hipStream_t s)
{
    const unsigned nb = unsigned((Nmax + AB * EPT - 1) / (AB * EPT));
    const dim3 agrid(nb, unsigned(R));
    const dim3 pgrid(nb, unsigned((m + 1 + KG - 1) / KG), unsigned(R));
    // first pass: one block per chunk over all basis vectors for the complex64
    // basis (measured 3% faster per solve); the FP16 and complex128 bases keep
    // the 8-vector blocks (the wide form was 10% slower for FP16, equal for
    // complex128).  BIE_DOTS_WIDE = 0 / 1 forces either (measurement).
    static const int wide_env = [] {
        const char *e = getenv("BIE_DOTS_WIDE");
        return e ? atoi(e) : -1;
    }();
    const bool wide = wide_env < 0 ? sizeof(VT) == 8 : wide_env != 0;
    constexpr int NG = sizeof(VT) >= 16 ? 2 : 4;   // groups of 8 basis loads in flight together
    if (wide && EPT == 1)
        hipLaunchKernelGGL((k_cgs_dots<VT, NG>), agrid, dim3(AB), 0, s, cl, m, j, V, w->W, w->P1, w->PW, w->st);
    else
        hipLaunchKernelGGL((k_cgs_pass1<VT, EPT>), pgrid, dim3(AB), 0, s, cl, m, j, V, w->W, w->P1, w->PW, w->st);
    hipLaunchKernelGGL((k_cgs_pass2<VT, EPT>), agrid, dim3(AB), 0, s, cl, m, j, V, w->W, w->P1, w->PW, w->P2, w->PN,
                       w->H, w->st);
    hipLaunchKernelGGL((k_cgs_pass3<VT, EPT>), agrid, dim3(AB), 0, s, cl, m, j, V, w->W, w->P2, w->PN, w->H, w->st);
    hipLaunchKernelGGL((k_cgs_finish<VT, EPT>), agrid, dim3(AB), 0, s, cl, m, j, tol, V, w->W, w->PN, w->PW, w->H,
                       w->cs, w->sn, w->g, w->st);
    BIE_HIP(hipGetLastError());
}
template <typename VT>
static void arnoldi_step(Workspace *w, const Cols &cl, int64_t Nmax, VT *V, int m, int j, double tol, int64_t R,
                         hipStream_t s)
{
    arnoldi_launch<VT, 1>(w, cl, Nmax, V, m, j, tol, R, s);
}

static Cols uniform_cols(int64_t N, int m)
{
    Cols c;
    c.N = N;
    c.m = m;
    return c;
}

static constexpr int MAX_RSCC_ROWS = 4096;

static Workspace *get_ws(bie_op *op, int64_t R, int m)
{
    const int64_t N = op->mesh.N;
    Workspace *w = op->ws;
    if (w && w->R >= R && w->m >= m && w->N == N) return w;
    delete w;
    op->ws = nullptr;
    w = new Workspace();
    try {
        w->N = N;
        w->R = R;
        w->m = m;
        w->nblk = unsigned((N + BE - 1) / BE);
        w->V = w->alloc<double2>(size_t(R) * (m + 1) * N);
        w->W = w->alloc<double2>(size_t(R) * N);
        w->Res = w->alloc<double2>(size_t(R) * N);
        w->H = w->alloc<double2>(size_t(R) * m * (m + 1));
        w->sn = w->alloc<double2>(size_t(R) * m);
        w->cs = w->alloc<double>(size_t(R) * m);
        w->g = w->alloc<double2>(size_t(R) * (m + 1));
        w->y = w->alloc<double2>(size_t(R) * m);
        w->h1 = w->alloc<double2>(size_t(R) * (m + 1));
        w->h2 = w->alloc<double2>(size_t(R) * (m + 1));
        w->part = w->alloc<double2>(size_t(R) * w->nblk * (m + 2));
        const size_t ab = size_t((N + AB - 1) / AB);
        w->P1 = w->alloc<double2>(size_t(R) * ab * (m + 1));
        w->P2 = w->alloc<double2>(size_t(R) * ab * (m + 1));
        w->PN = w->alloc<double>(size_t(R) * ab);
        w->PW = w->alloc<double>(size_t(R) * ab);
        w->dpart = w->alloc<double>(size_t(R) * std::max<unsigned>(w->nblk, 1));
        w->rs = w->alloc<double>(size_t(R) * MAX_RSCC_ROWS);
        w->counters = w->alloc<unsigned>(size_t(R));
        BIE_HIP(hipMemset(w->counters, 0, size_t(R) * sizeof(unsigned)));
        w->st = w->alloc<ColStat>(size_t(R));
        w->mask = w->alloc<int>(size_t(R));
        w->rows = w->alloc<int64_t>(size_t(R) * MAX_RSCC_ROWS);
        w->iters = w->alloc<int64_t>(size_t(R));
    } catch (...) {
        delete w;
        throw;
    }
    op->ws = w;
    return w;
}

void free_workspace(bie_op *op)
{
    delete op->ws;
    op->ws = nullptr;
}

// Solve driver shared by GMRES and CGNR (FP64 vectors).  mat64 selects the
// matrix of the products.  inner: the solve is the inner step of iterative
// refinement, its cycles end on the recursive estimate alone (no criterion on
// the true residual of this system).
static int solve_impl(const bie_op *opc, const void *Bv, void *Xv, int64_t R, const bie_solve_opts &o,
                      bie_solve_stat *stats, hipStream_t s, int mat, bool inner)
{
    bie_op *op = const_cast<bie_op *>(opc);
    const int64_t N = op->mesh.N;
    const int fp64 = mat;   // matrix of the products (MAT64 / MAT32 / MATBF16)
    const int m = o.method == BIE_GMRES ? o.restart : 1;
    Workspace *w = get_ws(op, R, m);
    const Cols ucols = uniform_cols(N, m);
    // Calderon preconditioner (GMRES only): two R x N scratch blocks
    const bie_calderon *pcd = o.method == BIE_GMRES ? o.calderon : nullptr;
    double2 *pcw = pcd ? calderon_scratch(pcd, R, s) : nullptr;
    const double2 *B = static_cast<const double2 *>(Bv);
    double2 *X = static_cast<double2 *>(Xv);
    std::vector<bie_solve_stat> hs(R);
    for (auto &h : hs) h = bie_solve_stat{ 0, 0, NAN, NAN, 0, 0, o.use_x0 ? 1 : 0 };
    std::vector<int64_t> checks(R, 0);

    // per-column masks on the device are "skip" arrays for the product kernels
    std::vector<int> skip(R, 0), active(R, 1);
    std::vector<ColStat> st(R);
    auto push_st = [&]() { BIE_HIP(hipMemcpyAsync(w->st, st.data(), R * sizeof(ColStat), hipMemcpyHostToDevice, s)); };
    auto pull_st = [&]() {
        BIE_HIP(hipMemcpyAsync(st.data(), w->st, R * sizeof(ColStat), hipMemcpyDeviceToHost, s));
        BIE_HIP(hipStreamSynchronize(s));
    };
    int *dskip = w->mask;
    auto push_skip = [&](const std::vector<int> &v) {
        BIE_HIP(hipMemcpyAsync(dskip, v.data(), R * sizeof(int), hipMemcpyHostToDevice, s));
    };
    const dim3 vgrid(w->nblk, unsigned(R));
    const dim3 egrid(unsigned(std::min<int64_t>((N + BT - 1) / BT, 1024)), unsigned(R));
    const int field_rnorm = offsetof(ColStat, rnorm) / sizeof(double);
    const int *done_flags = &w->st[0].done;                       // device address, strided
    const int64_t done_stride = sizeof(ColStat) / sizeof(int);
    const int field_bnorm = offsetof(ColStat, bnorm) / sizeof(double);

    // ||b||
    for (int64_t r = 0; r < R; ++r) {
        st[r] = ColStat{};
        st[r].active = 1;
    }
    push_st();
    hipLaunchKernelGGL(k_norm, vgrid, dim3(BT), 0, s, ucols, B, w->dpart, w->counters, w->st, field_bnorm,
                       (const int *)nullptr);
    BIE_HIP(hipGetLastError());
    if (!o.use_x0) hipLaunchKernelGGL(k_zero, dim3(1024), dim3(256), 0, s, R * N, X);
    pull_st();
    for (int64_t r = 0; r < R; ++r) {
        if (st[r].bnorm == 0.0) {
            active[r] = 0;
            hs[r].converged = 1;
            hs[r].relres_est = hs[r].relres_true = 0.0;
        }
    }
    // zero-RHS columns: x = 0
    for (int64_t r = 0; r < R; ++r)
        if (!active[r]) hipLaunchKernelGGL(k_zero, dim3(64), dim3(256), 0, s, N, X + r * N);

    // residual r0 = b - T x0 (x0 = 0 gives b without a product)
    auto full_residual = [&](const std::vector<int> &need) {
        std::vector<int> sk(R);
        for (int64_t r = 0; r < R; ++r) sk[r] = need[r] ? 0 : 1;
        push_skip(sk);
        product(op, fp64, true, X, N, w->Res, N, B, N, R, dskip, 1, false, s);
        // k_norm mask: need
        push_skip(need);
        hipLaunchKernelGGL(k_norm, vgrid, dim3(BT), 0, s, ucols, w->Res, w->dpart, w->counters, w->st, field_rnorm,
                           (const int *)dskip);
        BIE_HIP(hipGetLastError());
        for (int64_t r = 0; r < R; ++r)
            if (need[r]) hs[r].mvps += 1;
    };
    // have_res[r]: the criterion left the full residual of the current x in Res
    std::vector<int> have_res(R, 0);
    auto criterion = [&](const std::vector<int> &cand, std::vector<int> &met) {
        // returns per-column criterion value in hs[r].relres_true; met[r] set
        std::vector<int> need(R, 0);
        bool any = false;
        for (int64_t r = 0; r < R; ++r) { met[r] = 0; have_res[r] = 0; if (cand[r]) { need[r] = 1; any = true; } }
        if (!any) return;
        if (inner) {   // estimate only
            for (int64_t r = 0; r < R; ++r)
                if (need[r]) {
                    met[r] = 1;
                    hs[r].relres_true = hs[r].relres_est;
                }
            return;
        }
        if (o.crit == BIE_SCC) {
            full_residual(need);
            pull_st();
            for (int64_t r = 0; r < R; ++r)
                if (need[r]) {
                    const double v = st[r].rnorm / st[r].bnorm;
                    hs[r].relres_true = v;
                    hs[r].checks += 1;
                    met[r] = v <= o.tol;
                    have_res[r] = 1;
                }
        } else {
            const int64_t S = std::min<int64_t>(std::min<int64_t>(o.rscc_rows, N), MAX_RSCC_ROWS);
            std::vector<int64_t> rows(R * S, 0);
            for (int64_t r = 0; r < R; ++r)
                if (need[r]) {
                    auto v = rscc_rows(N, S, o.rscc_seed + uint64_t(checks[r]));
                    std::copy(v.begin(), v.end(), rows.begin() + r * S);
                }
            BIE_HIP(hipMemcpyAsync(w->rows, rows.data(), rows.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
            push_skip(need);
            sampled_residual(op, B, X, R, S, w->rows, w->rs, dskip, s);
            BIE_HIP(hipGetLastError());
            std::vector<double> rs(R * S);
            BIE_HIP(hipMemcpyAsync(rs.data(), w->rs, rs.size() * sizeof(double), hipMemcpyDeviceToHost, s));
            pull_st();
            for (int64_t r = 0; r < R; ++r)
                if (need[r]) {
                    double sum = 0.0;
                    for (int64_t i = 0; i < S; ++i) sum += rs[r * S + i];
                    const double v = std::sqrt(double(N) / double(S) * sum) / st[r].bnorm;
                    hs[r].relres_true = v;
                    hs[r].checks += 1;
                    checks[r] += 1;
                    hs[r].mvps += (S + N - 1) / N;   // S/N of a product, rounded up
                    met[r] = v <= o.tol;
                }
            if (o.crit == BIE_CCC) {
                // combined: a sampled estimate at or below the tolerance is
                // confirmed by the standard criterion on the full residual
                std::vector<int> conf(R, 0);
                bool anyc = false;
                for (int64_t r = 0; r < R; ++r)
                    if (need[r] && met[r]) { conf[r] = 1; anyc = true; }
                if (anyc) {
                    full_residual(conf);
                    pull_st();
                    for (int64_t r = 0; r < R; ++r)
                        if (conf[r]) {
                            const double v = st[r].rnorm / st[r].bnorm;
                            hs[r].relres_true = v;
                            met[r] = v <= o.tol;
                            have_res[r] = 1;
                        }
                }
            }
        }
    };

    std::vector<int> need(R, 0), met(R, 0);
    if (o.use_x0) {
        for (int64_t r = 0; r < R; ++r) need[r] = active[r];
        full_residual(need);
        if (o.use_x0 == 2) {   // fallback: a guess no better than zero is replaced by zero
            pull_st();
            std::vector<int> back(R, 0);
            bool any = false;
            for (int64_t r = 0; r < R; ++r)
                if (active[r] && !(st[r].rnorm < st[r].bnorm)) {
                    back[r] = 1;
                    any = true;
                    hs[r].x0_kept = 0;
                    hipLaunchKernelGGL(k_zero, dim3(64), dim3(256), 0, s, N, X + r * N);
                    hipLaunchKernelGGL(k_copy, dim3(64), dim3(256), 0, s, N, B + r * N, w->Res + r * N);
                }
            if (any) {
                push_skip(back);
                hipLaunchKernelGGL(k_norm, vgrid, dim3(BT), 0, s, ucols, w->Res, w->dpart, w->counters, w->st,
                                   field_rnorm, (const int *)dskip);
            }
        }
    } else {
        for (int64_t r = 0; r < R; ++r)
            if (active[r])
                hipLaunchKernelGGL(k_copy, dim3(64), dim3(256), 0, s, N, B + r * N, w->Res + r * N);
        for (int64_t r = 0; r < R; ++r) need[r] = active[r];
        push_skip(need);
        hipLaunchKernelGGL(k_norm, vgrid, dim3(BT), 0, s, ucols, w->Res, w->dpart, w->counters, w->st, field_rnorm,
                           (const int *)dskip);
    }
    pull_st();

    if (o.method == BIE_GMRES) {
        // x0 already meets the tolerance?
        if (o.use_x0) {
            std::vector<int> cand(R, 0);
            for (int64_t r = 0; r < R; ++r)
                if (active[r] && st[r].rnorm / st[r].bnorm <= o.tol) cand[r] = 1;
            criterion(cand, met);
            for (int64_t r = 0; r < R; ++r)
                if (cand[r] && met[r]) { active[r] = 0; hs[r].converged = 1; hs[r].relres_est = st[r].rnorm / st[r].bnorm; }
        }
        while (true) {
            bool any = false;
            for (int64_t r = 0; r < R; ++r) {
                if (active[r] && hs[r].mvps >= o.max_mvp) active[r] = 0;
                any = any || active[r];
            }
            if (!any) break;
            // start a cycle for the active columns
            for (int64_t r = 0; r < R; ++r) {
                ColStat &c = st[r];
                c.done = active[r] ? 0 : 1;
                c.active = active[r];
                c.jend = 0;
                c.brk = 0;
                c.jcap = int(std::min<int64_t>(m, std::max<int64_t>(1, o.max_mvp - hs[r].mvps)));
                need[r] = active[r];
            }
            push_st();
            push_skip(need);
            hipLaunchKernelGGL(k_restart<double2>, egrid, dim3(BT), 0, s, ucols, m, w->Res, w->V, w->g, w->st, (const int *)dskip);
            BIE_HIP(hipGetLastError());
            int jmax = 0;
            for (int64_t r = 0; r < R; ++r)
                if (active[r]) jmax = std::max(jmax, st[r].jcap);
            for (int j = 0; j < jmax; ++j) {
                const double2 *vj = w->V + int64_t(j) * N;
                if (pcd) {   // right preconditioning: w = T (M v_j)
                    calderon_apply(pcd, vj, int64_t(m + 1) * N, pcw, N, R, done_flags, done_stride, s);
                    product(op, fp64, true, pcw, N, w->W, N, nullptr, 0, R, done_flags, done_stride, false, s);
                } else {
                    product(op, fp64, true, vj, int64_t(m + 1) * N, w->W, N, nullptr, 0, R, done_flags, done_stride,
                            false, s);
                }
                arnoldi_step<double2>(w, ucols, N, w->V, m, j, o.tol, R, s);
            }
            hipLaunchKernelGGL(k_lsq, dim3(unsigned(R)), dim3(64), size_t(m) * m * sizeof(double2), s, m, w->H, w->g,
                               w->y, w->st);
            if (pcd) {   // x += M (V y): V y formed in the scratch block, then one preconditioner product
                zero_into(R * N, pcw, s);
                hipLaunchKernelGGL(k_xupd<double2>, egrid, dim3(BT), 0, s, ucols, m, w->V, w->y, pcw, w->st);
                calderon_apply(pcd, pcw, N, pcw + R * N, N, R, nullptr, 1, s);
                add_into(R * N, pcw + R * N, X, s);
            } else {
                hipLaunchKernelGGL(k_xupd<double2>, egrid, dim3(BT), 0, s, ucols, m, w->V, w->y, X, w->st);
            }
            BIE_HIP(hipGetLastError());
            pull_st();
            std::vector<int> cand(R, 0);
            for (int64_t r = 0; r < R; ++r) {
                if (!active[r]) continue;
                hs[r].iters += st[r].jend;
                hs[r].mvps += st[r].jend;
                hs[r].relres_est = st[r].est;
                if (st[r].est <= o.tol || st[r].brk) cand[r] = 1;
            }
            criterion(cand, met);
            for (int64_t r = 0; r < R; ++r)
                if (cand[r] && met[r]) {
                    active[r] = 0;
                    hs[r].converged = 1;
                }
            // restart the others from the true residual (SCC already has it)
            std::vector<int> nd(R, 0);
            bool anyr = false;
            for (int64_t r = 0; r < R; ++r)
                if (active[r] && hs[r].mvps < o.max_mvp && !(!inner && cand[r] && have_res[r])) {
                    nd[r] = 1;
                    anyr = true;
                }
            if (anyr) full_residual(nd);
            pull_st();
            for (int64_t r = 0; r < R; ++r)
                if (active[r] && st[r].rnorm == 0.0) { active[r] = 0; hs[r].converged = 1; hs[r].relres_true = 0.0; }
        }
    } else {
        // CGNR on T^H T x = T^H b.  P: search directions, Zv: z = T^H r.
        double2 *Pv = w->V;
        double2 *Zv = w->V + R * N;      // V holds R (m+1) N >= 2 R N complex
        std::vector<int64_t> it_dev(R, 0);
        // (re)start the recurrence for masked columns from the residual in Res
        auto cg_restart = [&](const std::vector<int> &msk) {
            for (int64_t r = 0; r < R; ++r)
                if (msk[r]) {
                    st[r].done = 0;
                    st[r].check = 0;
                    st[r].jcap = int(std::min<int64_t>(int64_t(1) << 30,
                                                       std::max<int64_t>(1, (o.max_mvp - hs[r].mvps) / 2)));
                    it_dev[r] = 0;
                    hs[r].mvps += 1;
                }
            push_st();
            BIE_HIP(hipMemcpyAsync(w->iters, it_dev.data(), R * sizeof(int64_t), hipMemcpyHostToDevice, s));
            std::vector<int> sk(R);
            for (int64_t r = 0; r < R; ++r) sk[r] = msk[r] ? 0 : 1;
            push_skip(sk);
            product(op, fp64, true, w->Res, N, Zv, N, nullptr, 0, R, dskip, 1, true, s);
            push_skip(msk);
            hipLaunchKernelGGL(k_cg_beta, vgrid, dim3(BT), 0, s, N, Zv, w->dpart, w->counters, w->st, 1,
                               (const int *)dskip);
            hipLaunchKernelGGL(k_cg_dir, egrid, dim3(BT), 0, s, N, Zv, Pv, w->st, (const int *)dskip);
            BIE_HIP(hipGetLastError());
            pull_st();
        };
        for (int64_t r = 0; r < R; ++r) {
            st[r].done = 1;
            need[r] = active[r];
        }
        cg_restart(need);
        std::vector<int64_t> base_it(R, 0);
        const int chunk = 16;
        while (true) {
            bool any = false;
            for (int64_t r = 0; r < R; ++r) any = any || active[r];
            if (!any) break;
            for (int it = 0; it < chunk; ++it) {
                product(op, fp64, true, Pv, N, w->W, N, nullptr, 0, R, done_flags, done_stride, false, s);
                hipLaunchKernelGGL(k_cg_alpha, vgrid, dim3(BT), 0, s, N, w->W, w->dpart, w->counters, w->st);
                hipLaunchKernelGGL(k_cg_step, vgrid, dim3(BT), 0, s, N, o.tol, Pv, w->W, X, w->Res, w->dpart,
                                   w->counters, w->st, w->iters);
                product(op, fp64, true, w->Res, N, Zv, N, nullptr, 0, R, done_flags, done_stride, true, s);
                hipLaunchKernelGGL(k_cg_beta, vgrid, dim3(BT), 0, s, N, Zv, w->dpart, w->counters, w->st, 0,
                                   (const int *)nullptr);
                hipLaunchKernelGGL(k_cg_dir, egrid, dim3(BT), 0, s, N, Zv, Pv, w->st, (const int *)nullptr);
                BIE_HIP(hipGetLastError());
            }
            std::vector<int64_t> its(R);
            BIE_HIP(hipMemcpyAsync(its.data(), w->iters, R * sizeof(int64_t), hipMemcpyDeviceToHost, s));
            pull_st();
            std::vector<int> cand(R, 0);
            for (int64_t r = 0; r < R; ++r) {
                if (!active[r]) continue;
                const int64_t newit = its[r] - it_dev[r];
                it_dev[r] = its[r];
                hs[r].iters += newit;
                // two products per iteration; the T^H r of the stopping iteration is skipped
                hs[r].mvps += 2 * newit - (st[r].done && newit > 0 ? 1 : 0);
                hs[r].relres_est = st[r].est;
                if (st[r].check) cand[r] = 1;
                else if (st[r].done) active[r] = 0;      // iteration cap or breakdown
            }
            criterion(cand, met);
            std::vector<int> again(R, 0);
            bool anyr = false;
            for (int64_t r = 0; r < R; ++r) {
                if (!cand[r]) continue;
                if (met[r]) { active[r] = 0; hs[r].converged = 1; }
                else if (hs[r].mvps < o.max_mvp) { again[r] = 1; anyr = true; }
                else active[r] = 0;
            }
            if (anyr) {
                std::vector<int> fr(R, 0);
                bool anyf = false;
                for (int64_t r = 0; r < R; ++r)
                    if (again[r] && !have_res[r]) { fr[r] = 1; anyf = true; }
                if (anyf) full_residual(fr);
                pull_st();
                cg_restart(again);
            }
            for (int64_t r = 0; r < R; ++r) {
                if (active[r] && hs[r].mvps >= o.max_mvp) active[r] = 0;
                if (!active[r]) st[r].done = 1;
            }
            push_st();
        }
    }
    BIE_HIP(hipStreamSynchronize(s));
    int status = BIE_OK;
    for (int64_t r = 0; r < R; ++r) {
        if (!hs[r].converged) status = BIE_NOT_CONVERGED;
        if (stats) stats[r] = hs[r];
    }
    return status;
}


namespace {

__global__ void k_axpy_cols(int64_t n, const double2 *__restrict__ d, double2 *__restrict__ x)
{
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        const double2 a = d[i];
        double2 b = x[i];
        b.x += a.x;
        b.y += a.y;
        x[i] = b;
    }
}

// ||v_r|| for R vectors into out[r] (deterministic: per-block partials, one wave adds them)
__global__ __launch_bounds__(BT) void k_colnorm_part(int64_t N, const double2 *__restrict__ v, double *__restrict__ part)
{
    const int r = blockIdx.y;
    double nn = 0.0;
    for (int t = threadIdx.x; t < BE; t += BT) {
        const int64_t e = int64_t(blockIdx.x) * BE + t;
        if (e < N) nn += v[int64_t(r) * N + e].x * v[int64_t(r) * N + e].x + v[int64_t(r) * N + e].y * v[int64_t(r) * N + e].y;
    }
    __shared__ double red[BT / 64];
    nn = wsum(nn);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nn;
    __syncthreads();
    if (threadIdx.x == 0) part[int64_t(r) * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}
__global__ void k_colnorm_fin(int nb, const double *__restrict__ part, double *__restrict__ out)
{
    const int r = blockIdx.x;
    double a = 0.0;
    for (int b = threadIdx.x; b < nb; b += 64) a += part[int64_t(r) * nb + b];
    a = wsum(a);
    if (threadIdx.x == 0) out[r] = sqrt(a);
}

struct DevBufs {
    std::vector<void *> all;
    template <typename T>
    T *get(size_t n)
    {
        void *p = nullptr;
        BIE_HIP(hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)));
        all.push_back(p);
        return static_cast<T *>(p);
    }
    ~DevBufs()
    {
        for (void *p : all) (void)hipFree(p);
    }
};

// phases of a slot of the refinement engine
enum { SL_EMPTY = 0, SL_CHECK = 1, SL_FROM_B = 2, SL_NEW = 3, SL_CONT = 4 };
constexpr int MAX_CHECKS = 100;   // outer refinement steps per right-hand side

}  // namespace

// Mixed precision with iterative refinement, as a continuous batch.
//
// Each right-hand side is refined as x <- x + d, where the outer residual
// r = b - T x uses the FP64 matrix (FP64 block product on the matrix cores over
// the slots being checked) and decides convergence (standard criterion in FP64) and the correction solves T_low d = r with GMRES(m) to a relative
// tolerance inner_tol on the low-precision matrix: the split-BF16 block
// product on the matrix cores (Krylov basis stored in complex64, FP64
// arithmetic) or the FP32 packed matrix (FP64 vectors).
//
// W = slots right-hand sides are in flight (all R when slots = 0).  The host
// loop alternates (1) FP64 checks of every slot whose correction has finished,
// one product launch over those slots; a converged slot writes its solution
// out and takes the next right-hand side; (2) one GMRES cycle (<= m
// iterations) over every slot inside a correction, with one product launch per
// iteration over exactly those slots.  A slot therefore never waits for the
// slowest right-hand side of a block: throughput follows the mean number of
// iterations, which is what a warm start reduces.
template <typename VT>
static int solve_stream(const bie_op *opc, const void *Bv, void *Xv, int64_t R, const bie_solve_opts &o,
                        bie_solve_stat *stats, hipStream_t s, int low)
{
    bie_op *op = const_cast<bie_op *>(opc);
    if (o.method != BIE_GMRES) throw Error(BIE_EINVAL, "mixed precision uses GMRES");
    const int64_t N = op->mesh.N;
    const int m = o.restart;
    const int64_t W = o.slots > 0 ? std::min<int64_t>(o.slots, R) : R;
    Workspace *w = get_ws(op, W, m);
    const Cols ucols = uniform_cols(N, m);
    const double2 *B = static_cast<const double2 *>(Bv);
    double2 *X = static_cast<double2 *>(Xv);
    VT *V = reinterpret_cast<VT *>(w->V);
    const int vtype = sizeof(VT) == 16 ? VEC_C128 : sizeof(VT) == 8 ? VEC_C64 : VEC_F16;
    const int terms = o.inner_terms ? o.inner_terms : 3;
    // BF16-rounded vectors (2 terms) bound the attainable inner residual near
    // 2^-9: the inner tolerance is kept at 1e-2 or above for them
    const double itol = std::max(o.inner_tol > 0.0 ? o.inner_tol : 1e-3, terms == 2 ? 1e-2 : 0.0);
    const unsigned nb = unsigned((N + BE - 1) / BE);

    DevBufs db;
    double2 *Bs = db.get<double2>(size_t(W) * N);   // slot right-hand sides
    double2 *Xs = db.get<double2>(size_t(W) * N);   // slot solutions
    double2 *Rs = db.get<double2>(size_t(W) * N);   // outer residuals (right-hand sides of the corrections)
    double2 *Ds = db.get<double2>(size_t(W) * N);   // corrections
    double *part = db.get<double>(size_t(std::max(R, W)) * nb);
    double *nrm = db.get<double>(size_t(std::max(R, W)));
    int *dcols = db.get<int>(size_t(3 * W));   // [0, W): cycle list, [W, 2W): continuing, [2W, 3W): checks
    int *dskip = w->mask;

    auto colnorms = [&](const double2 *v, int64_t cnt, std::vector<double> &out) {
        hipLaunchKernelGGL(k_colnorm_part, dim3(nb, unsigned(cnt)), dim3(BT), 0, s, N, v, part);
        hipLaunchKernelGGL(k_colnorm_fin, dim3(unsigned(cnt)), dim3(64), 0, s, int(nb), part, nrm);
        BIE_HIP(hipGetLastError());
        out.resize(cnt);
        BIE_HIP(hipMemcpyAsync(out.data(), nrm, cnt * sizeof(double), hipMemcpyDeviceToHost, s));
        BIE_HIP(hipStreamSynchronize(s));
    };
    auto copy = [&](const double2 *a, double2 *b) { hipLaunchKernelGGL(k_copy, dim3(64), dim3(256), 0, s, N, a, b); };

    std::vector<double> bn;
    colnorms(B, R, bn);
    std::vector<bie_solve_stat> hs(R, bie_solve_stat{ 0, 0, NAN, NAN, 0, 0, o.use_x0 ? 1 : 0 });
    std::vector<int64_t> rhs(W, -1);
    std::vector<int> phase(W, SL_EMPTY), skip(W, 1), colsh(2 * W, 0), chk;
    std::vector<double> rin(W, 0.0), rn;
    std::vector<ColStat> st(W);
    int64_t next = 0;

    auto load = [&](int64_t sl) {
        if (next >= R) {
            rhs[sl] = -1;
            phase[sl] = SL_EMPTY;
            return;
        }
        const int64_t r = next++;
        rhs[sl] = r;
        copy(B + r * N, Bs + sl * N);
        if (o.use_x0) {
            copy(X + r * N, Xs + sl * N);
            phase[sl] = SL_CHECK;
        } else {
            hipLaunchKernelGGL(k_zero, dim3(64), dim3(256), 0, s, N, Xs + sl * N);
            phase[sl] = SL_FROM_B;
        }
    };
    auto retire = [&](int64_t sl, bool converged) {
        const int64_t r = rhs[sl];
        hs[r].converged = converged;
        copy(Xs + sl * N, X + r * N);
        load(sl);
    };
    // product with the low-precision matrix for the slots listed in colsh[c0 ..
    // c0 + n) (device copy at dcols + c0); packed FP32: skip array instead
    // (Xp complex64 when xf32; the packed FP32 product takes complex128 only)
    auto low_product = [&](const void *Xp, int vtype, int64_t ldx, double2 *Y, const double2 *Bsub, int c0, int n,
                           const int *pskip, int64_t sks) {
        if (low == MATBF16) gemm_product(op, Xp, ldx, vtype, Y, N, Bsub, N, n, dcols + c0, s, terms);
        else product(op, MAT32, true, Xp, ldx, Y, N, Bsub, N, W, pskip, sks, false, s);
    };
    auto push_st = [&]() { BIE_HIP(hipMemcpyAsync(w->st, st.data(), W * sizeof(ColStat), hipMemcpyHostToDevice, s)); };
    auto pull_st = [&]() {
        BIE_HIP(hipMemcpyAsync(st.data(), w->st, W * sizeof(ColStat), hipMemcpyDeviceToHost, s));
        BIE_HIP(hipStreamSynchronize(s));
    };
    const int *done_flags = &w->st[0].done;
    const int64_t done_stride = sizeof(ColStat) / sizeof(int);
    const int field_rnorm = offsetof(ColStat, rnorm) / sizeof(double);
    const dim3 vgrid(w->nblk, unsigned(W));
    const dim3 egrid(unsigned(std::min<int64_t>((N + BT - 1) / BT, 1024)), unsigned(W));

    for (int64_t sl = 0; sl < W; ++sl) load(sl);
    while (true) {
        // (1) settle: zero right-hand sides, starts from b, FP64 checks.  Each
        // pass retires (consuming a right-hand side) or advances every slot it
        // looks at, so the loop ends.
        while (true) {
            bool changed = false;
            for (int64_t sl = 0; sl < W; ++sl) {
                if (phase[sl] != SL_FROM_B) continue;
                const int64_t r = rhs[sl];
                changed = true;
                if (bn[r] == 0.0) {
                    hs[r].relres_est = hs[r].relres_true = 0.0;
                    retire(sl, true);
                    continue;
                }
                copy(Bs + sl * N, Rs + sl * N);
                rin[sl] = bn[r];
                hs[r].relres_true = 1.0;
                phase[sl] = SL_NEW;
            }
            chk.clear();
            for (int64_t sl = 0; sl < W; ++sl) {
                skip[sl] = phase[sl] == SL_CHECK ? 0 : 1;
                if (!skip[sl]) chk.push_back(int(sl));
            }
            if (chk.empty()) {
                if (changed) continue;
                break;
            }
            // r = b - T64 x for the slots to check: one FP64 block product on the
            // matrix cores, or the packed FP64 product of a star-split operator
            if (op->star) {
                BIE_HIP(hipMemcpyAsync(dskip, skip.data(), W * sizeof(int), hipMemcpyHostToDevice, s));
                product(op, MAT64, true, Xs, N, Rs, N, Bs, N, W, dskip, 1, false, s);
            } else {
                BIE_HIP(hipMemcpyAsync(dcols + 2 * W, chk.data(), chk.size() * sizeof(int), hipMemcpyHostToDevice, s));
                gemm64_product(op, Xs, N, Rs, N, Bs, N, int64_t(chk.size()), dcols + 2 * W, s);
            }
            colnorms(Rs, W, rn);
            for (int64_t sl = 0; sl < W; ++sl) {
                if (skip[sl]) continue;
                const int64_t r = rhs[sl];
                hs[r].mvps += 1;
                hs[r].checks += 1;
                const double rel = bn[r] > 0.0 ? rn[sl] / bn[r] : 0.0;
                hs[r].relres_true = rel;
                if (bn[r] == 0.0 || rel <= o.tol) retire(sl, true);
                else if (hs[r].mvps >= o.max_mvp || hs[r].checks >= MAX_CHECKS) retire(sl, false);
                else if (o.use_x0 == 2 && hs[r].checks == 1 && !(rel < 1.0)) {
                    // fallback: a guess no better than zero is replaced by zero
                    hs[r].x0_kept = 0;
                    hipLaunchKernelGGL(k_zero, dim3(64), dim3(256), 0, s, N, Xs + sl * N);
                    phase[sl] = SL_FROM_B;
                    changed = true;
                } else {
                    rin[sl] = rn[sl];
                    phase[sl] = SL_NEW;
                }
            }
        }
        // (2) one GMRES cycle over the slots inside a correction
        int nin = 0, ncont = 0;
        for (int64_t sl = 0; sl < W; ++sl)
            if (phase[sl] == SL_NEW || phase[sl] == SL_CONT) colsh[nin++] = int(sl);
        if (nin == 0) break;   // every slot empty: all right-hand sides retired
        for (int64_t sl = 0; sl < W; ++sl)
            if (phase[sl] == SL_CONT) colsh[W + ncont++] = int(sl);
        BIE_HIP(hipMemcpyAsync(dcols, colsh.data(), 2 * W * sizeof(int), hipMemcpyHostToDevice, s));
        for (int64_t sl = 0; sl < W; ++sl) {
            const bool in = phase[sl] == SL_NEW || phase[sl] == SL_CONT;
            st[sl] = ColStat{};
            st[sl].bnorm = rin[sl];
            st[sl].rnorm = rin[sl];
            st[sl].active = in;
            st[sl].done = in ? 0 : 1;
            st[sl].jcap = in ? int(std::min<int64_t>(m, std::max<int64_t>(1, o.max_mvp - hs[rhs[sl]].mvps))) : 0;
            skip[sl] = phase[sl] == SL_CONT ? 0 : 1;
            if (phase[sl] == SL_NEW) {
                hipLaunchKernelGGL(k_zero, dim3(64), dim3(256), 0, s, N, Ds + sl * N);
                copy(Rs + sl * N, w->Res + sl * N);
            }
        }
        push_st();
        if (ncont > 0) {   // inner residual r - T_low d of the continuing corrections
            BIE_HIP(hipMemcpyAsync(dskip, skip.data(), W * sizeof(int), hipMemcpyHostToDevice, s));
            low_product(Ds, VEC_C128, N, w->Res, Rs, int(W), ncont, dskip, 1);
            std::vector<int> need(W);
            for (int64_t sl = 0; sl < W; ++sl) need[sl] = 1 - skip[sl];
            BIE_HIP(hipMemcpyAsync(dskip, need.data(), W * sizeof(int), hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_norm, vgrid, dim3(BT), 0, s, ucols, w->Res, w->dpart, w->counters, w->st,
                               field_rnorm, (const int *)dskip);
            BIE_HIP(hipGetLastError());
            pull_st();
            bool exact = false;
            for (int64_t sl = 0; sl < W; ++sl)
                if (phase[sl] == SL_CONT) {
                    hs[rhs[sl]].mvps += 1;
                    if (st[sl].rnorm == 0.0) {   // correction solves the system exactly: skip the cycle
                        st[sl].done = 1;
                        st[sl].active = 0;
                        exact = true;
                    }
                }
            if (exact) push_st();
        }
        std::vector<int> act(W);
        int jmax = 0;
        for (int64_t sl = 0; sl < W; ++sl) {
            act[sl] = st[sl].active;
            if (act[sl]) jmax = std::max(jmax, st[sl].jcap);
        }
        BIE_HIP(hipMemcpyAsync(dskip, act.data(), W * sizeof(int), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_restart<VT>, egrid, dim3(BT), 0, s, ucols, m, w->Res, V, w->g, w->st, (const int *)dskip);
        BIE_HIP(hipGetLastError());
        for (int j = 0; j < jmax; ++j) {
            low_product(V + int64_t(j) * N, vtype, int64_t(m + 1) * N, w->W, nullptr, 0, nin, done_flags,
                        done_stride);
            arnoldi_step<VT>(w, ucols, N, V, m, j, itol, W, s);
        }
        hipLaunchKernelGGL(k_lsq, dim3(unsigned(W)), dim3(64), size_t(m) * m * sizeof(double2), s, m, w->H, w->g,
                           w->y, w->st);
        hipLaunchKernelGGL(k_xupd<VT>, egrid, dim3(BT), 0, s, ucols, m, V, w->y, Ds, w->st);
        BIE_HIP(hipGetLastError());
        pull_st();
        for (int64_t sl = 0; sl < W; ++sl) {
            if (phase[sl] != SL_NEW && phase[sl] != SL_CONT) continue;
            const int64_t r = rhs[sl];
            if (act[sl]) {
                hs[r].iters += st[sl].jend;
                hs[r].mvps += st[sl].jend;
                hs[r].relres_est = st[sl].est * rin[sl] / bn[r];
            }
            if (!act[sl] || st[sl].est <= itol || st[sl].brk || hs[r].mvps >= o.max_mvp) {
                hipLaunchKernelGGL(k_axpy_cols, dim3(64), dim3(256), 0, s, N, Ds + sl * N, Xs + sl * N);
                phase[sl] = SL_CHECK;
            } else {
                phase[sl] = SL_CONT;
            }
        }
        BIE_HIP(hipGetLastError());
    }
    BIE_HIP(hipStreamSynchronize(s));
    int status = BIE_OK;
    for (int64_t r = 0; r < R; ++r) {
        if (!hs[r].converged) status = BIE_NOT_CONVERGED;
        if (stats) stats[r] = hs[r];
    }
    return status;
}


// ----------------------------------------------------------------------------- batched solves
// GMRES(m) for the right-hand sides of several operators of different sizes at
// once.  Every column keeps its own Krylov basis, Hessenberg matrix and
// criterion, as in one solve; the columns of all operators share each launch:
// the product is one grouped tile launch over (operator, tile unit, column
// group) items, longest first, and one grouped reduce over (column, row block)
// items, and the Arnoldi kernels read a column table (length and offsets).
// A tile item goes through the columns of its group with the unit's tiles
// kept in the caches, so each matrix is read from memory about once per group.
// The m iterations of a cycle are captured once in a HIP graph and replayed
// every cycle; columns whose cycle has ended skip on the device.  Tiles per
// unit and columns per group are chosen per batch by timing candidates on the
// batch itself (autotuner, cached per batch shape).

namespace {

struct BatchConfig {
    int unit = 0;      // tiles per work unit; 0: autotune
    int graph = 1;     // replay the cycles as a HIP graph
    int mfma = 1;      // precision 1, FP32 tiles: the grouped products on the matrix cores
};
BatchConfig g_batch;

// Device layout of a grouped product for one choice of tiles per unit (U) and
// columns per work item (G).
struct GLayout {
    int U = 0, G = 0;
    DevBufs db;
    GProb *probs = nullptr;
    int32_t *items = nullptr, *ritems = nullptr;
    int64_t nitems = 0, nritems = 0;
    int64_t *gpoff = nullptr;   // partial-vector offset per column
    double2 *gpart = nullptr;   // partial vectors of all columns
    std::vector<int32_t> h_items, h_ritems, h_c0, h_c1;   // host copies: items, reduce items, columns of each problem
    std::vector<GProb> h_probs;
};

// The problems of layout L with other matrices of the same sizes and units
// (the FP64 copies for the residuals, the preconditioners' matrices).
GProb *probs_on(DevBufs &db, const GLayout &L, const std::vector<const void *> &Z)
{
    std::vector<GProb> q = L.h_probs;
    for (size_t p = 0; p < q.size(); ++p) q[p].Z = Z[p];
    GProb *d = db.get<GProb>(q.size());
    BIE_HIP(hipMemcpy(d, q.data(), q.size() * sizeof(GProb), hipMemcpyHostToDevice));
    return d;
}

std::unique_ptr<GLayout> make_layout(const bie_op *const *ops, int64_t P, const int64_t *R, int U, int G, bool mat64)
{
    auto L = std::make_unique<GLayout>();
    L->U = U;
    L->G = G;
    std::vector<GProb> probs(P);
    std::vector<int64_t> nslots(P);
    std::vector<std::vector<int32_t>> unitsv(P);
    for (int64_t p = 0; p < P; ++p) {
        const int64_t nT = ops[p]->pk.nT;
        std::vector<int32_t> units, uptr;
        std::vector<int64_t> seg;
        if (U < 0) {   // the operator's own single-product units
            units = ops[p]->pk.h_units;
            uptr = ops[p]->pk.h_unit_ptr;
            seg = ops[p]->pk.h_seg;
        } else {
            build_units(nT, U, units, uptr, seg);
        }
        int32_t *du = L->db.get<int32_t>(units.size());
        int32_t *dp = L->db.get<int32_t>(uptr.size());
        int64_t *ds = L->db.get<int64_t>(seg.size());
        BIE_HIP(hipMemcpy(du, units.data(), units.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        BIE_HIP(hipMemcpy(dp, uptr.data(), uptr.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        BIE_HIP(hipMemcpy(ds, seg.data(), seg.size() * sizeof(int64_t), hipMemcpyHostToDevice));
        probs[p] = GProb{ mat64 ? ops[p]->Z64 : ops[p]->Z32, ops[p]->mesh.N, nT, seg[nT], du, dp, ds, 0, 0 };
        nslots[p] = seg[nT];
        unitsv[p] = std::move(units);
    }
    // tile items (p, u, g), longest first (work = columns x tiles)
    struct Item {
        int64_t work;
        int32_t p, u, g;
    };
    std::vector<Item> tl;
    for (int64_t p = 0; p < P; ++p)
        for (int64_t u = 0; u < int64_t(unitsv[p].size() / 3); ++u) {
            const int64_t nt = unitsv[p][3 * u + 2] - unitsv[p][3 * u + 1];
            for (int64_t g = 0; g * G < R[p]; ++g)
                tl.push_back(Item{ nt * std::min<int64_t>(G, R[p] - g * G), int32_t(p), int32_t(u), int32_t(g) });
        }
    std::stable_sort(tl.begin(), tl.end(), [](const Item &a, const Item &b) { return a.work > b.work; });
    std::vector<int32_t> items, ritems;
    items.reserve(3 * tl.size());
    for (const Item &it : tl) {
        items.push_back(it.p);
        items.push_back(it.u);
        items.push_back(it.g);
    }
    std::vector<int64_t> gpoff;
    int64_t c = 0, off = 0;
    for (int64_t p = 0; p < P; ++p) {
        probs[p].c0 = int32_t(c);
        for (int64_t r = 0; r < R[p]; ++r, ++c) {
            gpoff.push_back(off);
            off += nslots[p];
            for (int64_t I = 0; I < probs[p].nT; ++I) {
                ritems.push_back(int32_t(c));
                ritems.push_back(int32_t(I));
            }
        }
        probs[p].c1 = int32_t(c);
    }
    if (items.size() / 3 > 0x7fffffff || ritems.size() / 2 > 0x7fffffff)
        throw Error(BIE_EINVAL, "batch too large for one grouped launch");
    L->nitems = int64_t(items.size() / 3);
    L->nritems = int64_t(ritems.size() / 2);
    L->probs = L->db.get<GProb>(P);
    L->items = L->db.get<int32_t>(items.size());
    L->ritems = L->db.get<int32_t>(ritems.size());
    L->gpoff = L->db.get<int64_t>(gpoff.size());
    L->gpart = L->db.get<double2>(size_t(off) * TB);
    BIE_HIP(hipMemcpy(L->probs, probs.data(), P * sizeof(GProb), hipMemcpyHostToDevice));
    BIE_HIP(hipMemcpy(L->items, items.data(), items.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    BIE_HIP(hipMemcpy(L->ritems, ritems.data(), ritems.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    BIE_HIP(hipMemcpy(L->gpoff, gpoff.data(), gpoff.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    L->h_items = std::move(items);
    L->h_ritems = std::move(ritems);
    L->h_probs = probs;
    for (int64_t p = 0; p < P; ++p) {
        L->h_c0.push_back(probs[p].c0);
        L->h_c1.push_back(probs[p].c1);
    }
    return L;
}

// Autotuner choices of batched solves: batch shape -> (tiles per unit,
// columns per item), kept in the library's tuning registry (tune.cpp).
// The key names the precision, the number of operators and right-hand sides,
// and a 64-bit FNV-1a hash of the (N_p, R_p) list.
std::string batch_key(const bie_op *const *ops, int64_t P, const int64_t *R, bool mat64, bool mfma = false)
{
    uint64_t h = 1469598103934665603ull;
    int64_t nr = 0;
    auto mix = [&](int64_t v) {
        for (int b = 0; b < 8; ++b) {
            h ^= uint64_t(v >> (8 * b)) & 0xff;
            h *= 1099511628211ull;
        }
    };
    for (int64_t p = 0; p < P; ++p) {
        mix(ops[p]->mesh.N);
        mix(R[p]);
        nr += R[p];
    }
    char hex[17];
    snprintf(hex, sizeof hex, "%016llx", (unsigned long long)h);
    return std::string(mat64 ? "batch:f64" : (mfma ? "batch:f32mf" : "batch:f32")) + ":P" + std::to_string(P) + ":R" +
           std::to_string(nr) + ":" + hex;
}

}  // namespace

int solve_batch(const bie_op *const *ops, const bie_calderon *const *pcs, int64_t P, const void *const *Bp,
                void *const *Xp, const int64_t *Rp, const bie_solve_opts &o, bie_solve_stat *stats, hipStream_t user)
{
    if (o.method != BIE_GMRES || (o.precision != 0 && o.precision != 1))
        throw Error(BIE_EINVAL, "batched solves take GMRES with precision 0 or 1");
    if (o.crit != BIE_SCC && o.crit != BIE_RSCC && o.crit != BIE_CCC) throw Error(BIE_EINVAL, "unknown criterion");
    // precision 1: the cycles on the FP32 tiles, every residual (restart vector
    // and criterion) on the FP64 tiles of the same operator
    const bool prec1 = o.precision == 1;
    // split: precision 1 with split-BF16 operators: the cycles' products are the
    // split-BF16 block products of each operator (matrix cores, every column of
    // the operator at once), the residuals the grouped FP64 tile pass
    const bool split = prec1 && ops[0]->Abf != nullptr;
    const bool mat64 = !prec1 && ops[0]->Z64 != nullptr;
    const bool res64 = prec1 || mat64;
    const bool lay64 = split || mat64;   // tiles of the grouped layout
    // precision 1 on FP32 tiles: the cycles' grouped products on the FP32 matrix
    // cores (the FP64 residuals keep the certification)
    const bool mf = prec1 && !split && g_batch.mfma != 0;
    if (o.crit != BIE_SCC && !res64)
        throw Error(BIE_EINVAL, "the random-sampling criterion needs the FP64 matrices (FP64 storage or precision 1)");
    for (int64_t p = 0; p < P; ++p) {
        if (split) {
            if (!ops[p]->Z64 || !ops[p]->Abf)
                throw Error(BIE_EINVAL, "all operators of a split-BF16 batch need storage BIE_SPLIT_BF16");
        } else if (prec1) {
            if (!ops[p]->Z64 || !ops[p]->Z32)
                throw Error(BIE_EINVAL, "precision 1 needs the FP32 and the FP64 matrix of every operator "
                                        "(storage BIE_C64 with keep_fp64, or BIE_SPLIT_BF16)");
        } else if ((ops[p]->Z64 != nullptr) != mat64 || (!mat64 && !ops[p]->Z32)) {
            throw Error(BIE_EINVAL, "all operators of a batch need the same stored matrix (FP64 or FP32)");
        }
        if (ops[p]->device != ops[0]->device) throw Error(BIE_EINVAL, "all operators of a batch on one device");
        if (pcs && (!pcs[p] || calderon_operator(pcs[p]) != ops[p]))
            throw Error(BIE_EINVAL, "preconditioner " + std::to_string(p) + " is missing or was built for another operator");
    }
    const int m = o.restart;
    // column tables
    std::vector<int32_t> prob;
    std::vector<int64_t> cn, voff, woff, aoff;
    int64_t nv = 0, nw = 0, na = 0, Nmax = 0;
    for (int64_t p = 0; p < P; ++p) {
        const int64_t N = ops[p]->mesh.N;
        Nmax = std::max(Nmax, N);
        for (int64_t r = 0; r < Rp[p]; ++r) {
            prob.push_back(int32_t(p));
            cn.push_back(N);
            voff.push_back(nv);
            woff.push_back(nw);
            aoff.push_back(na);
            nv += (m + 1) * N;
            nw += N;
            na += (N + AB - 1) / AB;
        }
    }
    const int64_t C = int64_t(prob.size());
    if (C == 0) return BIE_OK;

    // own stream (graph capture is not possible on the null stream), ordered
    // after the caller's stream
    hipStream_t s;
    BIE_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    struct StreamGuard {
        hipStream_t s;
        ~StreamGuard() { (void)hipStreamDestroy(s); }
    } sguard{ s };
    {
        hipEvent_t ev;
        BIE_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        BIE_HIP(hipEventRecord(ev, user));
        BIE_HIP(hipStreamWaitEvent(s, ev, 0));
        BIE_HIP(hipStreamSynchronize(s));
        (void)hipEventDestroy(ev);
    }

    DevBufs db;
    Workspace ws;
    Workspace *w = &ws;
    w->N = Nmax;
    w->R = C;
    w->m = m;
    w->nblk = unsigned((Nmax + BE - 1) / BE);
    w->V = w->alloc<double2>(size_t(nv));
    w->W = w->alloc<double2>(size_t(nw));
    w->Res = w->alloc<double2>(size_t(nw));
    w->H = w->alloc<double2>(size_t(C) * m * (m + 1));
    w->sn = w->alloc<double2>(size_t(C) * m);
    w->cs = w->alloc<double>(size_t(C) * m);
    w->g = w->alloc<double2>(size_t(C) * (m + 1));
    w->y = w->alloc<double2>(size_t(C) * m);
    w->P1 = w->alloc<double2>(size_t(na) * (m + 1));
    w->P2 = w->alloc<double2>(size_t(na) * (m + 1));
    w->PN = w->alloc<double>(size_t(na));
    w->PW = w->alloc<double>(size_t(na));
    w->dpart = w->alloc<double>(size_t(C) * w->nblk);
    w->counters = w->alloc<unsigned>(size_t(C));
    BIE_HIP(hipMemsetAsync(w->counters, 0, size_t(C) * sizeof(unsigned), s));
    w->st = w->alloc<ColStat>(size_t(C));
    w->mask = w->alloc<int>(size_t(C));
    double2 *Xw = db.get<double2>(size_t(nw)), *Bw = db.get<double2>(size_t(nw));
    int32_t *dprob = db.get<int32_t>(C);
    int64_t *dcn = db.get<int64_t>(C), *dvo = db.get<int64_t>(C), *dwo = db.get<int64_t>(C),
            *dao = db.get<int64_t>(C);
    BIE_HIP(hipMemcpyAsync(dprob, prob.data(), C * sizeof(int32_t), hipMemcpyHostToDevice, s));
    BIE_HIP(hipMemcpyAsync(dcn, cn.data(), C * sizeof(int64_t), hipMemcpyHostToDevice, s));
    BIE_HIP(hipMemcpyAsync(dvo, voff.data(), C * sizeof(int64_t), hipMemcpyHostToDevice, s));
    BIE_HIP(hipMemcpyAsync(dwo, woff.data(), C * sizeof(int64_t), hipMemcpyHostToDevice, s));
    BIE_HIP(hipMemcpyAsync(dao, aoff.data(), C * sizeof(int64_t), hipMemcpyHostToDevice, s));
    Cols cl;
    cl.n = dcn;
    cl.voff = dvo;
    cl.woff = dwo;
    cl.poff = dao;
    cl.N = Nmax;
    cl.m = m;
    // right-hand sides and initial guesses into the column buffers
    for (int64_t p = 0; p < P; ++p) {
        const int64_t c0 = std::find(prob.begin(), prob.end(), int32_t(p)) - prob.begin();
        if (Rp[p] == 0) continue;
        const size_t bytes = size_t(Rp[p]) * ops[p]->mesh.N * sizeof(double2);
        BIE_HIP(hipMemcpyAsync(Bw + woff[c0], Bp[p], bytes, hipMemcpyDeviceToDevice, s));
        if (o.use_x0) BIE_HIP(hipMemcpyAsync(Xw + woff[c0], Xp[p], bytes, hipMemcpyDeviceToDevice, s));
    }
    if (!o.use_x0) hipLaunchKernelGGL(k_zero, dim3(1024), dim3(256), 0, s, nw, Xw);

    // grouped product layout: tiles per unit and columns per item from the autotuner
    std::unique_ptr<GLayout> L;
    const std::string key = batch_key(ops, P, Rp, lay64, mf);
    int U = g_batch.unit, G = 8;
    if (U == 0 && !tune_enabled()) U = 8;   // tuning off: the fixed default units
    if (U == 0) {
        std::vector<int> v;
        if (tune_get(key, v) && v.size() == 2 && v[0] >= 1 && v[0] <= 64 && v[1] >= 1 && v[1] <= 4096) {
            U = v[0];
            G = v[1];
        }
    }
    auto layout_cols = [&](const GLayout &gl, const int64_t *xoff, int64_t xstep) {
        return GCols{ dprob, xoff, dwo, gl.gpoff, xstep };
    };
    if (U == 0) {
        // time each candidate: 1 warm-up + 3 products of the right-hand sides
        hipEvent_t e0, e1;
        BIE_HIP(hipEventCreate(&e0));
        BIE_HIP(hipEventCreate(&e1));
        float best = 0.f;
        for (int cu : { 4, 8, 16 })
            for (int cg : { 4, 8, 16, 32 }) {
                auto Lc = make_layout(ops, P, Rp, cu, cg, lay64);
                const GCols gc = layout_cols(*Lc, dwo, 0);
                auto run = [&]() {
                    grouped_product(lay64, Lc->probs, gc, Lc->items, Lc->nitems, Lc->G, Lc->ritems, Lc->nritems, Bw,
                                    Lc->gpart, w->W, nullptr, nullptr, 1, s, mf);
                };
                run();
                BIE_HIP(hipEventRecord(e0, s));
                for (int rep = 0; rep < 3; ++rep) run();
                BIE_HIP(hipEventRecord(e1, s));
                BIE_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                BIE_HIP(hipEventElapsedTime(&ms, e0, e1));
                if (!L || ms < best) {
                    best = ms;
                    L = std::move(Lc);
                }
            }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        tune_put(key, { L->U, L->G });
    } else {
        L = make_layout(ops, P, Rp, U, G, lay64);
    }
    const GCols gres = layout_cols(*L, dwo, 0);
    // the residuals' matrices (FP64 tiles under precision 1)
    const GProb *probs_res = L->probs;
    if (res64 != lay64) {
        std::vector<const void *> Z(P);
        for (int64_t p = 0; p < P; ++p) Z[p] = ops[p]->Z64;
        probs_res = probs_on(db, *L, Z);
    }
    // the preconditioners' matrices M, in the precision of the cycles' products;
    // their unit tables are those of the operators' layout (the same sizes)
    // unless the layout uses each operator's own units
    const GProb *probs_m = nullptr;
    std::unique_ptr<GLayout> LM;
    double2 *Wz = nullptr;
    std::vector<const bie_op *> views(P, nullptr);
    if (pcs && split) {
        for (int64_t p = 0; p < P; ++p) views[p] = calderon_view(pcs[p], true, s);
        Wz = db.get<double2>(size_t(nw));
    } else if (pcs) {
        std::vector<const void *> Z(P);
        for (int64_t p = 0; p < P; ++p) {
            views[p] = mat64 ? calderon_view(pcs[p], false, s) : calderon_view32(pcs[p], s);
            Z[p] = mat64 ? views[p]->Z64 : views[p]->Z32;
        }
        if (L->U >= 1) {
            probs_m = probs_on(db, *L, Z);
        } else {
            LM = make_layout(views.data(), P, Rp, L->U, L->G, mat64);
            probs_m = LM->probs;
        }
        Wz = db.get<double2>(size_t(nw));
    }
    // partial vectors and items of the preconditioner's products
    const GLayout &LMr = LM ? *LM : *L;
    // split mode: first column of every problem, the problems the captured
    // cycle covers, and one uncaptured product of every operator (and
    // preconditioner) so that its staging buffers exist and its launch shape is
    // tuned before any capture
    std::vector<int64_t> pc0(P, 0);
    for (int64_t p = 1; p < P; ++p) pc0[p] = pc0[p - 1] + Rp[p - 1];
    std::vector<int> live_prob(P, 0);
    int64_t probs_built = -1;
    auto split_product = [&](const bie_op *op, int64_t p, const double2 *X0, int64_t ldx, double2 *Y0) {
        gemm_product(op, X0, ldx, VEC_C128, Y0, ops[p]->mesh.N, nullptr, 0, Rp[p], nullptr, s, 3);
    };
    if (split)
        for (int64_t p = 0; p < P; ++p) {
            if (Rp[p] == 0) continue;
            const int64_t c0 = pc0[p], N = ops[p]->mesh.N;
            split_product(ops[p], p, Bw + woff[c0], N, w->W + woff[c0]);
            if (pcs) split_product(views[p], p, Bw + woff[c0], N, w->W + woff[c0]);
        }
    // Live work: the tile items with at least one live column and the reduce
    // items of live columns, rebuilt (and the cycle graph captured again) when
    // the live columns have dropped by a quarter since the last build, so that
    // late cycles launch only the work of the slow columns.  Order and
    // arithmetic per column are unchanged (results are bitwise the same).
    int32_t *litems = db.get<int32_t>(std::max<size_t>(1, L->h_items.size()));
    int32_t *lritems = db.get<int32_t>(std::max<size_t>(1, L->h_ritems.size()));
    int64_t nlitems = 0, nlritems = 0, live_built = -1;
    auto build_live = [&](const std::vector<int> &live) {
        std::vector<int32_t> it, rit;
        for (size_t i = 0; 3 * i < L->h_items.size(); ++i) {
            const int32_t p = L->h_items[3 * i], g = L->h_items[3 * i + 2];
            const int32_t cb = L->h_c0[p] + g * L->G, ce = std::min(L->h_c1[p], cb + L->G);
            bool any = false;
            for (int32_t c = cb; c < ce && !any; ++c) any = live[c] != 0;
            if (any) it.insert(it.end(), { p, L->h_items[3 * i + 1], g });
        }
        for (size_t i = 0; 2 * i < L->h_ritems.size(); ++i)
            if (live[L->h_ritems[2 * i]]) rit.insert(rit.end(), { L->h_ritems[2 * i], L->h_ritems[2 * i + 1] });
        nlitems = int64_t(it.size() / 3);
        nlritems = int64_t(rit.size() / 2);
        if (!it.empty()) BIE_HIP(hipMemcpyAsync(litems, it.data(), it.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        if (!rit.empty())
            BIE_HIP(hipMemcpyAsync(lritems, rit.data(), rit.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        BIE_HIP(hipStreamSynchronize(s));
        live_built = 0;
        for (int v : live) live_built += v != 0;
    };
    std::vector<int> all_live(C, 1);
    build_live(all_live);
    auto full_residual = [&](const int *skipdev) {   // Res = B - T X for the columns not skipped
        grouped_product(res64, probs_res, gres, litems, nlitems, L->G, lritems, nlritems, Xw, L->gpart, w->Res, Bw,
                        skipdev, 1, s, mf);
    };

    std::vector<bie_solve_stat> hs(C, bie_solve_stat{ 0, 0, NAN, NAN, 0, 0, o.use_x0 ? 1 : 0 });
    std::vector<ColStat> st(C);
    std::vector<int> active(C, 1), need(C), skip(C);
    auto push_st = [&]() { BIE_HIP(hipMemcpyAsync(w->st, st.data(), C * sizeof(ColStat), hipMemcpyHostToDevice, s)); };
    auto pull_st = [&]() {
        BIE_HIP(hipMemcpyAsync(st.data(), w->st, C * sizeof(ColStat), hipMemcpyDeviceToHost, s));
        BIE_HIP(hipStreamSynchronize(s));
    };
    auto push_mask = [&](const std::vector<int> &v) {
        BIE_HIP(hipMemcpyAsync(w->mask, v.data(), C * sizeof(int), hipMemcpyHostToDevice, s));
    };
    const dim3 vgrid(w->nblk, unsigned(C));
    const dim3 egrid(unsigned(std::min<int64_t>((Nmax + BT - 1) / BT, 1024)), unsigned(C));
    const int field_rnorm = offsetof(ColStat, rnorm) / sizeof(double);
    const int field_bnorm = offsetof(ColStat, bnorm) / sizeof(double);
    auto norms = [&](const double2 *v, const std::vector<int> &msk, int field) {
        push_mask(msk);
        hipLaunchKernelGGL(k_norm, vgrid, dim3(BT), 0, s, cl, v, w->dpart, w->counters, w->st, field,
                           (const int *)w->mask);
        BIE_HIP(hipGetLastError());
    };
    for (int64_t c = 0; c < C; ++c) {
        st[c] = ColStat{};
        st[c].active = 1;
    }
    push_st();
    norms(Bw, active, field_bnorm);
    pull_st();
    for (int64_t c = 0; c < C; ++c)
        if (st[c].bnorm == 0.0) {
            active[c] = 0;
            hs[c].converged = 1;
            hs[c].relres_est = hs[c].relres_true = 0.0;
            hipLaunchKernelGGL(k_zero, dim3(64), dim3(256), 0, s, cn[c], Xw + woff[c]);
        }
    // skip array for the residual product: 1 = skip
    auto residual_of = [&](const std::vector<int> &nd) {
        for (int64_t c = 0; c < C; ++c) skip[c] = nd[c] ? 0 : 1;
        push_mask(skip);
        full_residual(w->mask);
        norms(w->Res, nd, field_rnorm);
        for (int64_t c = 0; c < C; ++c)
            if (nd[c]) hs[c].mvps += 1;
    };
    for (int64_t c = 0; c < C; ++c) need[c] = active[c];
    if (o.use_x0) {
        residual_of(need);
        if (o.use_x0 == 2) {
            pull_st();
            std::vector<int> back(C, 0);
            bool any = false;
            for (int64_t c = 0; c < C; ++c)
                if (active[c] && !(st[c].rnorm < st[c].bnorm)) {
                    back[c] = 1;
                    any = true;
                    hs[c].x0_kept = 0;
                    hipLaunchKernelGGL(k_zero, dim3(64), dim3(256), 0, s, cn[c], Xw + woff[c]);
                    hipLaunchKernelGGL(k_copy, dim3(64), dim3(256), 0, s, cn[c], Bw + woff[c], w->Res + woff[c]);
                }
            if (any) norms(w->Res, back, field_rnorm);
        }
    } else {
        BIE_HIP(hipMemcpyAsync(w->Res, Bw, size_t(nw) * sizeof(double2), hipMemcpyDeviceToDevice, s));
        norms(w->Res, need, field_rnorm);
    }
    pull_st();
    if (o.use_x0)
        for (int64_t c = 0; c < C; ++c)
            if (active[c] && st[c].rnorm / st[c].bnorm <= o.tol) {
                active[c] = 0;
                hs[c].converged = 1;
                hs[c].checks += 1;
                hs[c].relres_est = hs[c].relres_true = st[c].rnorm / st[c].bnorm;
            }

    // Random-sampling criterion (RSCC, and the gate of CCC) of the columns in
    // `on`: S_p rows of problem p drawn for each column from rscc_seed plus its
    // number of earlier checks, |b_i - (T x)_i|^2 on the FP64 tiles; the value
    // goes to relres_true, S_p / N_p of a product (rounded up) to its count.
    std::vector<int64_t> ncheck(C, 0);
    const int64_t Smax = std::min<int64_t>(std::max<int64_t>(o.rscc_rows, 1), MAX_RSCC_ROWS);
    int64_t *drows = nullptr;
    double *drs = nullptr;
    if (o.crit != BIE_SCC) {
        drows = db.get<int64_t>(size_t(C) * Smax);
        drs = db.get<double>(size_t(C) * Smax);
    }
    auto sampled_check = [&](const std::vector<int> &on) {
        std::vector<int64_t> rows(size_t(C) * Smax, 0);
        std::vector<int64_t> Sof(P, 0), c0of(P, 0);
        for (int64_t p = 0, c0 = 0; p < P; c0 += Rp[p], ++p) {
            c0of[p] = c0;
            Sof[p] = std::min<int64_t>(Smax, ops[p]->mesh.N);
            for (int64_t r = 0; r < Rp[p]; ++r)
                if (on[c0 + r]) {
                    const auto v = rscc_rows(ops[p]->mesh.N, Sof[p], o.rscc_seed + uint64_t(ncheck[c0 + r]));
                    std::copy(v.begin(), v.end(), rows.begin() + c0 * Smax + r * Sof[p]);
                }
        }
        BIE_HIP(hipMemcpyAsync(drows, rows.data(), rows.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
        push_mask(on);
        for (int64_t p = 0; p < P; ++p) {
            const int64_t c0 = c0of[p];
            bool any = false;
            for (int64_t r = 0; r < Rp[p] && !any; ++r) any = on[c0 + r] != 0;
            if (!any) continue;
            sampled_residual(ops[p], Bw + woff[c0], Xw + woff[c0], Rp[p], Sof[p], drows + c0 * Smax, drs + c0 * Smax,
                             w->mask + c0, s);
        }
        std::vector<double> rs(size_t(C) * Smax);
        BIE_HIP(hipMemcpyAsync(rs.data(), drs, rs.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        pull_st();
        for (int64_t p = 0; p < P; ++p)
            for (int64_t r = 0; r < Rp[p]; ++r) {
                const int64_t c = c0of[p] + r;
                if (!on[c]) continue;
                double sum = 0.0;
                for (int64_t i = 0; i < Sof[p]; ++i) sum += rs[c0of[p] * Smax + r * Sof[p] + i];
                const int64_t N = ops[p]->mesh.N;
                hs[c].relres_true = std::sqrt(double(N) / double(Sof[p]) * sum) / st[c].bnorm;
                hs[c].checks += 1;
                ncheck[c] += 1;
                hs[c].mvps += (Sof[p] + N - 1) / N;
            }
    };

    // the m iterations of a cycle, captured once, replayed per cycle
    const int *done_flags = &w->st[0].done;
    const int64_t done_stride = sizeof(ColStat) / sizeof(int);
    auto cycle_body = [&]() {
        for (int j = 0; j < m; ++j) {
            if (split) {   // per operator: all its columns in one split-BF16 block product
                for (int64_t p = 0; p < P; ++p) {
                    if (!live_prob[p]) continue;
                    const int64_t c0 = pc0[p], N = ops[p]->mesh.N;
                    const double2 *vj = w->V + voff[c0] + int64_t(j) * N;
                    if (pcs) {
                        split_product(views[p], p, vj, int64_t(m + 1) * N, Wz + woff[c0]);
                        split_product(ops[p], p, Wz + woff[c0], N, w->W + woff[c0]);
                    } else {
                        split_product(ops[p], p, vj, int64_t(m + 1) * N, w->W + woff[c0]);
                    }
                }
            } else if (pcs) {   // w = T (M v_j)
                const GCols gm = layout_cols(LMr, dvo, j);
                if (LM)
                    grouped_product(mat64, probs_m, gm, LM->items, LM->nitems, LM->G, LM->ritems, LM->nritems, w->V,
                                    LM->gpart, Wz, nullptr, done_flags, done_stride, s, mf);
                else
                    grouped_product(mat64, probs_m, gm, litems, nlitems, L->G, lritems, nlritems, w->V, L->gpart, Wz,
                                    nullptr, done_flags, done_stride, s, mf);
                grouped_product(mat64, L->probs, gres, litems, nlitems, L->G, lritems, nlritems, Wz, L->gpart, w->W,
                                nullptr, done_flags, done_stride, s, mf);
            } else {
                const GCols gv = layout_cols(*L, dvo, j);
                grouped_product(mat64, L->probs, gv, litems, nlitems, L->G, lritems, nlritems, w->V, L->gpart, w->W,
                                nullptr, done_flags, done_stride, s, mf);
            }
            arnoldi_step<double2>(w, cl, Nmax, w->V, m, j, o.tol, C, s);
        }
    };
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    struct GraphGuard {
        hipGraph_t &g;
        hipGraphExec_t &e;
        ~GraphGuard()
        {
            if (e) (void)hipGraphExecDestroy(e);
            if (g) (void)hipGraphDestroy(g);
        }
    } gguard{ graph, gexec };
    const bool use_graph = g_batch.graph != 0;
    const bool prof_was = prof_active();
    auto capture = [&]() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
        prof_enable(false);   // no event records inside the captured graph
        BIE_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        cycle_body();
        BIE_HIP(hipStreamEndCapture(s, &graph));
        BIE_HIP(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
        prof_enable(prof_was);
    };
    if (use_graph && !split) capture();

    while (true) {
        bool any = false;
        for (int64_t c = 0; c < C; ++c) {
            if (active[c] && hs[c].mvps >= o.max_mvp) active[c] = 0;
            any = any || active[c];
        }
        if (!any) break;
        int64_t nlive = 0;
        for (int64_t c = 0; c < C; ++c) nlive += active[c] != 0;
        if (4 * nlive <= 3 * live_built) {
            build_live(active);
            if (use_graph && !split) capture();
        }
        if (split) {   // the cycle covers the problems with live columns; recaptured when they drop by a quarter
            int64_t nlp = 0;
            for (int64_t p = 0; p < P; ++p) {
                bool any = false;
                for (int64_t r = 0; r < Rp[p] && !any; ++r) any = active[pc0[p] + r] != 0;
                nlp += any;
            }
            if (probs_built < 0 || 4 * nlp <= 3 * probs_built) {
                for (int64_t p = 0; p < P; ++p) {
                    bool any = false;
                    for (int64_t r = 0; r < Rp[p] && !any; ++r) any = active[pc0[p] + r] != 0;
                    live_prob[p] = any;
                }
                probs_built = nlp;
                if (use_graph) capture();
            }
        }
        for (int64_t c = 0; c < C; ++c) {
            ColStat &q = st[c];
            q.done = active[c] ? 0 : 1;
            q.active = active[c];
            q.jend = 0;
            q.brk = 0;
            q.jcap = int(std::min<int64_t>(m, std::max<int64_t>(1, o.max_mvp - hs[c].mvps)));
            need[c] = active[c];
        }
        push_st();
        push_mask(need);
        hipLaunchKernelGGL(k_restart<double2>, egrid, dim3(BT), 0, s, cl, m, w->Res, w->V, w->g, w->st,
                           (const int *)w->mask);
        BIE_HIP(hipGetLastError());
        if (use_graph) BIE_HIP(hipGraphLaunch(gexec, s));
        else cycle_body();
        hipLaunchKernelGGL(k_lsq, dim3(unsigned(C)), dim3(64), size_t(m) * m * sizeof(double2), s, m, w->H, w->g,
                           w->y, w->st);
        if (pcs && split) {   // x += M (V y) for the active columns, M in split-BF16
            hipLaunchKernelGGL(k_zero, dim3(1024), dim3(256), 0, s, nw, Wz);
            hipLaunchKernelGGL(k_xupd<double2>, egrid, dim3(BT), 0, s, cl, m, w->V, w->y, Wz, w->st);
            for (int64_t p = 0; p < P; ++p)
                if (live_prob[p])
                    split_product(views[p], p, Wz + woff[pc0[p]], ops[p]->mesh.N, w->W + woff[pc0[p]]);
            hipLaunchKernelGGL(k_add_active, egrid, dim3(BT), 0, s, cl, (const double2 *)w->W, Xw, w->st);
        } else if (pcs) {   // x += M (V y) for the active columns
            hipLaunchKernelGGL(k_zero, dim3(1024), dim3(256), 0, s, nw, Wz);
            hipLaunchKernelGGL(k_xupd<double2>, egrid, dim3(BT), 0, s, cl, m, w->V, w->y, Wz, w->st);
            for (int64_t c = 0; c < C; ++c) skip[c] = active[c] ? 0 : 1;
            push_mask(skip);
            const GCols gz = layout_cols(LMr, dwo, 0);
            if (LM)
                grouped_product(mat64, probs_m, gz, LM->items, LM->nitems, LM->G, LM->ritems, LM->nritems, Wz,
                                LM->gpart, w->W, nullptr, w->mask, 1, s, mf);
            else
                grouped_product(mat64, probs_m, gz, litems, nlitems, L->G, lritems, nlritems, Wz, L->gpart, w->W,
                                nullptr, w->mask, 1, s, mf);
            hipLaunchKernelGGL(k_add_active, egrid, dim3(BT), 0, s, cl, (const double2 *)w->W, Xw, w->st);
        } else {
            hipLaunchKernelGGL(k_xupd<double2>, egrid, dim3(BT), 0, s, cl, m, w->V, w->y, Xw, w->st);
        }
        BIE_HIP(hipGetLastError());
        pull_st();
        std::vector<int> nd(C, 0), cand(C, 0), sampled_met(C, 0);
        bool anyr = false, anyc = false;
        for (int64_t c = 0; c < C; ++c) {
            if (!active[c]) continue;
            hs[c].iters += st[c].jend;
            hs[c].mvps += st[c].jend;
            hs[c].relres_est = st[c].est;
            cand[c] = st[c].est <= o.tol || st[c].brk;
            anyc = anyc || cand[c];
        }
        if (o.crit != BIE_SCC && anyc) {
            // the candidates' sampled residuals (FP64 rows); RSCC accepts on them,
            // CCC confirms them on the full residual below
            sampled_check(cand);
            for (int64_t c = 0; c < C; ++c)
                if (cand[c]) {
                    sampled_met[c] = hs[c].relres_true <= o.tol;
                    if (o.crit == BIE_RSCC && sampled_met[c]) {
                        active[c] = 0;
                        hs[c].converged = 1;
                    }
                }
        }
        for (int64_t c = 0; c < C; ++c) {
            if (!active[c]) continue;
            if (hs[c].mvps < o.max_mvp || cand[c]) {
                nd[c] = 1;   // true residual: the criterion, or the restart
                anyr = true;
            }
        }
        if (anyr) residual_of(nd);
        pull_st();
        for (int64_t c = 0; c < C; ++c) {
            if (!active[c] || !nd[c]) continue;
            const bool decide = o.crit == BIE_SCC ? cand[c] != 0 : (o.crit == BIE_CCC && sampled_met[c]);
            if (decide) {
                if (o.crit == BIE_SCC) hs[c].checks += 1;
                hs[c].relres_true = st[c].rnorm / st[c].bnorm;
                if (hs[c].relres_true <= o.tol) {
                    active[c] = 0;
                    hs[c].converged = 1;
                }
            }
            if (active[c] && st[c].rnorm == 0.0) {
                active[c] = 0;
                hs[c].converged = 1;
                hs[c].relres_true = 0.0;
            }
        }
    }
    // solutions out
    for (int64_t p = 0, c0 = 0; p < P; c0 += Rp[p], ++p)
        if (Rp[p] > 0)
            BIE_HIP(hipMemcpyAsync(Xp[p], Xw + woff[c0], size_t(Rp[p]) * ops[p]->mesh.N * sizeof(double2),
                                   hipMemcpyDeviceToDevice, s));
    BIE_HIP(hipStreamSynchronize(s));
    int status = BIE_OK;
    for (int64_t c = 0; c < C; ++c) {
        if (!hs[c].converged) status = BIE_NOT_CONVERGED;
        if (stats) stats[c] = hs[c];
    }
    return status;
}

void batch_config(int unit, int graph, int mfma)
{
    g_batch.unit = unit;
    g_batch.graph = graph;
    g_batch.mfma = mfma;
}

// The batched solves' grouped product on its own: Y_p = T_p X_p for the
// columns of all operators in one tile launch and one reduce launch, through
// column buffers of the library (inputs copied in, outputs copied out).
void batch_apply(const bie_op *const *ops, int64_t P, const void *const *X, void *const *Y, const int64_t *R,
                 int mat, int unit, int G, hipStream_t s)
{
    if (mat < 0 || mat > 3)
        throw Error(BIE_EINVAL, "mat must be 0 (FP64 tiles), 1 (FP32 tiles), 2 (FP32 tiles on the matrix cores) or "
                                "3 (FP64 tiles on the matrix cores)");
    const bool m64 = mat == 0 || mat == 3, mf = mat >= 2;
    if (unit == 0) unit = 8;
    if (G == 0) G = mf ? 32 : 8;
    if (unit < 1 || unit > 64) throw Error(BIE_EINVAL, "tiles per unit must be 1..64");
    if (G < 1 || G > (mf ? 32 : 4096))
        throw Error(BIE_EINVAL, mf ? "the matrix-core passes take 1..32 columns per item" : "columns per item must be 1..4096");
    std::vector<int32_t> prob;
    std::vector<int64_t> off;
    int64_t nw = 0;
    for (int64_t p = 0; p < P; ++p) {
        const bie_op *op = ops[p];
        if (op->device != ops[0]->device) throw Error(BIE_EINVAL, "all operators on one device");
        if (!(m64 ? op->Z64 : op->Z32))
            throw Error(BIE_EINVAL, m64 ? "operator " + std::to_string(p) + " holds no FP64 matrix"
                                        : "operator " + std::to_string(p) + " holds no FP32 matrix");
        for (int64_t r = 0; r < R[p]; ++r) {
            prob.push_back(int32_t(p));
            off.push_back(nw);
            nw += op->mesh.N;
        }
    }
    const int64_t C = int64_t(prob.size());
    if (C == 0) return;
    auto L = make_layout(ops, P, R, unit, G, m64);
    DevBufs db;
    double2 *Xw = db.get<double2>(size_t(nw)), *Yw = db.get<double2>(size_t(nw));
    int32_t *dprob = db.get<int32_t>(size_t(C));
    int64_t *doff = db.get<int64_t>(size_t(C));
    BIE_HIP(hipMemcpy(dprob, prob.data(), size_t(C) * sizeof(int32_t), hipMemcpyHostToDevice));
    BIE_HIP(hipMemcpy(doff, off.data(), size_t(C) * sizeof(int64_t), hipMemcpyHostToDevice));
    int64_t c = 0;
    for (int64_t p = 0; p < P; ++p) {
        if (R[p] == 0) continue;
        BIE_HIP(hipMemcpyAsync(Xw + off[c], X[p], size_t(R[p]) * ops[p]->mesh.N * sizeof(double2),
                               hipMemcpyDeviceToDevice, s));
        c += R[p];
    }
    const GCols gc{ dprob, doff, doff, L->gpoff, 0 };
    grouped_product(m64, L->probs, gc, L->items, L->nitems, L->G, L->ritems, L->nritems, Xw, L->gpart, Yw, nullptr,
                    nullptr, 1, s, mf);
    c = 0;
    for (int64_t p = 0; p < P; ++p) {
        if (R[p] == 0) continue;
        BIE_HIP(hipMemcpyAsync(Y[p], Yw + off[c], size_t(R[p]) * ops[p]->mesh.N * sizeof(double2),
                               hipMemcpyDeviceToDevice, s));
        c += R[p];
    }
    BIE_HIP(hipStreamSynchronize(s));   // the column buffers are freed on return
}

int batch_unit_chosen(const bie_op *const *ops, int64_t P, const int64_t *R)
{
    std::vector<int> v;
    if (ops[0]->Z64 && tune_get(batch_key(ops, P, R, true), v) && !v.empty()) return v[0];
    if (ops[0]->Z32 && tune_get(batch_key(ops, P, R, false, true), v) && !v.empty()) return v[0];
    if (ops[0]->Z32 && tune_get(batch_key(ops, P, R, false), v) && !v.empty()) return v[0];
    return 0;
}

int solve(const bie_op *op, const void *B, void *X, int64_t R, const bie_solve_opts &o, bie_solve_stat *stats,
          hipStream_t s)
{
    if (op->fast) {
        if (o.method != BIE_GMRES || o.precision != 0 || o.crit != BIE_SCC || o.calderon)
            throw Error(BIE_EINVAL, "the fast operator solves with GMRES, precision 0 and the standard criterion");
        return solve_impl(op, B, X, R, o, stats, s, MAT64, false);
    }
    if (o.precision == 1) {
        if (!op->Z64 || !(op->Z32 || op->Abf))
            throw Error(BIE_EINVAL, "mixed precision needs the FP64 matrix and a low-precision copy "
                                    "(storage BIE_C64 with keep_fp64, or BIE_SPLIT_BF16)");
        if (op->Abf && o.basis == 1) return solve_stream<c32h>(op, B, X, R, o, stats, s, MATBF16);
        if (op->Abf) return solve_stream<float2>(op, B, X, R, o, stats, s, MATBF16);
        return solve_stream<double2>(op, B, X, R, o, stats, s, MAT32);
    }
    if (!op->Z64 && o.crit != BIE_SCC) throw Error(BIE_EINVAL, "the random-sampling criterion needs the FP64 matrix");
    return solve_impl(op, B, X, R, o, stats, s, op->Z64 ? MAT64 : MAT32, false);
}

}  // namespace bie
