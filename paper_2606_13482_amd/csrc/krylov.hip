// Krylov solvers on the device: restarted GMRES(m) and CGNR, with the
// standard and random-sampling convergence criteria.
//
// The paper solves eq:discretizedEFIE "using an iterative solver" (Sec. II)
// and names GMRES, CG and the two criteria only in its acronym list; the
// readings implemented:
//   GMRES(m): Arnoldi with classical Gram-Schmidt applied twice (CGS2),
//     complex Givens rotations kept in FP64 on the device, tolerance relative
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
#include <vector>

#include "bie_internal.hpp"

namespace bie {

void gemv_strided(bool fp64, const void *Z, int64_t N, const void *X, int64_t ldx, void *Y, int64_t ldy,
                  const void *B, int64_t ldb, int64_t R, const int *skip, int64_t sks, bool conj, hipStream_t s);

namespace {

constexpr int BT = 256;          // threads per block
constexpr int EPT = 4;           // elements per thread in vector kernels
constexpr int BE = BT * EPT;     // elements per block
constexpr int MAXM = 128;        // largest restart length

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
    int pad[2];
};
static_assert(sizeof(ColStat) == 96, "ColStat layout");

__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 cmulc(double2 a, double2 b)   // conj(a) * b
{
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

__device__ inline double wsum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
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

// Arnoldi pass 1: h1 = V_{0..j}^H w and ||w||.
__global__ __launch_bounds__(BT) void k_arn_dot1(int64_t N, int m, int j, const double2 *__restrict__ Vall,
                                                 const double2 *__restrict__ Wall, double2 *__restrict__ partall,
                                                 double2 *__restrict__ h1all, unsigned *__restrict__ counters,
                                                 ColStat *__restrict__ st)
{
    const int r = blockIdx.y;
    if (st[r].done) return;
    const unsigned nblk = gridDim.x;
    const int64_t e0 = int64_t(blockIdx.x) * BE;
    const double2 *V = Vall + int64_t(r) * (m + 1) * N;
    const double2 *W = Wall + int64_t(r) * N;
    double2 *part = partall + int64_t(r) * nblk * (m + 2);
    __shared__ double2 sw[BE];
    double nn = 0.0;
    for (int t = threadIdx.x; t < BE; t += BT) {
        const int64_t e = e0 + t;
        const double2 w = e < N ? W[e] : make_double2(0.0, 0.0);
        sw[t] = w;
        nn += w.x * w.x + w.y * w.y;
    }
    __syncthreads();
    chunk_dots(V, N, e0, j + 1, sw, part + int64_t(blockIdx.x) * (m + 2));
    __shared__ double red[BT / 64];
    nn = wsum(nn);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nn;
    __syncthreads();
    if (threadIdx.x == 0) part[int64_t(blockIdx.x) * (m + 2) + m + 1] = make_double2(red[0] + red[1] + red[2] + red[3], 0.0);
    if (!last_block(counters + r, nblk)) return;
    for (int k = threadIdx.x; k <= j + 1; k += BT) {
        const int kk = (k == j + 1) ? m + 1 : k;
        double ar = 0.0, ai = 0.0;
        for (unsigned b = 0; b < nblk; ++b) {
            const double2 p = part[int64_t(b) * (m + 2) + kk];
            ar += p.x;
            ai += p.y;
        }
        if (k <= j) h1all[int64_t(r) * (m + 1) + k] = make_double2(ar, ai);
        else st[r].wnorm0 = sqrt(ar);
    }
}

// Arnoldi pass 2: w -= V h1, then h2 = V^H w; H(:,j) = h1 + h2.
__global__ __launch_bounds__(BT) void k_arn_upd_dot2(int64_t N, int m, int j, const double2 *__restrict__ Vall,
                                                     double2 *__restrict__ Wall, double2 *__restrict__ partall,
                                                     const double2 *__restrict__ h1all, double2 *__restrict__ h2all,
                                                     double2 *__restrict__ Hall, unsigned *__restrict__ counters,
                                                     ColStat *__restrict__ st)
{
    const int r = blockIdx.y;
    if (st[r].done) return;
    const unsigned nblk = gridDim.x;
    const int64_t e0 = int64_t(blockIdx.x) * BE;
    const double2 *V = Vall + int64_t(r) * (m + 1) * N;
    double2 *W = Wall + int64_t(r) * N;
    double2 *part = partall + int64_t(r) * nblk * (m + 2);
    __shared__ double2 sh[MAXM];
    __shared__ double2 sw[BE];
    if (threadIdx.x <= j) sh[threadIdx.x] = h1all[int64_t(r) * (m + 1) + threadIdx.x];
    __syncthreads();
    for (int t = threadIdx.x; t < BE; t += BT) {
        const int64_t e = e0 + t;
        double2 w = make_double2(0.0, 0.0);
        if (e < N) {
            w = W[e];
            for (int k = 0; k <= j; ++k) {
                const double2 p = cmul(V[int64_t(k) * N + e], sh[k]);
                w.x -= p.x;
                w.y -= p.y;
            }
            W[e] = w;
        }
        sw[t] = w;
    }
    __syncthreads();
    chunk_dots(V, N, e0, j + 1, sw, part + int64_t(blockIdx.x) * (m + 2));
    if (!last_block(counters + r, nblk)) return;
    for (int k = threadIdx.x; k <= j; k += BT) {
        double ar = 0.0, ai = 0.0;
        for (unsigned b = 0; b < nblk; ++b) {
            const double2 p = part[int64_t(b) * (m + 2) + k];
            ar += p.x;
            ai += p.y;
        }
        h2all[int64_t(r) * (m + 1) + k] = make_double2(ar, ai);
        const double2 h1 = sh[k];
        Hall[(int64_t(r) * m + j) * (m + 1) + k] = make_double2(h1.x + ar, h1.y + ai);
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

// Arnoldi pass 3: w -= V h2, h_{j+1,j} = ||w||; Givens update of column j.
__global__ __launch_bounds__(BT) void k_arn_upd_norm(int64_t N, int m, int j, double tol,
                                                     const double2 *__restrict__ Vall, double2 *__restrict__ Wall,
                                                     double2 *__restrict__ partall, const double2 *__restrict__ h2all,
                                                     double2 *__restrict__ Hall, double *__restrict__ csall,
                                                     double2 *__restrict__ snall, double2 *__restrict__ gall,
                                                     unsigned *__restrict__ counters, ColStat *__restrict__ st)
{
    const int r = blockIdx.y;
    if (st[r].done) return;
    const unsigned nblk = gridDim.x;
    const int64_t e0 = int64_t(blockIdx.x) * BE;
    const double2 *V = Vall + int64_t(r) * (m + 1) * N;
    double2 *W = Wall + int64_t(r) * N;
    double2 *part = partall + int64_t(r) * nblk * (m + 2);
    __shared__ double2 sh[MAXM];
    if (threadIdx.x <= j) sh[threadIdx.x] = h2all[int64_t(r) * (m + 1) + threadIdx.x];
    __syncthreads();
    double nn = 0.0;
    for (int t = threadIdx.x; t < BE; t += BT) {
        const int64_t e = e0 + t;
        if (e < N) {
            double2 w = W[e];
            for (int k = 0; k <= j; ++k) {
                const double2 p = cmul(V[int64_t(k) * N + e], sh[k]);
                w.x -= p.x;
                w.y -= p.y;
            }
            W[e] = w;
            nn += w.x * w.x + w.y * w.y;
        }
    }
    __shared__ double red[BT / 64];
    nn = wsum(nn);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nn;
    __syncthreads();
    if (threadIdx.x == 0) part[int64_t(blockIdx.x) * (m + 2)] = make_double2(red[0] + red[1] + red[2] + red[3], 0.0);
    if (!last_block(counters + r, nblk)) return;
    if (threadIdx.x != 0) return;
    double s2 = 0.0;
    for (unsigned b = 0; b < nblk; ++b) s2 += part[int64_t(b) * (m + 2)].x;
    const double hn = sqrt(s2);
    ColStat &S = st[r];
    S.hn = hn;
    double2 *H = Hall + (int64_t(r) * m + j) * (m + 1);
    double *cs = csall + int64_t(r) * m;
    double2 *sn = snall + int64_t(r) * m;
    double2 *g = gall + int64_t(r) * (m + 1);
    H[j + 1] = make_double2(hn, 0.0);
    for (int i = 0; i < j; ++i) {
        const double2 a = H[i], b = H[i + 1];
        const double2 sb = cmul(sn[i], b);
        const double2 csa = cmul(make_double2(sn[i].x, -sn[i].y), a);
        H[i] = make_double2(cs[i] * a.x + sb.x, cs[i] * a.y + sb.y);
        H[i + 1] = make_double2(-csa.x + cs[i] * b.x, -csa.y + cs[i] * b.y);
    }
    double c;
    double2 s;
    givens(H[j], H[j + 1], c, s);
    cs[j] = c;
    sn[j] = s;
    const double2 sb = cmul(s, H[j + 1]);
    H[j] = make_double2(c * H[j].x + sb.x, c * H[j].y + sb.y);
    H[j + 1] = make_double2(0.0, 0.0);
    const double2 gj = g[j];
    const double2 t = cmul(make_double2(s.x, -s.y), gj);
    g[j + 1] = make_double2(-t.x, -t.y);
    g[j] = make_double2(c * gj.x, c * gj.y);
    S.est = hypot(g[j + 1].x, g[j + 1].y) / S.bnorm;
    const bool brk = hn <= 64.0 * 2.220446049250313e-16 * S.wnorm0;
    S.jend = j + 1;
    if (brk) S.brk = 1;
    if (S.est <= tol || brk || j + 1 >= S.jcap) S.done = 1;
}

// v_{j+1} = w / h_{j+1,j}
__global__ __launch_bounds__(BT) void k_arn_normalize(int64_t N, int m, int j, double2 *__restrict__ Vall,
                                                      const double2 *__restrict__ Wall, const ColStat *__restrict__ st)
{
    const int r = blockIdx.y;
    if (st[r].done) return;
    const double inv = 1.0 / st[r].hn;
    const double2 *W = Wall + int64_t(r) * N;
    double2 *v = Vall + (int64_t(r) * (m + 1) + j + 1) * N;
    for (int64_t e = int64_t(blockIdx.x) * BT + threadIdx.x; e < N; e += int64_t(gridDim.x) * BT) {
        const double2 w = W[e];
        v[e] = make_double2(w.x * inv, w.y * inv);
    }
}

// Upper-triangular solve H y = g for the iterations of the cycle (one thread per column).
__global__ void k_lsq(int R, int m, const double2 *__restrict__ Hall, const double2 *__restrict__ gall,
                      double2 *__restrict__ yall, const ColStat *__restrict__ st)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R || !st[r].active) return;
    const int je = st[r].jend;
    const double2 *g = gall + int64_t(r) * (m + 1);
    double2 *y = yall + int64_t(r) * m;
    for (int i = je - 1; i >= 0; --i) {
        double2 acc = g[i];
        for (int k = i + 1; k < je; ++k) {
            const double2 p = cmul(Hall[(int64_t(r) * m + k) * (m + 1) + i], y[k]);
            acc.x -= p.x;
            acc.y -= p.y;
        }
        const double2 d = Hall[(int64_t(r) * m + i) * (m + 1) + i];
        const double dd = d.x * d.x + d.y * d.y;
        y[i] = make_double2((acc.x * d.x + acc.y * d.y) / dd, (acc.y * d.x - acc.x * d.y) / dd);
    }
}

// x += V_{0..jend-1} y
__global__ __launch_bounds__(BT) void k_xupd(int64_t N, int m, const double2 *__restrict__ Vall,
                                             const double2 *__restrict__ yall, double2 *__restrict__ X,
                                             const ColStat *__restrict__ st)
{
    const int r = blockIdx.y;
    if (!st[r].active) return;
    const int je = st[r].jend;
    __shared__ double2 sy[MAXM];
    if (threadIdx.x < je) sy[threadIdx.x] = yall[int64_t(r) * m + threadIdx.x];
    __syncthreads();
    const double2 *V = Vall + int64_t(r) * (m + 1) * N;
    for (int64_t e = int64_t(blockIdx.x) * BT + threadIdx.x; e < N; e += int64_t(gridDim.x) * BT) {
        double2 x = X[int64_t(r) * N + e];
        for (int k = 0; k < je; ++k) {
            const double2 p = cmul(V[int64_t(k) * N + e], sy[k]);
            x.x += p.x;
            x.y += p.y;
        }
        X[int64_t(r) * N + e] = x;
    }
}

// ||v||^2 per column with last-block finish; writes sqrt into the field at `off`.
__global__ __launch_bounds__(BT) void k_norm(int64_t N, const double2 *__restrict__ Vb, int64_t ld,
                                             double *__restrict__ part, unsigned *__restrict__ counters,
                                             ColStat *__restrict__ st, int field, const int *__restrict__ mask)
{
    const int r = blockIdx.y;
    if (mask && !mask[r]) return;
    const unsigned nblk = gridDim.x;
    const double2 *v = Vb + int64_t(r) * ld;
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

// Sampled residual rows (RSCC): one wave per sampled row.
__global__ __launch_bounds__(BT) void k_rscc_rows(int64_t N, int S, const double2 *__restrict__ Z,
                                                  const double2 *__restrict__ B, const double2 *__restrict__ X,
                                                  const int64_t *__restrict__ rows, double *__restrict__ out,
                                                  const int *__restrict__ mask)
{
    const int r = blockIdx.y;
    if (!mask[r]) return;
    const int lane = threadIdx.x & 63;
    const int s = blockIdx.x * (BT / 64) + (threadIdx.x >> 6);
    if (s >= S) return;
    const int64_t i = rows[int64_t(r) * S + s];
    const double2 *z = Z + i * N;
    const double2 *x = X + int64_t(r) * N;
    double ar = 0.0, ai = 0.0;
    for (int64_t c = lane; c < N; c += 64) {
        const double2 p = cmul(z[c], x[c]);
        ar += p.x;
        ai += p.y;
    }
    ar = wsum(ar);
    ai = wsum(ai);
    if (lane == 0) {
        const double2 b = B[int64_t(r) * N + i];
        const double dr = b.x - ar, di = b.y - ai;
        out[int64_t(r) * S + s] = dr * dr + di * di;
    }
}

// Start a cycle from the residual: v0 = res/||res||, g = (||res||, 0, ...).
__global__ __launch_bounds__(BT) void k_restart(int64_t N, int m, const double2 *__restrict__ Res,
                                                double2 *__restrict__ Vall, double2 *__restrict__ gall,
                                                ColStat *__restrict__ st, const int *__restrict__ mask)
{
    const int r = blockIdx.y;
    if (!mask[r]) return;
    const double beta = st[r].rnorm;
    const double inv = 1.0 / beta;
    double2 *v = Vall + int64_t(r) * (m + 1) * N;
    for (int64_t e = int64_t(blockIdx.x) * BT + threadIdx.x; e < N; e += int64_t(gridDim.x) * BT) {
        const double2 w = Res[int64_t(r) * N + e];
        v[e] = make_double2(w.x * inv, w.y * inv);
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
    double2 *h1 = nullptr, *h2 = nullptr, *part = nullptr;
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

// Solve driver shared by GMRES and CGNR (FP64 vectors, FP64 or FP32 matrix).
int solve(const bie_op *opc, const void *Bv, void *Xv, int64_t R, const bie_solve_opts &o, bie_solve_stat *stats,
          hipStream_t s)
{
    bie_op *op = const_cast<bie_op *>(opc);
    const int64_t N = op->mesh.N;
    const bool fp64 = op->Z64 != nullptr;
    const void *Z = fp64 ? op->Z64 : op->Z32;
    const int m = o.method == BIE_GMRES ? o.restart : 1;
    Workspace *w = get_ws(op, R, m);
    const double2 *B = static_cast<const double2 *>(Bv);
    double2 *X = static_cast<double2 *>(Xv);
    std::vector<bie_solve_stat> hs(R);
    for (auto &h : hs) h = bie_solve_stat{ 0, 0, NAN, NAN, 0, 0 };
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
    hipLaunchKernelGGL(k_norm, vgrid, dim3(BT), 0, s, N, B, N, w->dpart, w->counters, w->st, field_bnorm,
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
        gemv_strided(fp64, Z, N, X, N, w->Res, N, B, N, R, dskip, 1, false, s);
        // k_norm mask: need
        push_skip(need);
        hipLaunchKernelGGL(k_norm, vgrid, dim3(BT), 0, s, N, w->Res, N, w->dpart, w->counters, w->st, field_rnorm,
                           (const int *)dskip);
        BIE_HIP(hipGetLastError());
        for (int64_t r = 0; r < R; ++r)
            if (need[r]) hs[r].mvps += 1;
    };
    auto criterion = [&](const std::vector<int> &cand, std::vector<int> &met) {
        // returns per-column criterion value in hs[r].relres_true; met[r] set
        std::vector<int> need(R, 0);
        bool any = false;
        for (int64_t r = 0; r < R; ++r) { met[r] = 0; if (cand[r]) { need[r] = 1; any = true; } }
        if (!any) return;
        if (o.crit == BIE_SCC) {
            full_residual(need);
            pull_st();
            for (int64_t r = 0; r < R; ++r)
                if (need[r]) {
                    const double v = st[r].rnorm / st[r].bnorm;
                    hs[r].relres_true = v;
                    hs[r].checks += 1;
                    met[r] = v <= o.tol;
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
            if (fp64) {
                hipLaunchKernelGGL(k_rscc_rows, dim3(unsigned((S + 3) / 4), unsigned(R)), dim3(BT), 0, s, N, int(S),
                                   (const double2 *)Z, B, X, w->rows, w->rs, dskip);
            } else {
                throw Error(BIE_EINVAL, "random-sampling criterion needs the FP64 matrix");
            }
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
        }
    };

    std::vector<int> need(R, 0), met(R, 0);
    if (o.use_x0) {
        for (int64_t r = 0; r < R; ++r) need[r] = active[r];
        full_residual(need);
    } else {
        for (int64_t r = 0; r < R; ++r)
            if (active[r])
                hipLaunchKernelGGL(k_copy, dim3(64), dim3(256), 0, s, N, B + r * N, w->Res + r * N);
        for (int64_t r = 0; r < R; ++r) need[r] = active[r];
        push_skip(need);
        hipLaunchKernelGGL(k_norm, vgrid, dim3(BT), 0, s, N, w->Res, N, w->dpart, w->counters, w->st, field_rnorm,
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
            hipLaunchKernelGGL(k_restart, egrid, dim3(BT), 0, s, N, m, w->Res, w->V, w->g, w->st, (const int *)dskip);
            BIE_HIP(hipGetLastError());
            int jmax = 0;
            for (int64_t r = 0; r < R; ++r)
                if (active[r]) jmax = std::max(jmax, st[r].jcap);
            for (int j = 0; j < jmax; ++j) {
                // skip array for the product = done flags, taken from the device status
                gemv_strided(fp64, Z, N, w->V + int64_t(j) * N, int64_t(m + 1) * N, w->W, N, nullptr, 0, R,
                             done_flags, done_stride, false, s);
                hipLaunchKernelGGL(k_arn_dot1, vgrid, dim3(BT), 0, s, N, m, j, w->V, w->W, w->part, w->h1,
                                   w->counters, w->st);
                hipLaunchKernelGGL(k_arn_upd_dot2, vgrid, dim3(BT), 0, s, N, m, j, w->V, w->W, w->part, w->h1,
                                   w->h2, w->H, w->counters, w->st);
                hipLaunchKernelGGL(k_arn_upd_norm, vgrid, dim3(BT), 0, s, N, m, j, o.tol, w->V, w->W, w->part,
                                   w->h2, w->H, w->cs, w->sn, w->g, w->counters, w->st);
                hipLaunchKernelGGL(k_arn_normalize, egrid, dim3(BT), 0, s, N, m, j, w->V, w->W, w->st);
                BIE_HIP(hipGetLastError());
            }
            hipLaunchKernelGGL(k_lsq, dim3(unsigned((R + 63) / 64)), dim3(64), 0, s, int(R), m, w->H, w->g, w->y, w->st);
            hipLaunchKernelGGL(k_xupd, egrid, dim3(BT), 0, s, N, m, w->V, w->y, X, w->st);
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
                if (active[r] && hs[r].mvps < o.max_mvp && !(o.crit == BIE_SCC && cand[r])) { nd[r] = 1; anyr = true; }
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
            gemv_strided(fp64, Z, N, w->Res, N, Zv, N, nullptr, 0, R, dskip, 1, true, s);
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
                gemv_strided(fp64, Z, N, Pv, N, w->W, N, nullptr, 0, R, done_flags, done_stride, false, s);
                hipLaunchKernelGGL(k_cg_alpha, vgrid, dim3(BT), 0, s, N, w->W, w->dpart, w->counters, w->st);
                hipLaunchKernelGGL(k_cg_step, vgrid, dim3(BT), 0, s, N, o.tol, Pv, w->W, X, w->Res, w->dpart,
                                   w->counters, w->st, w->iters);
                gemv_strided(fp64, Z, N, w->Res, N, Zv, N, nullptr, 0, R, done_flags, done_stride, true, s);
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
                if (o.crit != BIE_SCC) full_residual(again);
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

}  // namespace bie
