// Learned warm start: POD basis of solutions the method computed, and a small
// MLP that maps the incidence (direction, polarisation flag) to POD
// coefficients; trained and evaluated with the kernels below.
//
// POD basis: the leading K left singular vectors of the snapshot matrix
// A = [x_1 ... x_S] (N x S), by a randomised range finder with power
// iterations (Halko, Martinsson & Tropp, SIAM Rev. 53, 2011):
//   Y = A Omega (N x L, L = K + p), Y <- A (A^H Y) q times with CholeskyQR2
//   re-orthonormalisation, Q = orth(Y), B = Q^H A, B B^H = W S^2 W^H,
//   U = Q W(:, 1..K).
// The dense products are two complex FP64 kernels (linear combination of
// vectors, inner products over N); the L x L Cholesky and Hermitian Jacobi
// eigensolver run on the host (L ~ 300).
//
// MLP: inputs (d_x, d_y, d_z, s), Dense(4->H) tanh, Dense(H->H) tanh,
// Dense(H->2K) linear; outputs are Re and Im of the K coefficients divided by
// one global RMS scale.  FP32 weights and arithmetic, loss = mean squared
// error, Adam (0.9, 0.999, 1e-8) with a cosine learning rate lr_max -> lr_min.
// Glorot-uniform initial weights and the per-epoch shuffles come from
// SplitMix64 (published generator), so an independent implementation can
// reproduce them exactly.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <memory>
#include <vector>

#include "bie_internal.hpp"

namespace bie {

namespace {

struct SM64 {
    uint64_t s;
    explicit SM64(uint64_t seed) : s(seed) {}
    uint64_t next()
    {
        s += 0x9E3779B97F4A7C15ULL;
        uint64_t z = s;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        return z ^ (z >> 31);
    }
    double uniform() { return double(next() >> 11) * (1.0 / 9007199254740992.0); }   // [0, 1)
    uint64_t below(uint64_t n) { return uint64_t((unsigned __int128)next() * n >> 64); }
};

// ----------------------------------------------------------------------------- complex FP64 kernels
// Out[p][n] = sum_s Coef[p][s] In[s][n]   (Out P x N, Coef P x S row-major, In S x N)
constexpr int LP = 32, LS = 32;
__global__ __launch_bounds__(256) void k_lincomb(int64_t P, int64_t S, int64_t N, const double2 *__restrict__ Coef,
                                                 const double2 *__restrict__ In, double2 *__restrict__ Out)
{
    __shared__ double2 sc[LP][LS];
    const int64_t p0 = int64_t(blockIdx.y) * LP;
    const int64_t n = int64_t(blockIdx.x) * 256 + threadIdx.x;
    double2 acc[LP];
#pragma unroll
    for (int i = 0; i < LP; ++i) acc[i] = make_double2(0.0, 0.0);
    for (int64_t s0 = 0; s0 < S; s0 += LS) {
        __syncthreads();
        for (int e = threadIdx.x; e < LP * LS; e += 256) {
            const int i = e / LS, j = e % LS;
            sc[i][j] = (p0 + i < P && s0 + j < S) ? Coef[(p0 + i) * S + s0 + j] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        if (n < N) {
            for (int j = 0; j < LS && s0 + j < S; ++j) {
                const double2 x = In[(s0 + j) * N + n];
#pragma unroll
                for (int i = 0; i < LP; ++i) {
                    const double2 c = sc[i][j];
                    acc[i].x += c.x * x.x - c.y * x.y;
                    acc[i].y += c.x * x.y + c.y * x.x;
                }
            }
        }
    }
    if (n < N)
        for (int i = 0; i < LP; ++i)
            if (p0 + i < P) Out[(p0 + i) * N + n] = acc[i];
}

// G[p][s] = sum_n conj(A[p][n]) B[s][n]   (A P x N, B S x N, G P x S); 32 x 32 tile per block
__global__ __launch_bounds__(256) void k_inner(int64_t P, int64_t S, int64_t N, const double2 *__restrict__ A,
                                               const double2 *__restrict__ B, double2 *__restrict__ G)
{
    __shared__ double2 sa[32][33], sb[32][33];
    const int64_t p0 = int64_t(blockIdx.y) * 32, s0 = int64_t(blockIdx.x) * 32;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;   // ty: 0..7, 4 outputs per thread
    double2 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = make_double2(0.0, 0.0);
    for (int64_t n0 = 0; n0 < N; n0 += 32) {
        __syncthreads();
        for (int e = threadIdx.x; e < 32 * 32; e += 256) {
            const int i = e / 32, j = e % 32;
            sa[i][j] = (p0 + i < P && n0 + j < N) ? A[(p0 + i) * N + n0 + j] : make_double2(0.0, 0.0);
            sb[i][j] = (s0 + i < S && n0 + j < N) ? B[(s0 + i) * N + n0 + j] : make_double2(0.0, 0.0);
        }
        __syncthreads();
#pragma unroll 4
        for (int j = 0; j < 32; ++j) {
            const double2 b = sb[tx][j];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double2 a = sa[ty + 8 * q][j];
                acc[q].x += a.x * b.x + a.y * b.y;
                acc[q].y += a.x * b.y - a.y * b.x;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t p = p0 + ty + 8 * q, s = s0 + tx;
        if (p < P && s < S) G[p * S + s] = acc[q];
    }
}

// ----------------------------------------------------------------------------- FP32 MLP kernels
// C[m][n] = epi(sum_k opA(A)[m][k] opB(B)[k][n]) on the FP32 matrix cores
// (v_mfma_f32_32x32x2f32: A[i][k] in lane i + 32 k, B[k][j] in lane j + 32 k,
// value q of lane l at row 8 (q / 4) + 4 (l / 32) + q % 4, column l % 32).
// opA(A)[m][k] = TA ? A[k][m] : A[m][k] (lda = row length of A as stored), the
// same for B.  One block computes one 32 x 32 tile of C; its four waves take
// interleaved K chunks of 32 (staged in LDS, loads coalesced along the stored
// rows) and their partial tiles are summed in LDS in fixed order.
// Epilogues: EPI_STORE C = acc; EPI_BIAS_TANH C = tanh(acc + bias[n]);
// EPI_BIAS C = acc + bias[n]; EPI_TANH_BACK C = acc (1 - X[m][n]^2) with X the
// stored tanh output of the layer (the backward step through tanh).
typedef float f32x16 __attribute__((ext_vector_type(16)));
enum { EPI_STORE = 0, EPI_BIAS_TANH = 1, EPI_BIAS = 2, EPI_TANH_BACK = 3 };

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_sgemm_mf(int M, int N, int K, const float *__restrict__ A, int lda,
                                                  const float *__restrict__ Bm, int ldb, float *__restrict__ C, int ldc,
                                                  int epi, const float *__restrict__ bias, const float *__restrict__ X)
{
    __shared__ float As[4][32][33];   // per wave: [k][m] of its K chunk
    __shared__ float Bs[4][32][33];   // per wave: [k][n]
    __shared__ float red[3][16][64];  // partial tiles of waves 1..3
    const int m0 = blockIdx.y * 32, n0 = blockIdx.x * 32;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    f32x16 acc;
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.f;
    const int nit = (K + 127) / 128;
    // the wave's 32 x 32 chunks of A and B for one iteration, all 32 loads of a
    // lane issued together (element e = lane + 64 j: e / 32 across, e % 32
    // along the stored row); the next iteration's are loaded during the
    // current one's products
    float ra[16], rb[16];
    auto load = [&](int it) {
        const int kc = it * 128 + w * 32;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int e = lane + 64 * j, hi = e >> 5, lo = e & 31;
            if (TA) ra[j] = (m0 + lo < M && kc + hi < K) ? A[int64_t(kc + hi) * lda + m0 + lo] : 0.f;
            else ra[j] = (m0 + hi < M && kc + lo < K) ? A[int64_t(m0 + hi) * lda + kc + lo] : 0.f;
            if (TB) rb[j] = (n0 + hi < N && kc + lo < K) ? Bm[int64_t(n0 + hi) * ldb + kc + lo] : 0.f;
            else rb[j] = (n0 + lo < N && kc + hi < K) ? Bm[int64_t(kc + hi) * ldb + n0 + lo] : 0.f;
        }
    };
    load(0);
    for (int it = 0; it < nit; ++it) {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int e = lane + 64 * j, hi = e >> 5, lo = e & 31;
            if (TA) As[w][hi][lo] = ra[j];
            else As[w][lo][hi] = ra[j];
            if (TB) Bs[w][lo][hi] = rb[j];
            else Bs[w][hi][lo] = rb[j];
        }
        __syncthreads();
        if (it + 1 < nit) load(it + 1);
        const int i = lane & 31, h = lane >> 5;
#pragma unroll
        for (int kk = 0; kk < 32; kk += 2)
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(As[w][kk + h][i], Bs[w][kk + h][i], acc, 0, 0, 0);
        __syncthreads();
    }
    if (w > 0)
#pragma unroll
        for (int q = 0; q < 16; ++q) red[w - 1][q][lane] = acc[q];
    __syncthreads();
    if (w != 0) return;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const float v = ((acc[q] + red[0][q][lane]) + red[1][q][lane]) + red[2][q][lane];
        const int m = m0 + 8 * (q / 4) + 4 * (lane / 32) + q % 4, n = n0 + (lane & 31);
        if (m >= M || n >= N) continue;
        float o = v;
        if (epi == EPI_BIAS_TANH) o = tanhf(v + bias[n]);
        else if (epi == EPI_BIAS) o = v + bias[n];
        else if (epi == EPI_TANH_BACK) {
            const float a = X[int64_t(m) * ldc + n];
            o = v * (1.f - a * a);
        }
        C[int64_t(m) * ldc + n] = o;
    }
}

// loss partials and dL/dy = 2 (y - t) / (B O)
__global__ void k_mse(int n, const float *__restrict__ y, const float *__restrict__ t, float *__restrict__ g,
                      float inv, double *__restrict__ part)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float d = y[i] - t[i];
        g[i] = 2.f * d * inv;
        s += double(d) * double(d);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (int(threadIdx.x) < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// db[o] = sum_b dZ[b][o]: 64 columns per block of 16 waves, wave v summing the
// rows b = v, v + 16, ... (all its loads issued together), the 16 partial sums
// of a column then added in a fixed order
__global__ __launch_bounds__(1024) void k_colsum(int Bn, int O, const float *__restrict__ dZ, float *__restrict__ db)
{
    __shared__ float red[16][64];
    const int lane = threadIdx.x & 63, v = threadIdx.x >> 6;
    const int o = blockIdx.x * 64 + lane;
    float s = 0.f;
    if (o < O) {
        float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
        int b = v;
        for (; b + 48 < Bn; b += 64) {
            p0 += dZ[int64_t(b) * O + o];
            p1 += dZ[int64_t(b + 16) * O + o];
            p2 += dZ[int64_t(b + 32) * O + o];
            p3 += dZ[int64_t(b + 48) * O + o];
        }
        for (; b < Bn; b += 16) p0 += dZ[int64_t(b) * O + o];
        s = (p0 + p1) + (p2 + p3);
    }
    red[v][lane] = s;
    __syncthreads();
    if (v == 0 && o < O) {
        float a = 0.f;
#pragma unroll
        for (int u = 0; u < 16; ++u) a += red[u][lane];
        db[o] = a;
    }
}

__global__ void k_adam(int n, float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Linear-in-polarisation model: the network gives three coefficient sets
// f_c (c = x, y, z; each 2K reals: Re then Im) and the coefficients for
// polarisation e are y = sum_c e_c f_c.
__global__ void k_pol_combine(int B, int K2, const float *__restrict__ net, const float *__restrict__ E,
                              float *__restrict__ y)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * K2) return;
    const int b = i / K2, k = i % K2;
    const float *f = net + int64_t(b) * 3 * K2;
    y[i] = E[b * 3] * f[k] + E[b * 3 + 1] * f[K2 + k] + E[b * 3 + 2] * f[2 * K2 + k];
}
__global__ void k_pol_combine_back(int B, int K2, const float *__restrict__ dy, const float *__restrict__ E,
                                   float *__restrict__ dnet)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * 3 * K2) return;
    const int b = i / (3 * K2), r = i % (3 * K2), c = r / K2, k = r % K2;
    dnet[i] = E[b * 3 + c] * dy[b * K2 + k];
}

// coefficients from the network output: c[r][k] = scale (out[r][k] + j out[r][K + k])
__global__ void k_out_to_coef(int R, int K, const float *__restrict__ out, double scale, double2 *__restrict__ c)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= R * K) return;
    const int r = i / K, k = i % K;
    c[i] = make_double2(scale * out[r * 2 * K + k], scale * out[r * 2 * K + K + k]);
}

// targets t[s][k] = Re(C[k][s]) / scale, t[s][K + k] = Im(C[k][s]) / scale   (C = U^H X, K x S)
__global__ void k_targets(int S, int K, const double2 *__restrict__ C, double inv, float *__restrict__ t)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S * K) return;
    const int s = i / K, k = i % K;
    const double2 c = C[int64_t(k) * S + s];
    t[int64_t(s) * 2 * K + k] = float(c.x * inv);
    t[int64_t(s) * 2 * K + K + k] = float(c.y * inv);
}

// batch gather: in[r] = F[perm[b0 + r]], tgt[r] = T[perm[b0 + r]], pol[r] = E[perm[b0 + r]]
__global__ void k_gather(int B, int O, const int64_t *__restrict__ perm, int64_t b0, const float *__restrict__ F,
                         const float *__restrict__ Tg, const float *__restrict__ E, float *__restrict__ in,
                         float *__restrict__ tgt, float *__restrict__ pol)
{
    const int r = blockIdx.x;
    const int64_t i = perm[b0 + r];
    for (int c = threadIdx.x; c < O; c += blockDim.x) tgt[int64_t(r) * O + c] = Tg[i * O + c];
    if (threadIdx.x < 4) in[r * 4 + threadIdx.x] = F[i * 4 + threadIdx.x];
    if (E && threadIdx.x < 3) pol[r * 3 + threadIdx.x] = E[i * 3 + threadIdx.x];
}

// squared norms of R complex vectors (one block per vector, fixed reduction tree)
__global__ __launch_bounds__(256) void k_sqnorm(int64_t N, const double2 *__restrict__ v, double *__restrict__ out)
{
    const int64_t r = blockIdx.x;
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < N; i += 256) a += v[r * N + i].x * v[r * N + i].x + v[r * N + i].y * v[r * N + i].y;
    __shared__ double red[256];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (int(threadIdx.x) < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[r] = red[0];
}

template <typename T>
T *dmalloc(size_t n)
{
    void *p = nullptr;
    BIE_HIP(hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)));
    return static_cast<T *>(p);
}

void lincomb(int64_t P, int64_t S, int64_t N, const double2 *Coef, const double2 *In, double2 *Out, hipStream_t s)
{
    const dim3 grid(unsigned((N + 255) / 256), unsigned((P + LP - 1) / LP));
    hipLaunchKernelGGL(k_lincomb, grid, dim3(256), 0, s, P, S, N, Coef, In, Out);
    BIE_HIP(hipGetLastError());
}

void inner(int64_t P, int64_t S, int64_t N, const double2 *A, const double2 *B, double2 *G, hipStream_t s)
{
    const dim3 grid(unsigned((S + 31) / 32), unsigned((P + 31) / 32));
    hipLaunchKernelGGL(k_inner, grid, dim3(256), 0, s, P, S, N, A, B, G);
    BIE_HIP(hipGetLastError());
}

template <bool TA, bool TB>
void sgemm(int M, int N, int K, const float *A, int lda, const float *B, int ldb, float *C, int ldc, hipStream_t s,
           int epi = EPI_STORE, const float *bias = nullptr, const float *X = nullptr)
{
    const dim3 grid(unsigned((N + 31) / 32), unsigned((M + 31) / 32));
    hipLaunchKernelGGL((k_sgemm_mf<TA, TB>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, epi, bias, X);
    BIE_HIP(hipGetLastError());
}

using cd = std::complex<double>;

// Host: Cholesky G = R^H R of an L x L Hermitian positive definite matrix; returns R^{-1} (upper).
std::vector<cd> chol_inv_upper(const std::vector<cd> &G, int L)
{
    std::vector<cd> Rm(size_t(L) * L, 0.0);
    for (int j = 0; j < L; ++j) {
        cd d = G[size_t(j) * L + j];
        for (int k = 0; k < j; ++k) d -= std::conj(Rm[size_t(k) * L + j]) * Rm[size_t(k) * L + j];
        double dr = d.real();
        if (!(dr > 0.0)) throw Error(BIE_ENUMERIC, "snapshot basis is rank deficient (Cholesky)");
        const double rjj = std::sqrt(dr);
        Rm[size_t(j) * L + j] = rjj;
        for (int i = j + 1; i < L; ++i) {
            cd a = G[size_t(j) * L + i];
            for (int k = 0; k < j; ++k) a -= std::conj(Rm[size_t(k) * L + j]) * Rm[size_t(k) * L + i];
            Rm[size_t(j) * L + i] = a / rjj;
        }
    }
    // inverse of the upper-triangular R by back substitution
    std::vector<cd> Ri(size_t(L) * L, 0.0);
    for (int c = 0; c < L; ++c) {
        for (int i = c; i >= 0; --i) {
            cd a = (i == c) ? cd(1.0) : cd(0.0);
            for (int k = i + 1; k <= c; ++k) a -= Rm[size_t(i) * L + k] * Ri[size_t(k) * L + c];
            Ri[size_t(i) * L + c] = a / Rm[size_t(i) * L + i];
        }
    }
    return Ri;
}

// Host: cyclic Jacobi eigen-decomposition of a Hermitian L x L matrix (complex
// rotations); returns eigenvalues (descending) and eigenvectors as columns.
void jacobi_eig(std::vector<cd> A, int L, std::vector<double> &w, std::vector<cd> &V)
{
    V.assign(size_t(L) * L, 0.0);
    for (int i = 0; i < L; ++i) V[size_t(i) * L + i] = 1.0;
    auto at = [&](int i, int j) -> cd & { return A[size_t(i) * L + j]; };
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < L; ++i)
            for (int j = 0; j < L; ++j) {
                const double a = std::norm(at(i, j));
                tot += a;
                if (i != j) off += a;
            }
        if (off <= 1e-30 * tot) break;
        for (int p = 0; p < L - 1; ++p)
            for (int q = p + 1; q < L; ++q) {
                const cd apq = at(p, q);
                const double ab = std::abs(apq);
                if (ab < 1e-300) continue;
                const double app = at(p, p).real(), aqq = at(q, q).real();
                // rotation zeroing A(p,q): with apq = |apq| e^{i phi}
                const cd ph = apq / ab;
                const double tau = (aqq - app) / (2.0 * ab);
                const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), sn = t * c;
                // columns: A' = A J with J = [[c, s ph], [-s conj(ph), c]] acting on (p, q)
                for (int k = 0; k < L; ++k) {
                    const cd akp = at(k, p), akq = at(k, q);
                    at(k, p) = c * akp - sn * std::conj(ph) * akq;
                    at(k, q) = sn * ph * akp + c * akq;
                }
                for (int k = 0; k < L; ++k) {
                    const cd apk = at(p, k), aqk = at(q, k);
                    at(p, k) = c * apk - sn * ph * aqk;
                    at(q, k) = sn * std::conj(ph) * apk + c * aqk;
                }
                at(p, q) = 0.0;
                at(q, p) = 0.0;
                for (int k = 0; k < L; ++k) {
                    const cd vkp = V[size_t(k) * L + p], vkq = V[size_t(k) * L + q];
                    V[size_t(k) * L + p] = c * vkp - sn * std::conj(ph) * vkq;
                    V[size_t(k) * L + q] = sn * ph * vkp + c * vkq;
                }
            }
    }
    std::vector<int> idx(L);
    for (int i = 0; i < L; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return at(a, a).real() > at(b, b).real(); });
    std::vector<cd> Vs(size_t(L) * L);
    w.resize(L);
    for (int c = 0; c < L; ++c) {
        w[c] = at(idx[c], idx[c]).real();
        for (int r = 0; r < L; ++r) Vs[size_t(r) * L + c] = V[size_t(r) * L + idx[c]];
    }
    V.swap(Vs);
}

}  // namespace

}  // namespace bie

// ----------------------------------------------------------------------------- warm-start object
struct bie_ws {
    const bie_op *op = nullptr;
    int K = 0, H = 0, O = 0;            // O: network outputs (2K, or 6K for the linear-in-polarisation model)
    int pmodel = 0;                     // 0: inputs (d, s); 1: inputs d, outputs linear in the polarisation
    double scale = 1.0, final_loss = NAN;
    std::vector<double> sigma;          // POD singular values (descending)
    double2 *U = nullptr;               // K x N
    float *params = nullptr;            // W1 (H x 4), b1, W2 (H x H), b2, W3 (O x H), b3
    size_t nparams = 0;
    size_t off[6] = { 0 };
    // training / evaluation scratch
    float *grad = nullptr, *am = nullptr, *av = nullptr;
    int cap_batch = 0;
    float *in = nullptr, *a1 = nullptr, *a2 = nullptr, *y = nullptr, *dy = nullptr,
          *d2 = nullptr, *d1 = nullptr, *tgt = nullptr, *pol = nullptr, *yc = nullptr, *dyc = nullptr;
    double *lpart = nullptr;
    // prediction scratch, grown on demand: coefficients (R x K) and, for the
    // fallback, residuals (R x N) and squared norms (2R)
    double2 *coef = nullptr, *res = nullptr;
    double *nr = nullptr;
    int64_t cap_coef = 0, cap_res = 0;
    ~bie_ws()
    {
        for (void *p : { (void *)U, (void *)params, (void *)grad, (void *)am, (void *)av, (void *)in,
                         (void *)a1, (void *)a2, (void *)y, (void *)dy, (void *)d2, (void *)d1, (void *)tgt,
                         (void *)lpart, (void *)pol, (void *)yc, (void *)dyc, (void *)coef, (void *)res, (void *)nr })
            if (p) (void)hipFree(p);
    }
};

namespace bie {

namespace {

void ws_layout(bie_ws *w)
{
    const size_t H = w->H, O = w->O;
    w->off[0] = 0;                 // W1 H x 4
    w->off[1] = w->off[0] + H * 4; // b1
    w->off[2] = w->off[1] + H;     // W2 H x H
    w->off[3] = w->off[2] + H * H; // b2
    w->off[4] = w->off[3] + H;     // W3 O x H
    w->off[5] = w->off[4] + O * H; // b3
    w->nparams = w->off[5] + O;
}

void ws_alloc_params(bie_ws *w)
{
    ws_layout(w);
    w->params = dmalloc<float>(w->nparams);
    w->grad = dmalloc<float>(w->nparams);
    w->am = dmalloc<float>(w->nparams);
    w->av = dmalloc<float>(w->nparams);
}

void ws_batch_scratch(bie_ws *w, int B)
{
    if (w->cap_batch >= B) return;
    for (float **p : { &w->in, &w->a1, &w->a2, &w->y, &w->dy, &w->d2, &w->d1, &w->tgt, &w->pol,
                       &w->yc, &w->dyc })
        if (*p) { (void)hipFree(*p); *p = nullptr; }
    if (w->lpart) { (void)hipFree(w->lpart); w->lpart = nullptr; }
    const size_t H = w->H, O = w->O;
    w->in = dmalloc<float>(size_t(B) * 4);
    w->a1 = dmalloc<float>(size_t(B) * H);
    w->a2 = dmalloc<float>(size_t(B) * H);
    w->y = dmalloc<float>(size_t(B) * O);
    w->dy = dmalloc<float>(size_t(B) * O);
    w->d2 = dmalloc<float>(size_t(B) * H);
    w->d1 = dmalloc<float>(size_t(B) * H);
    w->tgt = dmalloc<float>(size_t(B) * O);
    w->pol = dmalloc<float>(size_t(B) * 3);
    w->yc = dmalloc<float>(size_t(B) * 2 * w->K);
    w->dyc = dmalloc<float>(size_t(B) * 2 * w->K);
    w->lpart = dmalloc<double>(64);
    w->cap_batch = B;
}

// forward for B inputs already in w->in; output in w->y
void mlp_forward(bie_ws *w, int B, hipStream_t s)
{
    const int H = w->H, O = w->O;
    float *P = w->params;
    sgemm<false, true>(B, H, 4, w->in, 4, P + w->off[0], 4, w->a1, H, s, EPI_BIAS_TANH, P + w->off[1]);
    sgemm<false, true>(B, H, H, w->a1, H, P + w->off[2], H, w->a2, H, s, EPI_BIAS_TANH, P + w->off[3]);
    sgemm<false, true>(B, O, H, w->a2, H, P + w->off[4], H, w->y, O, s, EPI_BIAS, P + w->off[5]);
}

// loss partials (w->lpart[0..nb)) and gradient of the mean squared error into
// w->grad.  combine: the loss is on y = sum_c e_c f_c against 2K targets
// (linear-in-polarisation model); otherwise on the raw outputs.
int mlp_backward(bie_ws *w, int B, hipStream_t s, bool combine = false)
{
    const int H = w->H, O = w->O;
    float *P = w->params, *G = w->grad;
    const int nb = 32;
    if (combine) {
        const int K2 = 2 * w->K;
        hipLaunchKernelGGL(k_pol_combine, dim3((B * K2 + 255) / 256), dim3(256), 0, s, B, K2, w->y, w->pol, w->yc);
        hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, s, B * K2, w->yc, w->tgt, w->dyc, 1.f / float(B * K2),
                           w->lpart);
        hipLaunchKernelGGL(k_pol_combine_back, dim3((B * O + 255) / 256), dim3(256), 0, s, B, K2, w->dyc, w->pol,
                           w->dy);
    } else {
        hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, s, B * O, w->y, w->tgt, w->dy, 1.f / float(B * O),
                           w->lpart);
    }
    // layer 3
    sgemm<true, false>(O, H, B, w->dy, O, w->a2, H, G + w->off[4], H, s);   // dW3 = dy^T a2
    hipLaunchKernelGGL(k_colsum, dim3((O + 63) / 64), dim3(1024), 0, s, B, O, w->dy, G + w->off[5]);
    // dZ2 = (dy W3) (1 - a2^2)
    sgemm<false, false>(B, H, O, w->dy, O, P + w->off[4], H, w->d2, H, s, EPI_TANH_BACK, nullptr, w->a2);
    // layer 2
    sgemm<true, false>(H, H, B, w->d2, H, w->a1, H, G + w->off[2], H, s);
    hipLaunchKernelGGL(k_colsum, dim3((H + 63) / 64), dim3(1024), 0, s, B, H, w->d2, G + w->off[3]);
    sgemm<false, false>(B, H, H, w->d2, H, P + w->off[2], H, w->d1, H, s, EPI_TANH_BACK, nullptr, w->a1);
    // layer 1
    sgemm<true, false>(H, 4, B, w->d1, H, w->in, 4, G + w->off[0], 4, s);
    hipLaunchKernelGGL(k_colsum, dim3((H + 63) / 64), dim3(1024), 0, s, B, H, w->d1, G + w->off[1]);
    BIE_HIP(hipGetLastError());
    return nb;
}

void glorot(bie_ws *w, uint64_t seed)
{
    const size_t H = w->H, O = w->O;
    std::vector<float> h(w->nparams, 0.f);
    SM64 g(seed);
    auto fill = [&](size_t off, size_t fan_out, size_t fan_in) {
        const double lim = std::sqrt(6.0 / double(fan_in + fan_out));
        for (size_t i = 0; i < fan_out * fan_in; ++i) h[off + i] = float((2.0 * g.uniform() - 1.0) * lim);
    };
    fill(w->off[0], H, 4);
    fill(w->off[2], H, H);
    fill(w->off[4], O, H);
    BIE_HIP(hipMemcpy(w->params, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice));
}

}  // namespace

// Network inputs as FP32 on the device (S x 4; the linear-in-polarisation
// model takes the direction alone, its fourth input is 0).
static float *upload_features(const bie_ws *w, const double *feats, int64_t S)
{
    std::vector<float> fh(size_t(S) * 4);
    for (size_t i = 0; i < fh.size(); ++i) fh[i] = float(feats[i]);
    if (w->pmodel == 1)
        for (int64_t i = 0; i < S; ++i) fh[i * 4 + 3] = 0.f;
    float *F = dmalloc<float>(fh.size());
    BIE_HIP(hipMemcpy(F, fh.data(), fh.size() * sizeof(float), hipMemcpyHostToDevice));
    return F;
}

static float *upload_pols(const double *pols, int64_t S)
{
    std::vector<float> eh(size_t(S) * 3);
    for (size_t i = 0; i < eh.size(); ++i) eh[i] = float(pols[i]);
    float *E = dmalloc<float>(eh.size());
    BIE_HIP(hipMemcpy(E, eh.data(), eh.size() * sizeof(float), hipMemcpyHostToDevice));
    return E;
}

// Adam on mini-batches of the device inputs F (S x 4), targets T (S x 2K) and
// polarisations E (S x 3, linear-in-polarisation model only): per epoch a
// Fisher-Yates shuffle from SplitMix64(seed + 1 + epoch), batches in that order,
// learning rate cosine-decayed from lr_max (first step) to lr_min (last step),
// Adam (0.9, 0.999, 1e-8) with bias correction 1 - beta^step.  Returns the mean
// squared error over the last epoch (NaN for 0 epochs).
static double ws_fit_dev(bie_ws *w, const float *F, const float *T, const float *E, int64_t S, int epochs, int batch,
                         double lr_max, double lr_min, uint64_t seed, hipStream_t s)
{
    const int TW = 2 * w->K;   // target width
    BIE_HIP(hipMemsetAsync(w->am, 0, w->nparams * sizeof(float), s));
    BIE_HIP(hipMemsetAsync(w->av, 0, w->nparams * sizeof(float), s));
    const int Bsz = int(std::min<int64_t>(batch, S));
    ws_batch_scratch(w, Bsz);
    const int64_t nbatch = (S + Bsz - 1) / Bsz;
    const int64_t total = int64_t(epochs) * nbatch;
    int64_t step = 0;
    std::vector<int64_t> perm(S);
    int64_t *dperm = dmalloc<int64_t>(size_t(S));
    std::vector<double> lp(64);
    double last = NAN;
    const double PI = 3.14159265358979323846;
    try {
        for (int ep = 0; ep < epochs; ++ep) {
            for (int64_t i = 0; i < S; ++i) perm[i] = i;
            SM64 g(seed + 1 + uint64_t(ep));
            for (int64_t i = S - 1; i > 0; --i) std::swap(perm[i], perm[g.below(uint64_t(i + 1))]);
            BIE_HIP(hipMemcpyAsync(dperm, perm.data(), size_t(S) * sizeof(int64_t), hipMemcpyHostToDevice, s));
            double eloss = 0.0;
            for (int64_t bi = 0; bi < nbatch; ++bi) {
                const int64_t b0 = bi * Bsz;
                const int B = int(std::min<int64_t>(Bsz, S - b0));
                hipLaunchKernelGGL(k_gather, dim3(unsigned(B)), dim3(256), 0, s, B, TW, dperm, b0, F, T, E, w->in,
                                   w->tgt, w->pol);
                mlp_forward(w, B, s);
                const int nb = mlp_backward(w, B, s, w->pmodel == 1);
                ++step;
                const double lr = lr_min + 0.5 * (lr_max - lr_min) *
                                               (1.0 + std::cos(PI * double(step - 1) /
                                                               double(std::max<int64_t>(1, total - 1))));
                const float c1 = float(1.0 - std::pow(0.9, double(step)));
                const float c2 = float(1.0 - std::pow(0.999, double(step)));
                hipLaunchKernelGGL(k_adam, dim3(unsigned((w->nparams + 255) / 256)), dim3(256), 0, s,
                                   int(w->nparams), w->params, w->grad, w->am, w->av, float(lr), 0.9f, 0.999f, 1e-8f,
                                   c1, c2);
                BIE_HIP(hipGetLastError());
                if (ep == epochs - 1) {
                    BIE_HIP(hipMemcpyAsync(lp.data(), w->lpart, nb * sizeof(double), hipMemcpyDeviceToHost, s));
                    BIE_HIP(hipStreamSynchronize(s));
                    double a = 0.0;
                    for (int q = 0; q < nb; ++q) a += lp[q];
                    eloss += a / double(B * TW) * B;
                }
            }
            if (ep == epochs - 1) last = eloss / double(S);
            // the host permutation is rewritten next epoch: wait for its upload
            BIE_HIP(hipStreamSynchronize(s));
        }
    } catch (...) {
        (void)hipFree(dperm);
        throw;
    }
    (void)hipFree(dperm);
    BIE_HIP(hipStreamSynchronize(s));
    return last;
}

// POD basis of the S snapshots X (S x N, device) with K modes.
static void pod_basis(bie_ws *w, const double2 *X, int64_t S, int oversample, int power, uint64_t seed, hipStream_t s)
{
    const int64_t N = w->op->mesh.N;
    const int K = w->K;
    const int L = int(std::min<int64_t>(int64_t(K) + oversample, S));
    if (K > L) throw Error(BIE_EINVAL, "pod_rank exceeds the number of snapshots");
    // Omega (L x S) uniform in [-1, 1] + j[-1, 1] from SplitMix64
    std::vector<double2> om(size_t(L) * S);
    SM64 g(seed ^ 0x5bd1e995ULL);
    for (auto &v : om) v = make_double2(2.0 * g.uniform() - 1.0, 2.0 * g.uniform() - 1.0);
    double2 *dOm = dmalloc<double2>(om.size());
    double2 *Y = dmalloc<double2>(size_t(L) * N), *Yt = dmalloc<double2>(size_t(L) * N);
    double2 *Zs = dmalloc<double2>(size_t(L) * S), *Gd = dmalloc<double2>(size_t(L) * L);
    double2 *Wd = dmalloc<double2>(size_t(L) * L);
    auto cleanup = [&]() {
        for (void *p : { (void *)dOm, (void *)Y, (void *)Yt, (void *)Zs, (void *)Gd, (void *)Wd }) (void)hipFree(p);
    };
    try {
        BIE_HIP(hipMemcpy(dOm, om.data(), om.size() * sizeof(double2), hipMemcpyHostToDevice));
        lincomb(L, S, N, dOm, X, Y, s);   // Y_l = sum_s Omega[l][s] x_s
        std::vector<cd> G(size_t(L) * L);
        auto orthonormalise = [&]() {   // CholeskyQR applied twice: Y <- Y R^{-1}
            for (int pass = 0; pass < 2; ++pass) {
                inner(L, L, N, Y, Y, Gd, s);   // G[p][q] = <y_p, y_q>
                BIE_HIP(hipMemcpyAsync(G.data(), Gd, G.size() * sizeof(cd), hipMemcpyDeviceToHost, s));
                BIE_HIP(hipStreamSynchronize(s));
                // G here is G[p][q] = y_p^H y_q: the Gram matrix Y^H Y
                std::vector<cd> Ri = chol_inv_upper(G, L);
                // new y_c = sum_i y_i Ri[i][c]  ->  coefficients Coef[c][i] = Ri[i][c]
                std::vector<cd> coef(size_t(L) * L);
                for (int c = 0; c < L; ++c)
                    for (int i = 0; i < L; ++i) coef[size_t(c) * L + i] = Ri[size_t(i) * L + c];
                BIE_HIP(hipMemcpy(Wd, coef.data(), coef.size() * sizeof(cd), hipMemcpyHostToDevice));
                lincomb(L, L, N, Wd, Y, Yt, s);
                std::swap(Y, Yt);
            }
        };
        orthonormalise();
        for (int it = 0; it < power; ++it) {
            inner(L, S, N, Y, X, Zs, s);   // Zs[l][s] = y_l^H x_s  (= (A^H Y)^H)
            // Y <- A (A^H Y): y_l = sum_s x_s conj(Zs[l][s])
            std::vector<cd> zs(size_t(L) * S);
            BIE_HIP(hipMemcpy(zs.data(), Zs, zs.size() * sizeof(cd), hipMemcpyDeviceToHost));
            for (auto &v : zs) v = std::conj(v);
            BIE_HIP(hipMemcpy(Zs, zs.data(), zs.size() * sizeof(cd), hipMemcpyHostToDevice));
            lincomb(L, S, N, Zs, X, Y, s);
            orthonormalise();
        }
        // B = Q^H A (L x S), M = B B^H (L x L)
        inner(L, S, N, Y, X, Zs, s);            // B[l][s] = q_l^H x_s
        inner(L, L, S, Zs, Zs, Gd, s);          // G[p][q] = sum_s conj(B[p][s]) B[q][s] = conj((B B^H)[p][q])
        std::vector<cd> M(size_t(L) * L);
        BIE_HIP(hipMemcpyAsync(M.data(), Gd, M.size() * sizeof(cd), hipMemcpyDeviceToHost, s));
        BIE_HIP(hipStreamSynchronize(s));
        for (auto &v : M) v = std::conj(v);
        std::vector<double> ev;
        std::vector<cd> Wv;
        jacobi_eig(M, L, ev, Wv);
        w->sigma.resize(K);
        for (int k = 0; k < K; ++k) w->sigma[k] = std::sqrt(std::max(ev[k], 0.0));
        // u_k = sum_l q_l W[l][k]  -> coefficients Coef[k][l] = W[l][k]
        std::vector<cd> coef(size_t(K) * L);
        for (int k = 0; k < K; ++k)
            for (int l = 0; l < L; ++l) coef[size_t(k) * L + l] = Wv[size_t(l) * L + k];
        BIE_HIP(hipMemcpy(Wd, coef.data(), coef.size() * sizeof(cd), hipMemcpyHostToDevice));
        w->U = dmalloc<double2>(size_t(K) * N);
        lincomb(K, L, N, Wd, Y, w->U, s);
        BIE_HIP(hipStreamSynchronize(s));
    } catch (...) {
        cleanup();
        throw;
    }
    cleanup();
}

bie_ws *ws_train(const bie_op *op, const double *feats, const double *pols, const void *Xv, int64_t S,
                 const bie_ws_opts &o, hipStream_t s)
{
    const int64_t N = op->mesh.N;
    auto w = std::make_unique<bie_ws>();
    w->op = op;
    w->K = o.pod_rank;
    w->H = o.hidden;
    w->pmodel = o.pol_model;
    w->O = (o.pol_model == 1 ? 6 : 2) * o.pod_rank;
    if (o.pol_model == 1 && !pols) throw Error(BIE_EINVAL, "the linear-in-polarisation model needs the polarisations");
    const double2 *X = static_cast<const double2 *>(Xv);
    pod_basis(w.get(), X, S, o.oversample, o.power_iters, o.seed, s);
    // targets: C = U^H X (K x S), one global RMS scale
    double2 *C = dmalloc<double2>(size_t(w->K) * S);
    float *T = dmalloc<float>(size_t(S) * 2 * w->K);
    std::vector<cd> ch(size_t(w->K) * S);
    inner(w->K, S, N, w->U, X, C, s);
    BIE_HIP(hipMemcpy(ch.data(), C, ch.size() * sizeof(cd), hipMemcpyDeviceToHost));
    double ss = 0.0;
    for (const cd &c : ch) ss += std::norm(c);
    w->scale = std::sqrt(ss / double(2 * ch.size()));
    if (!(w->scale > 0.0)) w->scale = 1.0;
    hipLaunchKernelGGL(k_targets, dim3(unsigned((S * w->K + 255) / 256)), dim3(256), 0, s, int(S), w->K, C,
                       1.0 / w->scale, T);
    BIE_HIP(hipGetLastError());
    ws_alloc_params(w.get());
    glorot(w.get(), o.seed);
    float *F = nullptr, *E = nullptr;
    try {
        F = upload_features(w.get(), feats, S);
        if (w->pmodel == 1) E = upload_pols(pols, S);
        w->final_loss = ws_fit_dev(w.get(), F, T, E, S, o.epochs, o.batch, o.lr_max, o.lr_min, o.seed, s);
    } catch (...) {
        for (void *p : { (void *)C, (void *)T, (void *)F, (void *)E }) (void)hipFree(p);
        throw;
    }
    for (void *p : { (void *)C, (void *)T, (void *)F, (void *)E }) (void)hipFree(p);
    return w.release();
}

double ws_fit(bie_ws *w, const double *feats, const double *pols, const float *targets, int64_t S, int epochs,
              int batch, double lr_max, double lr_min, uint64_t seed, hipStream_t s)
{
    if (w->pmodel == 1 && !pols) throw Error(BIE_EINVAL, "the linear-in-polarisation model needs the polarisations");
    float *F = nullptr, *E = nullptr, *T = nullptr;
    double loss = NAN;
    try {
        F = upload_features(w, feats, S);
        if (w->pmodel == 1) E = upload_pols(pols, S);
        T = dmalloc<float>(size_t(S) * 2 * w->K);
        BIE_HIP(hipMemcpy(T, targets, size_t(S) * 2 * w->K * sizeof(float), hipMemcpyHostToDevice));
        loss = ws_fit_dev(w, F, T, E, S, epochs, batch, lr_max, lr_min, seed, s);
    } catch (...) {
        for (void *p : { (void *)F, (void *)E, (void *)T }) (void)hipFree(p);
        throw;
    }
    for (void *p : { (void *)F, (void *)E, (void *)T }) (void)hipFree(p);
    return loss;
}

// Network outputs for R feature rows (host FP64 in, device FP32 out in w->y).
static void ws_eval(bie_ws *w, const double *feats, int64_t R, hipStream_t s)
{
    ws_batch_scratch(w, int(R));
    std::vector<float> fh(size_t(R) * 4);
    for (size_t i = 0; i < fh.size(); ++i) fh[i] = float(feats[i]);
    if (w->pmodel == 1)
        for (int64_t i = 0; i < R; ++i) fh[i * 4 + 3] = 0.f;
    BIE_HIP(hipMemcpyAsync(w->in, fh.data(), fh.size() * sizeof(float), hipMemcpyHostToDevice, s));
    mlp_forward(w, int(R), s);
}

void ws_predict(bie_ws *w, const double *feats, const double *pols, int64_t R, const void *B, void *X0, int *used,
                hipStream_t s)
{
    const int64_t N = w->op->mesh.N;
    if (!w->U) throw Error(BIE_EINVAL, "warm start has no POD basis (untrained)");
    if (w->pmodel == 1 && !pols) throw Error(BIE_EINVAL, "the linear-in-polarisation model needs the polarisations");
    ws_eval(w, feats, R, s);
    const float *out = w->y;
    if (w->pmodel == 1) {
        std::vector<float> eh(size_t(R) * 3);
        for (size_t i = 0; i < eh.size(); ++i) eh[i] = float(pols[i]);
        BIE_HIP(hipMemcpyAsync(w->pol, eh.data(), eh.size() * sizeof(float), hipMemcpyHostToDevice, s));
        const int K2 = 2 * w->K;
        hipLaunchKernelGGL(k_pol_combine, dim3(unsigned((R * K2 + 255) / 256)), dim3(256), 0, s, int(R), K2, w->y,
                           w->pol, w->yc);
        out = w->yc;
    }
    if (w->cap_coef < R) {
        if (w->coef) (void)hipFree(w->coef);
        w->coef = nullptr;
        w->coef = dmalloc<double2>(size_t(R) * w->K);
        w->cap_coef = R;
    }
    hipLaunchKernelGGL(k_out_to_coef, dim3(unsigned((R * w->K + 255) / 256)), dim3(256), 0, s, int(R), w->K, out,
                       w->scale, w->coef);
    lincomb(R, w->K, N, w->coef, w->U, static_cast<double2 *>(X0), s);
    if (!B) {
        if (used)
            for (int64_t r = 0; r < R; ++r) used[r] = 1;
        return;
    }
    // fallback: keep x0 only where ||b - T x0|| < ||b||
    if (w->cap_res < R) {
        for (void *p : { (void *)w->res, (void *)w->nr }) if (p) (void)hipFree(p);
        w->res = nullptr;
        w->nr = nullptr;
        w->res = dmalloc<double2>(size_t(R) * N);
        w->nr = dmalloc<double>(size_t(2 * R));
        w->cap_res = R;
    }
    const bool m64 = w->op->Z64 != nullptr;
    if (m64 && R >= 8) gemm64_product(w->op, X0, N, w->res, N, B, N, R, nullptr, s);   // many columns: matrix cores
    else product(w->op, m64 ? MAT64 : MAT32, true, X0, N, w->res, N, B, N, R, nullptr, 1, false, s);
    hipLaunchKernelGGL(k_sqnorm, dim3(unsigned(R)), dim3(256), 0, s, N, w->res, w->nr);
    hipLaunchKernelGGL(k_sqnorm, dim3(unsigned(R)), dim3(256), 0, s, N, static_cast<const double2 *>(B), w->nr + R);
    std::vector<double> h(size_t(2 * R));
    BIE_HIP(hipMemcpyAsync(h.data(), w->nr, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    BIE_HIP(hipStreamSynchronize(s));
    for (int64_t r = 0; r < R; ++r) {
        const bool keep = h[r] < h[R + r];
        if (used) used[r] = keep;
        if (!keep) BIE_HIP(hipMemsetAsync(static_cast<double2 *>(X0) + r * N, 0, N * sizeof(double2), s));
    }
}

// Loss and gradient of the MSE for given inputs (R x 4; R x 3 polarisations
// for the linear-in-polarisation model) and targets (R x 2K), host buffers.
double ws_loss_grad(bie_ws *w, const double *feats, const double *pols, const float *targets, int64_t R,
                    float *grad_host, hipStream_t s)
{
    if (w->pmodel == 1 && !pols) throw Error(BIE_EINVAL, "the linear-in-polarisation model needs the polarisations");
    ws_eval(w, feats, R, s);
    const int TW = 2 * w->K;
    BIE_HIP(hipMemcpyAsync(w->tgt, targets, size_t(R) * TW * sizeof(float), hipMemcpyHostToDevice, s));
    std::vector<float> eh;
    if (w->pmodel == 1) {
        eh.resize(size_t(R) * 3);
        for (size_t i = 0; i < eh.size(); ++i) eh[i] = float(pols[i]);
        BIE_HIP(hipMemcpyAsync(w->pol, eh.data(), eh.size() * sizeof(float), hipMemcpyHostToDevice, s));
    }
    const int nb = mlp_backward(w, int(R), s, w->pmodel == 1);
    std::vector<double> lp(nb);
    BIE_HIP(hipMemcpyAsync(lp.data(), w->lpart, nb * sizeof(double), hipMemcpyDeviceToHost, s));
    if (grad_host) BIE_HIP(hipMemcpyAsync(grad_host, w->grad, w->nparams * sizeof(float), hipMemcpyDeviceToHost, s));
    BIE_HIP(hipStreamSynchronize(s));
    double a = 0.0;
    for (double v : lp) a += v;
    return a / double(R * TW);
}

void ws_forward(bie_ws *w, const double *feats, int64_t R, float *out_host, hipStream_t s)
{
    ws_eval(w, feats, R, s);
    BIE_HIP(hipMemcpyAsync(out_host, w->y, size_t(R) * w->O * sizeof(float), hipMemcpyDeviceToHost, s));
    BIE_HIP(hipStreamSynchronize(s));
}

void ws_destroy(bie_ws *w) { delete w; }

void ws_info(const bie_ws *w, int64_t *K, int64_t *H, int64_t *nparams, double *scale, double *loss, double *sigma)
{
    if (K) *K = w->K;
    if (H) *H = w->H;
    if (nparams) *nparams = int64_t(w->nparams);
    if (scale) *scale = w->scale;
    if (loss) *loss = w->final_loss;
    if (sigma)
        for (size_t i = 0; i < w->sigma.size(); ++i) sigma[i] = w->sigma[i];
}

bie_ws *ws_create_untrained(const bie_op *op, int K, int H, uint64_t seed, int pol_model)
{
    auto w = std::make_unique<bie_ws>();
    w->op = op;
    w->K = K;
    w->H = H;
    w->pmodel = pol_model;
    w->O = (pol_model == 1 ? 6 : 2) * K;
    ws_alloc_params(w.get());
    glorot(w.get(), seed);
    return w.release();
}

void ws_params(bie_ws *w, float *host, bool set)
{
    if (set) BIE_HIP(hipMemcpy(w->params, host, w->nparams * sizeof(float), hipMemcpyHostToDevice));
    else BIE_HIP(hipMemcpy(host, w->params, w->nparams * sizeof(float), hipMemcpyDeviceToHost));
}

void ws_basis(const bie_ws *w, void *U, hipStream_t s)
{
    if (!w->U) throw Error(BIE_EINVAL, "warm start has no POD basis (untrained)");
    BIE_HIP(hipMemcpyAsync(U, w->U, size_t(w->K) * w->op->mesh.N * sizeof(double2), hipMemcpyDeviceToDevice, s));
    BIE_HIP(hipStreamSynchronize(s));
}

void ws_save(const bie_ws *w, const char *path)
{
    FILE *f = std::fopen(path, "wb");
    if (!f) throw Error(BIE_EINVAL, std::string("cannot open ") + path);
    const int64_t N = w->op->mesh.N;
    std::vector<double2> U(size_t(w->K) * N);
    std::vector<float> P(w->nparams);
    BIE_HIP(hipMemcpy(U.data(), w->U, U.size() * sizeof(double2), hipMemcpyDeviceToHost));
    BIE_HIP(hipMemcpy(P.data(), w->params, P.size() * sizeof(float), hipMemcpyDeviceToHost));
    const char magic[8] = { 'B', 'I', 'E', 'W', 'S', '0', '0', '2' };
    const int64_t hdr[5] = { N, w->K, w->H, int64_t(w->nparams), w->pmodel };
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(hdr, sizeof(hdr), 1, f) == 1 &&
              std::fwrite(&w->scale, sizeof(double), 1, f) == 1 &&
              std::fwrite(w->sigma.data(), sizeof(double), w->sigma.size(), f) == w->sigma.size() &&
              std::fwrite(U.data(), sizeof(double2), U.size(), f) == U.size() &&
              std::fwrite(P.data(), sizeof(float), P.size(), f) == P.size();
    std::fclose(f);
    if (!ok) throw Error(BIE_EINVAL, std::string("write failed: ") + path);
}

bie_ws *ws_load(const bie_op *op, const char *path)
{
    FILE *f = std::fopen(path, "rb");
    if (!f) throw Error(BIE_EINVAL, std::string("cannot open ") + path);
    char magic[8];
    int64_t hdr[5];
    double scale;
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "BIEWS002", 8) == 0 &&
              std::fread(hdr, sizeof(hdr), 1, f) == 1 && std::fread(&scale, sizeof(double), 1, f) == 1;
    if (!ok || hdr[0] != op->mesh.N || hdr[1] < 1 || hdr[2] < 1) {
        std::fclose(f);
        throw Error(BIE_EINVAL, "warm-start file does not match this operator");
    }
    auto w = std::make_unique<bie_ws>();
    w->op = op;
    w->K = int(hdr[1]);
    w->H = int(hdr[2]);
    w->pmodel = int(hdr[4]);
    w->O = (w->pmodel == 1 ? 6 : 2) * w->K;
    w->scale = scale;
    ws_alloc_params(w.get());
    if (int64_t(w->nparams) != hdr[3]) {
        std::fclose(f);
        throw Error(BIE_EINVAL, "warm-start file: parameter count mismatch");
    }
    w->sigma.resize(w->K);
    std::vector<double2> U(size_t(w->K) * op->mesh.N);
    std::vector<float> P(w->nparams);
    ok = std::fread(w->sigma.data(), sizeof(double), w->K, f) == size_t(w->K) &&
         std::fread(U.data(), sizeof(double2), U.size(), f) == U.size() &&
         std::fread(P.data(), sizeof(float), P.size(), f) == P.size();
    std::fclose(f);
    if (!ok) throw Error(BIE_EINVAL, "warm-start file truncated");
    w->U = dmalloc<double2>(U.size());
    BIE_HIP(hipMemcpy(w->U, U.data(), U.size() * sizeof(double2), hipMemcpyHostToDevice));
    BIE_HIP(hipMemcpy(w->params, P.data(), P.size() * sizeof(float), hipMemcpyHostToDevice));
    return w.release();
}

}  // namespace bie
