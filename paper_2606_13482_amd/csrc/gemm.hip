// Block product Y = T X for many right-hand sides on the matrix cores.
//
// The complex product is one real GEMM with re/im interleaved along K and the
// two output parts of each right-hand side in adjacent columns:
//   A[m][2n] = Re T_mn, A[m][2n+1] = Im T_mn                        (M = N, K = 2N)
//   B[2n][2r]   = Re x_rn, B[2n+1][2r]   = -Im x_rn   (column 2r   -> Re y_r)
//   B[2n][2r+1] = Im x_rn, B[2n+1][2r+1] =  Re x_rn   (column 2r+1 -> Im y_r)
// Both operands are split into BF16 pairs (hi = rne(v), lo = rne(v - hi)) and
// C = Ah Bh + Ah Bl + Al Bh is accumulated in FP32 with
// v_mfma_f32_32x32x16_bf16 (about 16 significant bits per product entry; the
// dropped lo*lo term is below the FP32 accumulation error).
//
// Tiling: a block of 8 waves computes a 256 x 256 tile of C over one slice of
// K; wave (wm, wn) owns rows 128 wm .. +128 and columns 64 wn .. +64 as 4 x 2
// MFMA tiles of 32 x 32 (12 fragment reads from LDS feed 24 MFMAs per 16-deep
// step).  K advances in stages of 32; both planes of the A and B stage sit in
// LDS, double-buffered (160 KiB), rows padded to 40 BF16 to spread banks.
// While a stage is computed the next one goes from registers to the other
// buffer and the one after it is loaded from memory into registers: one
// barrier per stage, loads issued two stages ahead.
//
// Split K: when the output tiles alone cannot fill the 256 compute units (one
// 160 KiB block per CU), K is cut into KS slices (grid z).  Every block writes
// its FP32 tile to a partial buffer [KS][Mp][NCp] (lanes along columns: 128-byte
// runs); a second kernel sums the slices in FP64, subtracts from B if asked,
// and transposes through LDS so that the complex128 output is written in
// contiguous runs along m.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>

#include "bie_internal.hpp"

namespace bie {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int GBM = 256, GBN = 256, GBK = 32, PK = GBK + 8;
constexpr int TI = 4, TJ = 2;   // 32x32 MFMA tiles per wave (128 rows x 64 columns)

// XCD-aware tile order: workgroups are dealt to the 8 XCDs round robin by
// linear id p, so logical tile L = (p % 8) Q + p / 8 (Q = P / 8) gives each XCD
// a run of consecutive L.  L enumerates column tiles innermost, so the blocks
// sharing one A slice (same row tile and K slice) run on one XCD, at the same
// time, and all but the first read A from that XCD's L2.
__device__ inline void xcd_tile(unsigned &bx, unsigned &by, unsigned &bz)
{
    const unsigned gx = gridDim.x, gy = gridDim.y, P = gx * gy * gridDim.z;
    const unsigned p = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z), Q = P / 8;
    const unsigned L = p < 8 * Q ? (p % 8) * Q + p / 8 : p;
    by = L % gy;
    bx = (L / gy) % gx;
    bz = L / (gy * gx);
}

__device__ inline void split_bf16(float v, __bf16 &hi, __bf16 &lo)
{
    hi = (__bf16)v;
    lo = (__bf16)(v - (float)hi);
}

// A planes [Mp][Kp] from the packed symmetric FP64 tiles (zero padding).
__global__ __launch_bounds__(256) void k_split_matrix(const double2 *__restrict__ Zp, int64_t N, int64_t nT,
                                                      int64_t Kp, __bf16 *__restrict__ Ah, __bf16 *__restrict__ Al)
{
    const int64_t m = blockIdx.y;
    for (int64_t n = int64_t(blockIdx.x) * 256 + threadIdx.x; 2 * n < Kp; n += int64_t(gridDim.x) * 256) {
        double2 z = make_double2(0.0, 0.0);
        if (m < N && n < N) {
            const int64_t I = m / TB, J = n / TB;
            z = I <= J ? Zp[tile_of(I, J, nT) * TB * TB + (m % TB) * TB + (n % TB)]
                       : Zp[tile_of(J, I, nT) * TB * TB + (n % TB) * TB + (m % TB)];
        }
        __bf16 h0, l0, h1, l1;
        split_bf16(float(z.x), h0, l0);
        split_bf16(float(z.y), h1, l1);
        Ah[m * Kp + 2 * n] = h0;
        Ah[m * Kp + 2 * n + 1] = h1;
        Al[m * Kp + 2 * n] = l0;
        Al[m * Kp + 2 * n + 1] = l1;
    }
}

// B planes [NCp][Kp] from R complex vectors (complex128 or complex64 XT):
// GEMM column pair r reads the vector at X + v*ldx, v = cols ? cols[r] : r.
template <typename XT>
__global__ __launch_bounds__(256) void k_split_vectors(const XT *__restrict__ X, int64_t ldx, const int *__restrict__ cols,
                                                       int64_t N, int64_t R, int64_t Kp, __bf16 *__restrict__ Bh,
                                                       __bf16 *__restrict__ Bl, bool lo)
{
    const int64_t c = blockIdx.y;
    const int64_t v = c < 2 * R ? (cols ? int64_t(cols[c >> 1]) : (c >> 1)) : 0;
    for (int64_t n = int64_t(blockIdx.x) * 256 + threadIdx.x; 2 * n < Kp; n += int64_t(gridDim.x) * 256) {
        float a = 0.f, b = 0.f;
        if (n < N && c < 2 * R) {
            const XT x = X[v * ldx + n];
            if (!(c & 1)) { a = float(x.x); b = float(-x.y); }
            else { a = float(x.y); b = float(x.x); }
        }
        __bf16 h0, l0, h1, l1;
        split_bf16(a, h0, l0);
        split_bf16(b, h1, l1);
        Bh[c * Kp + 2 * n] = h0;
        Bh[c * Kp + 2 * n + 1] = h1;
        if (lo) {
            Bl[c * Kp + 2 * n] = l0;
            Bl[c * Kp + 2 * n + 1] = l1;
        }
    }
}

// Partial C = Ah Bh + Al Bh (+ Ah Bl when TERMS == 3) over the stages of one K
// slice, into P[z][Mp][NCp].  TERMS == 2 keeps the matrix split (about 16
// significant bits) and rounds the vectors to BF16 (2^-9 relative): the form
// for the inner corrections of iterative refinement, whose tolerance is far
// above that rounding; the B lo plane is then neither loaded nor stored.
template <int TERMS>
__global__ __launch_bounds__(512) void k_gemm_split(const __bf16 *__restrict__ Ah, const __bf16 *__restrict__ Al,
                                                    const __bf16 *__restrict__ Bh, const __bf16 *__restrict__ Bl,
                                                    int64_t Kp, int64_t Mp, int64_t NCp, float *__restrict__ P)
{
    __shared__ __attribute__((aligned(16))) __bf16 sA[2][2][GBM][PK];   // [buffer][plane][row][k]
    __shared__ __attribute__((aligned(16))) __bf16 sB[2][2][GBN][PK];   // [buffer][plane][col][k]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 2, wn = wave & 3;   // wave tile: rows 128 wm .. +128, columns 64 wn .. +64
    unsigned bx, by, bz;
    xcd_tile(bx, by, bz);
    const int64_t m0 = int64_t(bx) * GBM, c0 = int64_t(by) * GBN;

    // global -> register staging (16-byte chunks): per plane, A 256 x 32 and
    // B 256 x 32 = 1024 chunks each (2 per thread)
    constexpr int CPR = GBK / 8;   // chunks per row
    u32x4 ra[2][2], rb[2][2];
    auto gload = [&](int64_t k0) {
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int c = tid + 512 * q;
                ra[p][q] = *reinterpret_cast<const u32x4 *>((p ? Al : Ah) + (m0 + c / CPR) * Kp + k0 + (c % CPR) * 8);
                if (TERMS == 3 || p == 0)
                    rb[p][q] = *reinterpret_cast<const u32x4 *>((p ? Bl : Bh) + (c0 + c / CPR) * Kp + k0 + (c % CPR) * 8);
            }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int c = tid + 512 * q;
                *reinterpret_cast<u32x4 *>(&sA[buf][p][c / CPR][(c % CPR) * 8]) = ra[p][q];
                if (TERMS == 3 || p == 0) *reinterpret_cast<u32x4 *>(&sB[buf][p][c / CPR][(c % CPR) * 8]) = rb[p][q];
            }
    };

    f32x16 acc[TI][TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[i][j][q] = 0.f;

    const int fr = lane & 31, fk = (lane >> 5) * 8;
    // pipeline: stage s is computed from LDS buffer s%2 while stage s+1 is
    // stored into the other buffer and stage s+2 is in flight to registers;
    // one barrier per stage
    const int64_t nall = Kp / GBK, sb = nall * bz / gridDim.z, se = nall * (bz + 1) / gridDim.z;
    gload(sb * GBK);
    lstore(0);
    if (se - sb > 1) gload((sb + 1) * GBK);
    __syncthreads();
    for (int64_t st = sb; st < se; ++st) {
        const int buf = int((st - sb) & 1);
#pragma unroll
        for (int kk = 0; kk < GBK; kk += 16) {
            bf16x8 a[TI][2], b[TJ][2];   // [tile][plane]
#pragma unroll
            for (int p = 0; p < 2; ++p) {
#pragma unroll
                for (int t = 0; t < TI; ++t)
                    a[t][p] = *reinterpret_cast<const bf16x8 *>(&sA[buf][p][wm * 128 + t * 32 + fr][kk + fk]);
                if (TERMS == 3 || p == 0)
#pragma unroll
                    for (int t = 0; t < TJ; ++t)
                        b[t][p] = *reinterpret_cast<const bf16x8 *>(&sB[buf][p][wn * 64 + t * 32 + fr][kk + fk]);
            }
            // the products, each over the 8 independent accumulators
#pragma unroll
            for (int i = 0; i < TI; ++i)
#pragma unroll
                for (int j = 0; j < TJ; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][0], b[j][0], acc[i][j], 0, 0, 0);
            if (TERMS == 3)
#pragma unroll
                for (int i = 0; i < TI; ++i)
#pragma unroll
                    for (int j = 0; j < TJ; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][0], b[j][1], acc[i][j], 0, 0, 0);
#pragma unroll
            for (int i = 0; i < TI; ++i)
#pragma unroll
                for (int j = 0; j < TJ; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][1], b[j][0], acc[i][j], 0, 0, 0);
        }
        if (st + 1 < se) {
            lstore(buf ^ 1);                         // stage st+1 (already in registers)
            if (st + 2 < se) gload((st + 2) * GBK);  // stage st+2 in flight during the next compute
        }
        __syncthreads();
    }
    // accumulator q of lane l holds row 8(q/4) + 4(l/32) + q%4, column l%32 of its 32x32 tile
    float *Pz = P + int64_t(bz) * Mp * NCp;
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
            const int64_t c = c0 + wn * 64 + j * 32 + (lane & 31);
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int64_t m = m0 + wm * 128 + i * 32 + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
                Pz[m * NCp + c] = acc[i][j][q];
            }
        }
}

// Y[v][m] = sum_z (P[z][m][2r], P[z][m][2r+1]) (or Bsub[v][m] - that), v = cols ?
// cols[r] : r, for a tile of 64 rows x 32 right-hand sides; the slices are
// summed in FP64.
template <typename PT>
__global__ __launch_bounds__(256) void k_gemm_reduce(const PT *__restrict__ P, int KS, int64_t Mp, int64_t NCp,
                                                     int64_t N, int64_t R, const int *__restrict__ cols,
                                                     double2 *__restrict__ Y, int64_t ldy,
                                                     const double2 *__restrict__ Bsub, int64_t ldb)
{
    __shared__ double sd[64][65];   // [column][row]
    const int t = threadIdx.x;
    const int64_t m0 = int64_t(blockIdx.x) * 64, cb = int64_t(blockIdx.y) * 64;
    const int cl = t & 63;
#pragma unroll 4
    for (int it = 0; it < 16; ++it) {
        const int ml = it * 4 + (t >> 6);
        double v = 0.0;
        for (int z = 0; z < KS; ++z) v += double(P[(int64_t(z) * Mp + m0 + ml) * NCp + cb + cl]);
        sd[cl][ml] = v;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < 8; ++it) {
        const int idx = it * 256 + t, rl = idx >> 6, ml = idx & 63;
        const int64_t r = cb / 2 + rl, m = m0 + ml;
        if (r >= R || m >= N) continue;
        const int64_t v = cols ? int64_t(cols[r]) : r;
        double2 y = make_double2(sd[2 * rl][ml], sd[2 * rl + 1][ml]);
        if (Bsub) {
            const double2 b = Bsub[v * ldb + m];
            y = make_double2(b.x - y.x, b.y - y.y);
        }
        Y[v * ldy + m] = y;
    }
}

// ---------------------------------------------------------------------------
// FP64 block product on the matrix cores: the same real GEMM (re/im
// interleaved along K, output parts of right-hand side r in columns 2r, 2r+1)
// on a dense FP64 copy A64 [Mp64][Kp64] of the matrix, with
// v_mfma_f64_16x16x4f64 (A: lane l holds row l%16, k l/16; B: column l%16,
// k l/16; D: 4 values per lane, value q in row l/16 + 4q, column l%16 -- not
// the 4(l/16) + q of the FP32-output instructions).  The B operand
// is built from the complex vectors as they are staged into LDS: x_rn gives the
// 2x2 block [[Re, Im], [-Im, Re]] at k = 2n, 2n+1 and columns 2r, 2r+1.
// Block tile 128 x 128 (64 right-hand sides) by 4 waves of 64 x 64 (4 x 4
// MFMA tiles); K stages of 16 reals double-buffered in LDS (rows padded to 17
// doubles: conflict-free 8-byte fragment reads); split K and the XCD-aware
// order as in the BF16 product; FP64 partial tiles reduced in fixed order.
constexpr int DBM = 128, DBN = 128, DBK = 16, DPK = DBK + 1;
typedef double f64x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_dense64(const double2 *__restrict__ Zp, int64_t N, int64_t nT, int64_t Kp,
                                                 double *__restrict__ A)
{
    const int64_t m = blockIdx.y;
    for (int64_t n = int64_t(blockIdx.x) * 256 + threadIdx.x; 2 * n < Kp; n += int64_t(gridDim.x) * 256) {
        double2 z = make_double2(0.0, 0.0);
        if (m < N && n < N) {
            const int64_t I = m / TB, J = n / TB;
            z = I <= J ? Zp[tile_of(I, J, nT) * TB * TB + (m % TB) * TB + (n % TB)]
                       : Zp[tile_of(J, I, nT) * TB * TB + (n % TB) * TB + (m % TB)];
        }
        A[m * Kp + 2 * n] = z.x;
        A[m * Kp + 2 * n + 1] = z.y;
    }
}

__global__ __launch_bounds__(256) void k_gemm64(const double *__restrict__ A, int64_t Kp, int64_t N,
                                                const double2 *__restrict__ X, int64_t ldx,
                                                const int *__restrict__ cols, int64_t R, int64_t Mp, int64_t NCp,
                                                double *__restrict__ P)
{
    __shared__ double sA[2][DBM][DPK];
    __shared__ double sB[2][DBN][DPK];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;   // wave tile: rows 64 wm .. +64, columns 64 wn .. +64
    unsigned bx, by, bz;
    xcd_tile(bx, by, bz);
    const int64_t m0 = int64_t(bx) * DBM, c0 = int64_t(by) * DBN, r0 = c0 / 2;

    // staging: A 128 x 16 doubles = 1024 double2 (4 per thread); X 64 rhs x 8
    // complex = 512 double2 (2 per thread)
    double2 ra[4], rx[2];
    int64_t xv[2];   // vector index of the two right-hand sides this thread stages (-1: padding)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int64_t r = r0 + (tid + 256 * q) / 8;
        xv[q] = r < R ? (cols ? int64_t(cols[r]) : r) : -1;
    }
    auto gload = [&](int64_t k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = tid + 256 * q;   // row c / 8, pair c % 8
            ra[q] = *reinterpret_cast<const double2 *>(A + (m0 + c / 8) * Kp + k0 + 2 * (c % 8));
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int64_t n = k0 / 2 + (tid + 256 * q) % 8;
            rx[q] = (xv[q] >= 0 && n < N) ? X[xv[q] * ldx + n] : make_double2(0.0, 0.0);
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = tid + 256 * q;
            sA[buf][c / 8][2 * (c % 8)] = ra[q].x;
            sA[buf][c / 8][2 * (c % 8) + 1] = ra[q].y;
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int c = tid + 256 * q, rl = c / 8, nl = c % 8;
            sB[buf][2 * rl][2 * nl] = rx[q].x;
            sB[buf][2 * rl][2 * nl + 1] = -rx[q].y;
            sB[buf][2 * rl + 1][2 * nl] = rx[q].y;
            sB[buf][2 * rl + 1][2 * nl + 1] = rx[q].x;
        }
    };

    f64x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f64x4{ 0.0, 0.0, 0.0, 0.0 };

    const int fr = lane & 15, fk = lane >> 4;
    const int64_t nall = Kp / DBK, sb = nall * bz / gridDim.z, se = nall * (bz + 1) / gridDim.z;
    gload(sb * DBK);
    lstore(0);
    if (se - sb > 1) gload((sb + 1) * DBK);
    __syncthreads();
    for (int64_t st = sb; st < se; ++st) {
        const int buf = int((st - sb) & 1);
#pragma unroll
        for (int kk = 0; kk < DBK; kk += 4) {
            double a[4], b[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                a[t] = sA[buf][wm * 64 + t * 16 + fr][kk + fk];
                b[t] = sB[buf][wn * 64 + t * 16 + fr][kk + fk];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if (st + 1 < se) {
            lstore(buf ^ 1);
            if (st + 2 < se) gload((st + 2) * DBK);
        }
        __syncthreads();
    }
    double *Pz = P + int64_t(bz) * Mp * NCp;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t c = c0 + wn * 64 + j * 16 + (lane & 15);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t m = m0 + wm * 64 + i * 16 + (lane >> 4) + 4 * q;
                Pz[m * NCp + c] = acc[i][j][q];
            }
        }
}

// Slices of K per launch: enough blocks for the 256 compute units, at least
// 8 stages per slice; BIE_GEMM_SPLITK overrides (measurement).
int gemm_splitk(int64_t blocks, int64_t nst)
{
    static const int env = [] {
        const char *e = getenv("BIE_GEMM_SPLITK");
        return e ? atoi(e) : 0;
    }();
    int64_t ks = env > 0 ? env : std::max<int64_t>(1, 256 / blocks);
    ks = std::min<int64_t>(ks, std::max<int64_t>(1, nst / 8));
    return int(std::max<int64_t>(1, std::min<int64_t>(ks, 64)));
}

}  // namespace

int64_t gemm_pad_rows(int64_t N) { return (N + GBM - 1) / GBM * GBM; }
int64_t gemm_pad_k(int64_t N) { return (2 * N + GBK - 1) / GBK * GBK; }
int64_t gemm_pad_cols(int64_t R) { return (2 * R + GBN - 1) / GBN * GBN; }

// Split-BF16 copy of the FP64 matrix (A planes, hi then lo).
void split_matrix(bie_op *op, hipStream_t s)
{
    const int64_t N = op->mesh.N, Mp = gemm_pad_rows(N), Kp = gemm_pad_k(N);
    const size_t plane = size_t(Mp) * size_t(Kp);
    BIE_HIP(hipMalloc(&op->Abf, 2 * plane * sizeof(__bf16)));
    op->gemm_Mp = Mp;
    op->gemm_Kp = Kp;
    __bf16 *Ah = static_cast<__bf16 *>(op->Abf), *Al = Ah + plane;
    const dim3 grid(unsigned(std::min<int64_t>((Kp / 2 + 255) / 256, 64)), unsigned(Mp));
    hipLaunchKernelGGL(k_split_matrix, grid, dim3(256), 0, s, (const double2 *)op->Z64, N, op->pk.nT, Kp, Ah, Al);
    BIE_HIP(hipGetLastError());
    BIE_HIP(hipStreamSynchronize(s));
}

// Y = T X (or Bsub - T X) for R vectors with the split-BF16 matrix; X
// complex128 or complex64 (xf32), Y and Bsub complex128; cols (device, R
// entries, or null for 0..R-1) names the vectors taking part.
void gemm_product(const bie_op *opc, const void *X, int64_t ldx, bool xf32, void *Y, int64_t ldy, const void *Bsub,
                  int64_t ldb, int64_t R, const int *cols, hipStream_t s, int terms)
{
    if (terms != 2 && terms != 3) throw Error(BIE_EINVAL, "the split-BF16 product has 2 or 3 terms");
    bie_op *op = const_cast<bie_op *>(opc);
    const int64_t N = op->mesh.N, Kp = op->gemm_Kp, Mp = op->gemm_Mp, NCp = gemm_pad_cols(R);
    const size_t plane = size_t(NCp) * size_t(Kp);
    if (op->bstage_cols < NCp) {
        BIE_HIP(hipStreamSynchronize(s));
        if (op->Bbf) (void)hipFree(op->Bbf);
        op->Bbf = nullptr;
        op->bstage_cols = 0;
        BIE_HIP(hipMalloc(&op->Bbf, 2 * plane * sizeof(__bf16)));
        op->bstage_cols = NCp;
    }
    const int64_t blocks = (Mp / GBM) * (NCp / GBN);
    const int KS = gemm_splitk(blocks, Kp / GBK);
    const size_t pelems = size_t(KS) * size_t(Mp) * size_t(NCp);
    if (op->gemm_part_elems < pelems) {
        BIE_HIP(hipStreamSynchronize(s));
        if (op->gemm_part) (void)hipFree(op->gemm_part);
        op->gemm_part = nullptr;
        op->gemm_part_elems = 0;
        BIE_HIP(hipMalloc(&op->gemm_part, pelems * sizeof(float)));
        op->gemm_part_elems = pelems;
    }
    __bf16 *Bh = static_cast<__bf16 *>(op->Bbf), *Bl = Bh + plane;
    const __bf16 *Ah = static_cast<const __bf16 *>(op->Abf), *Al = Ah + size_t(Mp) * size_t(Kp);
    float *P = static_cast<float *>(op->gemm_part);
    const dim3 sgrid(unsigned(std::min<int64_t>((Kp / 2 + 255) / 256, 64)), unsigned(NCp));
    if (xf32)
        hipLaunchKernelGGL(k_split_vectors<float2>, sgrid, dim3(256), 0, s, (const float2 *)X, ldx, cols, N, R, Kp, Bh,
                           Bl, terms == 3);
    else
        hipLaunchKernelGGL(k_split_vectors<double2>, sgrid, dim3(256), 0, s, (const double2 *)X, ldx, cols, N, R, Kp,
                           Bh, Bl, terms == 3);
    prof_begin(1, s, R);
    const dim3 ggrid(unsigned(Mp / GBM), unsigned(NCp / GBN), unsigned(KS));
    if (terms == 3)
        hipLaunchKernelGGL(k_gemm_split<3>, ggrid, dim3(512), 0, s, Ah, Al, Bh, Bl, Kp, Mp, NCp, P);
    else
        hipLaunchKernelGGL(k_gemm_split<2>, ggrid, dim3(512), 0, s, Ah, Al, Bh, Bl, Kp, Mp, NCp, P);
    prof_end(1, s);
    hipLaunchKernelGGL(k_gemm_reduce<float>, dim3(unsigned(Mp / 64), unsigned(NCp / 64)), dim3(256), 0, s, P, KS, Mp,
                       NCp, N, R, cols, (double2 *)Y, ldy, (const double2 *)Bsub, ldb);
    BIE_HIP(hipGetLastError());
}


// Dense FP64 copy of the packed matrix for the FP64 block product.
void dense64_setup(bie_op *op, hipStream_t s)
{
    if (op->A64) return;
    const int64_t N = op->mesh.N, Mp = (N + DBM - 1) / DBM * DBM, Kp = (2 * N + DBK - 1) / DBK * DBK;
    BIE_HIP(hipMalloc(&op->A64, size_t(Mp) * size_t(Kp) * sizeof(double)));
    op->d64_Mp = Mp;
    op->d64_Kp = Kp;
    const dim3 grid(unsigned(std::min<int64_t>((Kp / 2 + 255) / 256, 64)), unsigned(Mp));
    hipLaunchKernelGGL(k_dense64, grid, dim3(256), 0, s, (const double2 *)op->Z64, N, op->pk.nT, Kp,
                       (double *)op->A64);
    BIE_HIP(hipGetLastError());
}

// Y = T X (or Bsub - T X) in FP64 on the matrix cores for R complex128 vectors
// (cols: device list of vector indices, or null for 0..R-1).
void gemm64_product(const bie_op *opc, const void *X, int64_t ldx, void *Y, int64_t ldy, const void *Bsub,
                    int64_t ldb, int64_t R, const int *cols, hipStream_t s)
{
    bie_op *op = const_cast<bie_op *>(opc);
    if (!op->Z64) throw Error(BIE_EINVAL, "the FP64 block product needs the FP64 matrix");
    dense64_setup(op, s);
    const int64_t N = op->mesh.N, Mp = op->d64_Mp, Kp = op->d64_Kp, NCp = (2 * R + DBN - 1) / DBN * DBN;
    const int64_t blocks = (Mp / DBM) * (NCp / DBN), nst = Kp / DBK;
    int64_t ks = std::max<int64_t>(1, 256 / blocks);
    ks = std::max<int64_t>(1, std::min<int64_t>({ ks, nst / 16, 64 }));
    const size_t pelems = size_t(ks) * size_t(Mp) * size_t(NCp);
    if (op->d64_part_elems < pelems) {
        BIE_HIP(hipStreamSynchronize(s));
        if (op->d64_part) (void)hipFree(op->d64_part);
        op->d64_part = nullptr;
        op->d64_part_elems = 0;
        BIE_HIP(hipMalloc(&op->d64_part, pelems * sizeof(double)));
        op->d64_part_elems = pelems;
    }
    double *P = static_cast<double *>(op->d64_part);
    prof_begin(2, s, R);
    hipLaunchKernelGGL(k_gemm64, dim3(unsigned(Mp / DBM), unsigned(NCp / DBN), unsigned(ks)), dim3(256), 0, s,
                       (const double *)op->A64, Kp, N, (const double2 *)X, ldx, cols, R, Mp, NCp, P);
    hipLaunchKernelGGL(k_gemm_reduce<double>, dim3(unsigned(Mp / 64), unsigned(NCp / 64)), dim3(256), 0, s, P,
                       int(ks), Mp, NCp, N, R, cols, (double2 *)Y, ldy, (const double2 *)Bsub, ldb);
    prof_end(2, s);
    BIE_HIP(hipGetLastError());
}

}  // namespace bie
