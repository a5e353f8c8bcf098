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
// Operand layout.  Every BF16 plane (A rows m, B columns c, both along K) is
// stored as 1 KiB tiles of 32 rows x 16 K values, one MFMA K step: tile
// (strip s = row / 32, stage t = k / 16) starts at element (s Kp/16 + t) 512,
// and inside it the 16-byte chunk h = (k / 8) mod 2 of row r sits in slot
// 2r + (h ^ ((r / 8) & 1)).  A tile is one contiguous run in HBM, so one LDS
// DMA instruction of one wave (global_load_lds_dwordx4: lane i's 16 bytes land
// at LDS base + 16 i) moves it into LDS unchanged, and the fragment read of a
// 32x32x16 MFMA (lane l: row l % 32, chunk l / 32) touches 16 distinct
// 16-byte bank groups in every 16 lanes: no bank conflicts.
//
// Tiling: a block computes a 256 x 256 tile of C over one slice of K, with 8
// waves of 128 x 64 (4 x 2 MFMA tiles: 12 fragment reads feed 24 MFMAs per K
// stage) or, selectable for measurement, 8 waves of 64 x 128 or 4 of 128 x 128.
// K stages of 16 (both planes of the A and B stage: 32 KiB) rotate through
// NS = 4 LDS buffers.  Step i: each wave waits for its own DMA of stage i+1,
// one barrier, the DMA of stage i+NS goes into the buffer of stage i (whose
// fragments are already in registers), stage i+1 is read into the second
// register set, and the MFMAs of stage i run from the first.  The DMA is
// three stages ahead of its use and the fragment reads one stage ahead.
//
// Split K: when the output tiles alone cannot fill the 256 compute units (one
// 128 KiB block per CU), K is cut into KS slices (grid z).  Every block writes
// its FP32 tile to a partial buffer [KS][Mp][NCp] (lanes along columns: 128-byte
// runs); a second kernel sums the slices in FP64, subtracts from B if asked,
// and transposes through LDS so that the complex128 output is written in
// contiguous runs along m.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <cstdint>
#include <cstdlib>

#include "bie_internal.hpp"

namespace bie {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int GBM = 256, GBN = 256, GBK = 16;   // block tile rows, columns; K stage

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

// Tile and slot of the 16-byte chunk h of row r (r < 32) in the tiled layout.
__device__ inline int tile_slot(int r, int h) { return 2 * r + (h ^ ((r >> 3) & 1)); }

// One wave per tile writes its 64 slots: lane l -> row l / 2 of the strip and
// the chunk stored in slot l.
__device__ inline void slot_owner(int lane, int &r, int &h)
{
    r = lane >> 1;
    h = (lane & 1) ^ ((r >> 3) & 1);
}

// A planes (tiled, [Mp / 32][Kp / 16] tiles) from the packed symmetric FP64
// matrix (zero padding); one wave per tile, 4 tiles per block.
__global__ __launch_bounds__(256) void k_split_matrix(const double2 *__restrict__ Zp, int64_t N, int64_t nT,
                                                      int64_t Mp, int64_t Kp, __bf16 *__restrict__ Ah,
                                                      __bf16 *__restrict__ Al)
{
    const int64_t nst = Kp / GBK, tile = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (tile >= (Mp / 32) * nst) return;
    int r, h;
    slot_owner(threadIdx.x & 63, r, h);
    const int64_t m = (tile / nst) * 32 + r, n0 = (tile % nst) * 8 + h * 4;   // 4 complex entries n0 .. n0+3
    bf16x8 hi, lo;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t n = n0 + e;
        double2 z = make_double2(0.0, 0.0);
        if (m < N && n < N) {
            const int64_t I = m / TB, J = n / TB;
            z = I <= J ? Zp[tile_of(I, J, nT) * TB * TB + (m % TB) * TB + (n % TB)]
                       : Zp[tile_of(J, I, nT) * TB * TB + (n % TB) * TB + (m % TB)];
        }
        __bf16 h0, l0, h1, l1;
        split_bf16(float(z.x), h0, l0);
        split_bf16(float(z.y), h1, l1);
        hi[2 * e] = h0;
        hi[2 * e + 1] = h1;
        lo[2 * e] = l0;
        lo[2 * e + 1] = l1;
    }
    const int64_t off = tile * 512 + (threadIdx.x & 63) * 8;
    *reinterpret_cast<bf16x8 *>(Ah + off) = hi;
    *reinterpret_cast<bf16x8 *>(Al + off) = lo;
}

// A planes from a dense complex128 N x N matrix, column-major (entry (m, n) at
// n N + m), zero padding; one wave per tile as above.
__global__ __launch_bounds__(256) void k_split_dense(const double2 *__restrict__ A, int64_t N, int64_t Mp, int64_t Kp,
                                                     __bf16 *__restrict__ Ah, __bf16 *__restrict__ Al)
{
    const int64_t nst = Kp / GBK, tile = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (tile >= (Mp / 32) * nst) return;
    int r, h;
    slot_owner(threadIdx.x & 63, r, h);
    const int64_t m = (tile / nst) * 32 + r, n0 = (tile % nst) * 8 + h * 4;
    bf16x8 hi, lo;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t n = n0 + e;
        const double2 z = (m < N && n < N) ? A[n * N + m] : make_double2(0.0, 0.0);
        __bf16 h0, l0, h1, l1;
        split_bf16(float(z.x), h0, l0);
        split_bf16(float(z.y), h1, l1);
        hi[2 * e] = h0;
        hi[2 * e + 1] = h1;
        lo[2 * e] = l0;
        lo[2 * e + 1] = l1;
    }
    const int64_t off = tile * 512 + (threadIdx.x & 63) * 8;
    *reinterpret_cast<bf16x8 *>(Ah + off) = hi;
    *reinterpret_cast<bf16x8 *>(Al + off) = lo;
}

// B planes (tiled, [NCp / 32][Kp / 16] tiles) from R complex vectors
// (complex128, complex64 or FP16 pairs XT): GEMM column pair r reads the vector at X + v*ldx,
// v = cols ? cols[r] : r.  One wave per tile.
template <typename XT>
__global__ __launch_bounds__(256) void k_split_vectors(const XT *__restrict__ X, int64_t ldx, const int *__restrict__ cols,
                                                       int64_t N, int64_t R, int64_t NCp, int64_t Kp,
                                                       __bf16 *__restrict__ Bh, __bf16 *__restrict__ Bl, bool lo)
{
    const int64_t nst = Kp / GBK, tile = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (tile >= (NCp / 32) * nst) return;
    int r, h;
    slot_owner(threadIdx.x & 63, r, h);
    const int64_t c = (tile / nst) * 32 + r, n0 = (tile % nst) * 8 + h * 4;
    const bool live = c < 2 * R;
    const int64_t v = live ? (cols ? int64_t(cols[c >> 1]) : (c >> 1)) : 0;
    bf16x8 hi, lw;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t n = n0 + e;
        float a = 0.f, b = 0.f;
        if (live && n < N) {
            const XT x = X[v * ldx + n];
            if (!(c & 1)) { a = float(x.x); b = float(-x.y); }
            else { a = float(x.y); b = float(x.x); }
        }
        __bf16 h0, l0, h1, l1;
        split_bf16(a, h0, l0);
        split_bf16(b, h1, l1);
        hi[2 * e] = h0;
        hi[2 * e + 1] = h1;
        lw[2 * e] = l0;
        lw[2 * e + 1] = l1;
    }
    const int64_t off = tile * 512 + (threadIdx.x & 63) * 8;
    *reinterpret_cast<bf16x8 *>(Bh + off) = hi;
    if (lo) *reinterpret_cast<bf16x8 *>(Bl + off) = lw;
}

// vmcnt(N) and lgkmcnt(0) in one wait (expcnt not waited on)
template <int N> __device__ inline void wait_vm_lds()
{
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt(0x070 | (N & 15) | ((N >> 4) << 14));
}

// Workgroup barrier without a memory fence: the LDS DMA completions it must
// order are waited for explicitly (wait_vm_lds) by every wave before it.  The
// empty asm statements keep the compiler from moving memory accesses across.
__device__ inline void block_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// 16 bytes per lane from global memory into LDS at l + 16 * lane (l uniform).
__device__ inline void lds_dma16(const void *g, void *l)
{
    __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void *)l, 16, 0, 0);
}

// Partial C = Ah Bh + Al Bh (+ Ah Bl when TERMS == 3) over the stages of one K
// slice, into P[z][Mp][NCp].  TERMS == 2 keeps the matrix split (about 16
// significant bits) and rounds the vectors to BF16 (2^-9 relative): the form
// for the inner corrections of iterative refinement, whose tolerance is far
// above that rounding; the B lo plane is then not loaded.
template <int TERMS, int WM, int WN, int NS>
__global__ __launch_bounds__(64 * (GBM / WM) * (GBN / WN)) void k_gemm_split(
    const __bf16 *__restrict__ Ah, const __bf16 *__restrict__ Al, const __bf16 *__restrict__ Bh,
    const __bf16 *__restrict__ Bl, int64_t Kp, int64_t Mp, int64_t NCp, float *__restrict__ P)
{
    constexpr int TIw = WM / 32, TJw = WN / 32, NWN = GBN / WN, W = (GBM / WM) * (GBN / WN);
    constexpr int SA = GBM / 32, SB = GBN / 32;                  // tiles of A and of B per plane and stage
    constexpr int LOADS = 2 * SA + (TERMS == 3 ? 2 : 1) * SB;   // DMA instructions per stage
    static_assert(LOADS % W == 0 && NS >= 3, "stage loads are shared evenly by the waves");
    constexpr int LPW = LOADS / W;
    constexpr int STAGE = (2 * SA + 2 * SB) * 512;              // BF16 per stage buffer
    __shared__ __attribute__((aligned(1024))) __bf16 lds[NS][STAGE];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = wave / NWN, wn = wave % NWN;
    unsigned bx, by, bz;
    xcd_tile(bx, by, bz);
    const int64_t m0 = int64_t(bx) * GBM, c0 = int64_t(by) * GBN;
    const int64_t nst = Kp / GBK;

    // the DMA instructions of this wave: tile q of the stage, its source (stage
    // 0) and its place in the stage buffer
    const __bf16 *src[LPW];
    int dst[LPW];
#pragma unroll
    for (int q = 0; q < LPW; ++q) {
        const int i = wave + W * q;
        if (i < 2 * SA) {
            const int p = i / SA, t = i % SA;
            src[q] = (p ? Al : Ah) + (m0 / 32 + t) * nst * 512;
            dst[q] = (p * SA + t) * 512;
        } else {
            const int j = i - 2 * SA, p = j / SB, t = j % SB;
            src[q] = (p ? Bl : Bh) + (c0 / 32 + t) * nst * 512;
            dst[q] = (2 * SA + p * SB + t) * 512;
        }
    }
    const int64_t sb = nst * bz / gridDim.z, n = nst * (bz + 1) / gridDim.z - sb;
    auto issue = [&](int64_t st, int buf) {
#pragma unroll
        for (int q = 0; q < LPW; ++q) lds_dma16(src[q] + (sb + st) * 512 + lane * 8, &lds[buf][dst[q]]);
    };

    f32x16 acc[TIw][TJw];
#pragma unroll
    for (int i = 0; i < TIw; ++i)
#pragma unroll
        for (int j = 0; j < TJw; ++j)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[i][j][q] = 0.f;

    const int fr = lane & 31, foff = tile_slot(fr, lane >> 5) * 8;
    const int aoff = (wm * WM / 32) * 512 + foff, boff = (2 * SA + wn * WN / 32) * 512 + foff;
    bf16x8 xa[TIw][2], xb[TJw][2], ya[TIw][2], yb[TJw][2];   // [tile][plane], two register sets
    auto fetch = [&](int buf, bf16x8 (&fa)[TIw][2], bf16x8 (&fb)[TJw][2]) {
        const __bf16 *L = &lds[buf][0];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
#pragma unroll
            for (int t = 0; t < TIw; ++t) fa[t][p] = *reinterpret_cast<const bf16x8 *>(L + aoff + (p * SA + t) * 512);
            if (TERMS == 3 || p == 0)
#pragma unroll
                for (int t = 0; t < TJw; ++t)
                    fb[t][p] = *reinterpret_cast<const bf16x8 *>(L + boff + (p * SB + t) * 512);
        }
    };
    // the products, each over the independent accumulators
    auto mfma = [&](const bf16x8 (&fa)[TIw][2], const bf16x8 (&fb)[TJw][2]) {
#pragma unroll
        for (int i = 0; i < TIw; ++i)
#pragma unroll
            for (int j = 0; j < TJw; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i][0], fb[j][0], acc[i][j], 0, 0, 0);
        if (TERMS == 3)
#pragma unroll
            for (int i = 0; i < TIw; ++i)
#pragma unroll
                for (int j = 0; j < TJw; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i][0], fb[j][1], acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < TIw; ++i)
#pragma unroll
            for (int j = 0; j < TJw; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i][1], fb[j][0], acc[i][j], 0, 0, 0);
    };
    // step i while stage i + NS exists: stages i+1 .. i+NS-1 are in flight;
    // wait for i+1 (its NS-2 successors may stay outstanding)
    auto steady = [&](int64_t i, const bf16x8 (&fa)[TIw][2], const bf16x8 (&fb)[TJw][2], bf16x8 (&ga)[TIw][2],
                      bf16x8 (&gb)[TJw][2]) {
        __builtin_amdgcn_sched_barrier(0);
        wait_vm_lds<(NS - 2) * LPW>();
        block_barrier();
        issue(i + NS, int(i % NS));
        fetch(int((i + 1) % NS), ga, gb);
        __builtin_amdgcn_sched_barrier(0);
        mfma(fa, fb);
    };
    // the last steps: wait for everything in flight
    auto tail = [&](int64_t i, const bf16x8 (&fa)[TIw][2], const bf16x8 (&fb)[TJw][2], bf16x8 (&ga)[TIw][2],
                    bf16x8 (&gb)[TJw][2]) {
        __builtin_amdgcn_sched_barrier(0);
        wait_vm_lds<0>();
        block_barrier();
        if (i + NS < n) issue(i + NS, int(i % NS));
        if (i + 1 < n) fetch(int((i + 1) % NS), ga, gb);
        __builtin_amdgcn_sched_barrier(0);
        mfma(fa, fb);
    };

    if (n >= NS) {
#pragma unroll
        for (int d = 0; d < NS; ++d) issue(d, d);
        wait_vm_lds<(NS - 1) * LPW>();
    } else {
        for (int64_t d = 0; d < n; ++d) issue(d, int(d));
        wait_vm_lds<0>();
    }
    block_barrier();
    if (n > 0) fetch(0, xa, xb);
    int64_t i = 0;
    for (; i + 1 + NS < n; i += 2) {   // two steps per trip: the register sets swap roles
        steady(i, xa, xb, ya, yb);
        steady(i + 1, ya, yb, xa, xb);
    }
    for (; i < n; i += 2) {
        tail(i, xa, xb, ya, yb);
        if (i + 1 < n) tail(i + 1, ya, yb, xa, xb);
    }

    // accumulator q of lane l holds row 8(q/4) + 4(l/32) + q%4, column l%32 of its 32x32 tile
    float *Pz = P + int64_t(bz) * Mp * NCp;
#pragma unroll
    for (int i2 = 0; i2 < TIw; ++i2)
#pragma unroll
        for (int j = 0; j < TJw; ++j) {
            const int64_t c = c0 + wn * WN + j * 32 + (lane & 31);
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int64_t m = m0 + wm * WM + i2 * 32 + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
                Pz[m * NCp + c] = acc[i2][j][q];
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

int env_int(const char *name, int def)
{
    const char *e = getenv(name);
    return e ? atoi(e) : def;
}

// Slices of K per launch: enough blocks for the 256 compute units, at least
// 8 stages per slice (the default; the autotuner also tries half and twice);
// BIE_GEMM_SPLITK overrides (measurement).
int gemm_splitk(int64_t blocks, int64_t nst, int want = 0)
{
    static const int env = env_int("BIE_GEMM_SPLITK", 0);
    int64_t ks = want > 0 ? want : (env > 0 ? env : std::max<int64_t>(1, 256 / blocks));
    ks = std::min<int64_t>(ks, std::max<int64_t>(1, nst / 8));
    return int(std::max<int64_t>(1, std::min<int64_t>(ks, 64)));
}

template <int WM, int WN, int NS>
void launch_split(int terms, dim3 grid, hipStream_t s, const __bf16 *Ah, const __bf16 *Al, const __bf16 *Bh,
                  const __bf16 *Bl, int64_t Kp, int64_t Mp, int64_t NCp, float *P)
{
    constexpr int NT = 64 * (GBM / WM) * (GBN / WN);
    if (terms == 3)
        hipLaunchKernelGGL((k_gemm_split<3, WM, WN, NS>), grid, dim3(NT), 0, s, Ah, Al, Bh, Bl, Kp, Mp, NCp, P);
    else
        hipLaunchKernelGGL((k_gemm_split<2, WM, WN, NS>), grid, dim3(NT), 0, s, Ah, Al, Bh, Bl, Kp, Mp, NCp, P);
}

typedef void (*SplitLaunch)(int, dim3, hipStream_t, const __bf16 *, const __bf16 *, const __bf16 *, const __bf16 *,
                            int64_t, int64_t, int64_t, float *);
// wave tiles of the 256 x 256 block: 128 x 64 (default), 64 x 128, 128 x 128
// (accumulators in AGPRs); BIE_GEMM_CFG = 0, 1, 2 fixes one (measurement),
// else the autotuner picks per shape
const SplitLaunch kSplitLaunch[] = { launch_split<128, 64, 4>, launch_split<64, 128, 4>, launch_split<128, 128, 4> };
constexpr int kSplitCfgs = int(sizeof(kSplitLaunch) / sizeof(kSplitLaunch[0]));

int split_cfg_env()
{
    static const int v = env_int("BIE_GEMM_CFG", -1);
    return v >= 0 && v < kSplitCfgs ? v : -1;
}

// Wave-tile form and K slices of a split-BF16 product of this shape: the
// environment's if set; else the autotuner's choice for (Mp, Kp, NCp, terms),
// timing every form with the default, half and twice the default K slices on
// the staged operands the first time the shape occurs (not while the stream is
// being captured); else the defaults.
void split_choice(int64_t Mp, int64_t Kp, int64_t NCp, int terms, hipStream_t s, const __bf16 *Ah, const __bf16 *Al,
                  const __bf16 *Bh, const __bf16 *Bl, bie_op *op, int &cfg, int &ks)
{
    const int64_t blocks = (Mp / GBM) * (NCp / GBN), nst = Kp / GBK;
    cfg = split_cfg_env();
    ks = gemm_splitk(blocks, nst);
    const bool env_fixed = cfg >= 0 || env_int("BIE_GEMM_SPLITK", 0) > 0;
    if (cfg < 0) cfg = 0;
    if (env_fixed || !tune_enabled()) return;
    const std::string key = "gemm_split:" + std::to_string(Mp) + "x" + std::to_string(Kp) + ":" +
                            std::to_string(NCp) + ":t" + std::to_string(terms);
    std::vector<int> v;
    const bool have = tune_get(key, v) && v.size() == 2 && v[0] >= 0 && v[0] < kSplitCfgs && v[1] >= 1;
    if (!have && stream_capturing(s)) return;   // no timing inside a captured graph: the defaults
    if (!have) {
        std::vector<int> kss;
        for (int want : { ks / 2, ks, 2 * ks }) {
            const int k2 = gemm_splitk(blocks, nst, std::max(1, want));
            if (std::find(kss.begin(), kss.end(), k2) == kss.end()) kss.push_back(k2);
        }
        const int kmax = *std::max_element(kss.begin(), kss.end());
        const size_t pelems = size_t(kmax) * size_t(Mp) * size_t(NCp);
        if (op->gemm_part_elems < pelems) {
            BIE_HIP(hipStreamSynchronize(s));
            if (op->gemm_part) (void)hipFree(op->gemm_part);
            op->gemm_part = nullptr;
            op->gemm_part_elems = 0;
            BIE_HIP(hipMalloc(&op->gemm_part, pelems * sizeof(float)));
            op->gemm_part_elems = pelems;
        }
        float *P = static_cast<float *>(op->gemm_part);
        float best = 0.f;
        v = { 0, ks };
        for (int c = 0; c < kSplitCfgs; ++c)
            for (int k2 : kss) {
                // the split-K reduction reads KS partial tiles: charged at 5 TB/s
                const float red = float(double(k2) * Mp * NCp * 4.0 / 5e12 * 1e3);
                const float ms = time_launches(s, 2, [&]() {
                    kSplitLaunch[c](terms, dim3(unsigned(Mp / GBM), unsigned(NCp / GBN), unsigned(k2)), s, Ah, Al, Bh,
                                    Bl, Kp, Mp, NCp, P);
                }) + red;
                if (best == 0.f || ms < best) {
                    best = ms;
                    v = { c, k2 };
                }
            }
        tune_put(key, v);
    }
    cfg = v[0];
    ks = v[1];
}

}  // namespace

int64_t gemm_pad_rows(int64_t N) { return (N + GBM - 1) / GBM * GBM; }
int64_t gemm_pad_k(int64_t N) { return (2 * N + GBK - 1) / GBK * GBK; }
int64_t gemm_pad_cols(int64_t R) { return (2 * R + GBN - 1) / GBN * GBN; }

// Split-BF16 copy of the FP64 matrix (A planes, hi then lo, tiled).
void split_matrix(bie_op *op, hipStream_t s)
{
    const int64_t N = op->mesh.N, Mp = gemm_pad_rows(N), Kp = gemm_pad_k(N);
    const size_t plane = size_t(Mp) * size_t(Kp);
    BIE_HIP(hipMalloc(&op->Abf, 2 * plane * sizeof(__bf16)));
    op->gemm_Mp = Mp;
    op->gemm_Kp = Kp;
    __bf16 *Ah = static_cast<__bf16 *>(op->Abf), *Al = Ah + plane;
    const int64_t tiles = (Mp / 32) * (Kp / GBK);
    hipLaunchKernelGGL(k_split_matrix, dim3(unsigned((tiles + 3) / 4)), dim3(256), 0, s, (const double2 *)op->Z64, N,
                       op->pk.nT, Mp, Kp, Ah, Al);
    BIE_HIP(hipGetLastError());
    BIE_HIP(hipStreamSynchronize(s));
}

// Y = T X (or Bsub - T X) for R vectors with the split-BF16 matrix; X
// complex128, complex64 or FP16 pairs (vtype), Y and Bsub complex128; cols
// (device, R entries, or null for 0..R-1) names the vectors taking part.
void gemm_product(const bie_op *opc, const void *X, int64_t ldx, int vtype, void *Y, int64_t ldy, const void *Bsub,
                  int64_t ldb, int64_t R, const int *cols, hipStream_t s, int terms)
{
    if (terms != 2 && terms != 3) throw Error(BIE_EINVAL, "the split-BF16 product has 2 or 3 terms");
    if (R <= 0) return;
    bie_op *op = const_cast<bie_op *>(opc);
    const int64_t N = op->mesh.N, Kp = op->gemm_Kp, Mp = op->gemm_Mp, NCp = gemm_pad_cols(R);
    const size_t plane = size_t(NCp) * size_t(Kp);
    if (op->bstage_cols < NCp) {
        if (stream_capturing(s))
            throw Error(BIE_EINVAL, "split-BF16 product: vector staging for " + std::to_string(NCp) + " columns (have " +
                                        std::to_string(op->bstage_cols) + ", N " + std::to_string(N) +
                                        ") cannot grow inside a captured graph");
        BIE_HIP(hipStreamSynchronize(s));
        if (op->Bbf) (void)hipFree(op->Bbf);
        op->Bbf = nullptr;
        op->bstage_cols = 0;
        BIE_HIP(hipMalloc(&op->Bbf, 2 * plane * sizeof(__bf16)));
        op->bstage_cols = NCp;
    }
    __bf16 *Bh = static_cast<__bf16 *>(op->Bbf), *Bl = Bh + plane;
    const __bf16 *Ah = static_cast<const __bf16 *>(op->Abf), *Al = Ah + size_t(Mp) * size_t(Kp);
    const int64_t btiles = (NCp / 32) * (Kp / GBK);
    const dim3 sgrid(unsigned((btiles + 3) / 4));
    if (vtype == VEC_F16)
        hipLaunchKernelGGL(k_split_vectors<c32h>, sgrid, dim3(256), 0, s, (const c32h *)X, ldx, cols, N, R, NCp, Kp,
                           Bh, Bl, terms == 3);
    else if (vtype == VEC_C64)
        hipLaunchKernelGGL(k_split_vectors<float2>, sgrid, dim3(256), 0, s, (const float2 *)X, ldx, cols, N, R, NCp,
                           Kp, Bh, Bl, terms == 3);
    else
        hipLaunchKernelGGL(k_split_vectors<double2>, sgrid, dim3(256), 0, s, (const double2 *)X, ldx, cols, N, R, NCp,
                           Kp, Bh, Bl, terms == 3);
    int cfg = 0, KS = 1;
    split_choice(Mp, Kp, NCp, terms, s, Ah, Al, Bh, Bl, op, cfg, KS);
    const size_t pelems = size_t(KS) * size_t(Mp) * size_t(NCp);
    if (op->gemm_part_elems < pelems) {
        if (stream_capturing(s))
            throw Error(BIE_EINVAL, "split-BF16 product: partial sums of " + std::to_string(pelems) + " (have " +
                                        std::to_string(op->gemm_part_elems) + ", K slices " + std::to_string(KS) +
                                        ", N " + std::to_string(N) + ") cannot grow inside a captured graph");
        BIE_HIP(hipStreamSynchronize(s));
        if (op->gemm_part) (void)hipFree(op->gemm_part);
        op->gemm_part = nullptr;
        op->gemm_part_elems = 0;
        BIE_HIP(hipMalloc(&op->gemm_part, pelems * sizeof(float)));
        op->gemm_part_elems = pelems;
    }
    float *P = static_cast<float *>(op->gemm_part);
    prof_begin(1, s, R);
    kSplitLaunch[cfg](terms, dim3(unsigned(Mp / GBM), unsigned(NCp / GBN), unsigned(KS)), s, Ah, Al, Bh, Bl, Kp, Mp,
                      NCp, P);
    prof_end(1, s);
    hipLaunchKernelGGL(k_gemm_reduce<float>, dim3(unsigned(Mp / 64), unsigned(NCp / 64)), dim3(256), 0, s, P, KS, Mp,
                       NCp, N, R, cols, (double2 *)Y, ldy, (const double2 *)Bsub, ldb);
    BIE_HIP(hipGetLastError());
}

// Split-BF16 operand of a general (not symmetric) dense complex128 matrix A
// (column-major, N = op->mesh.N), for gemm_product on op.
void split_dense(bie_op *op, const void *A, hipStream_t s)
{
    const int64_t N = op->mesh.N, Mp = gemm_pad_rows(N), Kp = gemm_pad_k(N);
    const size_t plane = size_t(Mp) * size_t(Kp);
    BIE_HIP(hipMalloc(&op->Abf, 2 * plane * sizeof(__bf16)));
    op->gemm_Mp = Mp;
    op->gemm_Kp = Kp;
    __bf16 *Ah = static_cast<__bf16 *>(op->Abf), *Al = Ah + plane;
    const int64_t tiles = (Mp / 32) * (Kp / GBK);
    hipLaunchKernelGGL(k_split_dense, dim3(unsigned((tiles + 3) / 4)), dim3(256), 0, s, (const double2 *)A, N, Mp, Kp,
                       Ah, Al);
    BIE_HIP(hipGetLastError());
    BIE_HIP(hipStreamSynchronize(s));
}

// Dense FP64 copy of the packed matrix for the FP64 block product.
void dense64_setup(bie_op *op, hipStream_t s)
{
    if (op->A64) return;
    const int64_t N = op->mesh.N, Mp = (N + DBM - 1) / DBM * DBM, Kp = (2 * N + DBK - 1) / DBK * DBK;
    if (op->pooled) op->A64 = setup_pool_get(2, size_t(Mp) * size_t(Kp) * sizeof(double));
    else BIE_HIP(hipMalloc(&op->A64, size_t(Mp) * size_t(Kp) * sizeof(double)));
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
    if (R <= 0) return;
    bie_op *op = const_cast<bie_op *>(opc);
    if (!op->Z64) throw Error(BIE_EINVAL, "the FP64 block product needs the FP64 matrix");
    dense64_setup(op, s);
    const int64_t N = op->mesh.N, Mp = op->d64_Mp, Kp = op->d64_Kp, NCp = (2 * R + DBN - 1) / DBN * DBN;
    const int64_t blocks = (Mp / DBM) * (NCp / DBN), nst = Kp / DBK;
    auto clampks = [&](int64_t want) { return std::max<int64_t>(1, std::min<int64_t>({ want, nst / 16, 64 })); };
    int64_t ks = clampks(std::max<int64_t>(1, 256 / blocks));
    // K slices: the autotuner's choice for (Mp, Kp, NCp) among half, the
    // default and twice the default, timed the first time the shape occurs
    if (tune_enabled() && !stream_capturing(s)) {
        const std::string key = "gemm64:" + std::to_string(Mp) + "x" + std::to_string(Kp) + ":" + std::to_string(NCp);
        std::vector<int> v;
        if (!tune_get(key, v) || v.size() != 1 || v[0] < 1) {
            std::vector<int64_t> kss;
            for (int64_t want : { ks / 2, ks, 2 * ks }) {
                const int64_t k2 = clampks(std::max<int64_t>(1, want));
                if (std::find(kss.begin(), kss.end(), k2) == kss.end()) kss.push_back(k2);
            }
            const size_t pmax = size_t(*std::max_element(kss.begin(), kss.end())) * size_t(Mp) * size_t(NCp);
            if (op->d64_part_elems < pmax) {
                BIE_HIP(hipStreamSynchronize(s));
                if (op->d64_part) (void)hipFree(op->d64_part);
                op->d64_part = nullptr;
                op->d64_part_elems = 0;
                BIE_HIP(hipMalloc(&op->d64_part, pmax * sizeof(double)));
                op->d64_part_elems = pmax;
            }
            double *Pt = static_cast<double *>(op->d64_part);
            float best = 0.f;
            v = { int(ks) };
            for (int64_t k2 : kss) {
                const float red = float(double(k2) * Mp * NCp * 8.0 / 5e12 * 1e3);
                const float ms = time_launches(s, 2, [&]() {
                    hipLaunchKernelGGL(k_gemm64, dim3(unsigned(Mp / DBM), unsigned(NCp / DBN), unsigned(k2)), dim3(256), 0,
                                       s, (const double *)op->A64, Kp, N, (const double2 *)X, ldx, cols, R, Mp, NCp, Pt);
                }) + red;
                if (best == 0.f || ms < best) {
                    best = ms;
                    v = { int(k2) };
                }
            }
            tune_put(key, v);
        }
        ks = clampks(v[0]);
    }
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
