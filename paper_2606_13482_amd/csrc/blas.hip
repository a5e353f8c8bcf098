// Products with the dense impedance matrix in packed symmetric storage.
//
// The matrix-vector product is the O(N^2) operation of every Krylov
// iteration (Sec. I and II: dense storage and MVP cost).  The Galerkin EFIE
// matrix is symmetric (identical test and basis functions), and the fill makes
// it exactly so, which halves the bytes a product must stream: only the tiles
// (I, J), I <= J, of 64 x 64 entries are stored.  One pass over the tiles
// applies every off-diagonal tile twice,
//     y_I += T_IJ x_J     (row sums, kept in registers along a tile row)
//     y_J += T_IJ^T x_I   (column sums, one 64-entry partial per tile),
// and a second small kernel adds the partials of each 64-row block in a fixed
// order (deterministic, no atomics).
//
// Tile pass: one block of 4 waves walks a run of consecutive tiles of one tile
// row; wave w owns rows 16w..16w+15 of the row block, lane c owns column c.
// Every tile row (1 KiB in FP64) is read by one wave with one load per lane,
// 16 rows in flight per wave, and the next tile's loads are issued before the
// current tile's arithmetic.  Column sums of the 4 waves are combined through
// double-buffered LDS with one barrier per tile; x of the wave's 16 rows sits in
// scalar registers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <utility>
#include <mutex>
#include <string>
#include <vector>

#include "bie_internal.hpp"

namespace bie {

// Optional timing of the dense product kernels: events recorded on the launch
// stream around every launch (record 0: tile pass of the packed FP64/FP32
// product, 1: split-BF16 block product, 2: FP64 block product, 3: reduction of
// the packed product's partial sums, 4: block GMRES basis dots, 5: block GMRES
// basis update).
namespace prof {
bool on = false;
struct Rec {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    size_t used = 0;
    int64_t cols = 0;   // right-hand sides over the recorded launches
};
Rec rec[10];

void begin(int k, hipStream_t s, int64_t ncols)
{
    if (!on) return;
    Rec &r = rec[k];
    r.cols += ncols;
    if (r.used == r.ev.size()) {
        hipEvent_t a, b;
        BIE_HIP(hipEventCreate(&a));
        BIE_HIP(hipEventCreate(&b));
        r.ev.emplace_back(a, b);
    }
    BIE_HIP(hipEventRecord(r.ev[r.used].first, s));
}
void end(int k, hipStream_t s)
{
    if (!on) return;
    Rec &r = rec[k];
    BIE_HIP(hipEventRecord(r.ev[r.used].second, s));
    ++r.used;
}
}  // namespace prof

void prof_enable(bool enable) { prof::on = enable; }
bool prof_active() { return prof::on; }
void prof_begin(int kernel, hipStream_t s, int64_t ncols) { prof::begin(kernel, s, ncols); }
void prof_end(int kernel, hipStream_t s) { prof::end(kernel, s); }

void prof_read(int kernel, int64_t *launches, double *total_ms, int64_t *columns)
{
    if (kernel < 0 || kernel > 9) throw Error(BIE_EINVAL, "unknown kernel record");
    prof::Rec &r = prof::rec[kernel];
    double t = 0.0;
    for (size_t i = 0; i < r.used; ++i) {
        BIE_HIP(hipEventSynchronize(r.ev[i].second));
        float ms = 0.f;
        BIE_HIP(hipEventElapsedTime(&ms, r.ev[i].first, r.ev[i].second));
        t += ms;
    }
    *launches = int64_t(r.used);
    *total_ms = t;
    if (columns) *columns = r.cols;
    r.used = 0;
    r.cols = 0;
}

namespace {

// Work of the single-operator tile pass: units of 8 tiles, one per block
// (default); BIE_SYM_UNIT = 1..64 selects another unit length, 0 balanced runs
// (measurement: at N = 7680 both take the same time, and on the small
// matrices of the uneven batch the runs were slower).
int unit_tiles()
{
    static int v = [] {
        const char *e = getenv("BIE_SYM_UNIT");
        const int u = e ? atoi(e) : 8;
        return u >= 0 && u <= 64 ? u : 8;
    }();
    return v;
}

typedef double nd2 __attribute__((ext_vector_type(2)));
typedef float nf2 __attribute__((ext_vector_type(2)));

template <typename T>
struct Cx;   // complex element as a native 2-vector (one load instruction)
template <>
struct Cx<double> {
    using type = nd2;
};
template <>
struct Cx<float> {
    using type = nf2;
};

template <typename T>
__device__ inline T wsum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sums 8 complex values over a wave: each exchange halves what a lane carries
// (4+2+1 exchanges, then 3 plain steps).  pr[0], pi[0] of lane L end with the
// total of value (L >> 3) & 7.
template <typename T>
__device__ inline void wave_sum8(T pr[8], T pi[8])
{
    const int lane = threadIdx.x & 63;
    {
        const bool b = lane & 32;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const T sr = b ? pr[i] : pr[i + 4], si = b ? pi[i] : pi[i + 4];
            const T kr = b ? pr[i + 4] : pr[i], ki = b ? pi[i + 4] : pi[i];
            pr[i] = kr + __shfl_xor(sr, 32, 64);
            pi[i] = ki + __shfl_xor(si, 32, 64);
        }
    }
    {
        const bool b = lane & 16;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const T sr = b ? pr[i] : pr[i + 2], si = b ? pi[i] : pi[i + 2];
            const T kr = b ? pr[i + 2] : pr[i], ki = b ? pi[i + 2] : pi[i];
            pr[i] = kr + __shfl_xor(sr, 16, 64);
            pi[i] = ki + __shfl_xor(si, 16, 64);
        }
    }
    {
        const bool b = lane & 8;
        const T sr = b ? pr[0] : pr[1], si = b ? pi[0] : pi[1];
        const T kr = b ? pr[1] : pr[0], ki = b ? pi[1] : pi[0];
        pr[0] = kr + __shfl_xor(sr, 8, 64);
        pi[0] = ki + __shfl_xor(si, 8, 64);
    }
#pragma unroll
    for (int o = 4; o > 0; o >>= 1) {
        pr[0] += __shfl_xor(pr[0], o, 64);
        pi[0] += __shfl_xor(pi[0], o, 64);
    }
}

// Tile pass of one work unit: tiles (I, J0 .. J1-1) of row block I, the
// unit being the uo-th of its row.  Writes 64-entry partial vectors (complex
// T) into the slots of the row block they belong to (see reduce_rows).
// M: matrix storage type, T: vector and accumulation type (T >= M).  NT:
// non-temporal tile loads (one vector streams the matrix once; several
// vectors re-read the unit's tiles from the caches).
template <typename M, typename T, bool CONJ, bool PREFETCH, bool NT = true>
__device__ __forceinline__ void tile_pass(const M *__restrict__ Zp, int64_t N, int64_t nT, int32_t I, int32_t J0, int32_t J1,
                                 int64_t uo, const int64_t *__restrict__ seg,
                                 const typename Cx<T>::type *__restrict__ x, typename Cx<T>::type *__restrict__ pv)
{
    using V2 = typename Cx<T>::type;
    using MV = typename Cx<M>::type;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: x rows in scalar registers
    // partials of row block K live in slots seg[K]..: first the column sums of
    // tiles (0..K-1, K), then the row sums of the units of tile row K
    const MV *Z = reinterpret_cast<const MV *>(Zp);

    // x of this wave's 16 rows (the same for every lane)
    T xir[16], xii[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int64_t m = int64_t(I) * TB + wave * 16 + i;
        V2 xv = { 0, 0 };
        if (m < N) xv = x[m];
        xir[i] = xv.x;
        xii[i] = xv.y;
    }
    T rar[16], rai[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) { rar[i] = 0; rai[i] = 0; }
    __shared__ V2 red[2][4][TB];

    // x_J of lane's column, loaded with the tile it multiplies (a load issued
    // just before its use would expose its latency once per tile)
    auto xcol = [&](int32_t J) {
        const int64_t n = int64_t(J) * TB + lane;
        V2 v = { 0, 0 };
        if (n < N) v = x[n];
        return v;
    };
    MV t[16];
    V2 xt = { 0, 0 };
    if (PREFETCH) {
        const MV *tile = Z + tile_of(I, J0, nT) * TB * TB + (wave * 16) * TB + lane;
#pragma unroll
        for (int i = 0; i < 16; ++i) t[i] = NT ? __builtin_nontemporal_load(tile + i * TB) : tile[i * TB];
        xt = xcol(J0);
    }
    for (int32_t J = J0; J < J1; ++J) {
        V2 xj;
        MV cur[16];
        if (PREFETCH) {
#pragma unroll
            for (int i = 0; i < 16; ++i) cur[i] = t[i];
            xj = xt;
            if (J + 1 < J1) {   // next tile's loads go out before this tile's arithmetic
                const MV *tile = Z + tile_of(I, J + 1, nT) * TB * TB + (wave * 16) * TB + lane;
#pragma unroll
                for (int i = 0; i < 16; ++i) t[i] = NT ? __builtin_nontemporal_load(tile + i * TB) : tile[i * TB];
                xt = xcol(J + 1);
            }
        } else {
            xj = xcol(J);
            const MV *tile = Z + tile_of(I, J, nT) * TB * TB + (wave * 16) * TB + lane;
#pragma unroll
            for (int i = 0; i < 16; ++i) cur[i] = NT ? __builtin_nontemporal_load(tile + i * TB) : tile[i * TB];
        }
        T car = 0, cai = 0;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const T zr = T(cur[i].x), zi = CONJ ? -T(cur[i].y) : T(cur[i].y);
            rar[i] += zr * xj.x - zi * xj.y;
            rai[i] += zr * xj.y + zi * xj.x;
            car += zr * xir[i] - zi * xii[i];
            cai += zr * xii[i] + zi * xir[i];
        }
        if (J != I) {   // uniform over the block
            // double-buffered by tile parity: one barrier per tile; the barrier of
            // the next tile orders this tile's reads before the buffer is reused
            const int par = (J - J0) & 1;
            red[par][wave][lane] = V2{ car, cai };
            __syncthreads();
            if (wave == ((J - J0) & 3)) {
                V2 a = red[par][0][lane];
#pragma unroll
                for (int w = 1; w < 4; ++w) a += red[par][w][lane];
                pv[(seg[J] + I) * TB + lane] = a;
            }
        }
    }
    // row sums: 16 values per wave, two groups of 8
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        T pr[8], pi[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) { pr[i] = rar[8 * g + i]; pi[i] = rai[8 * g + i]; }
        wave_sum8(pr, pi);
        if ((lane & 7) == 0) pv[(seg[I] + I + uo) * TB + wave * 16 + 8 * g + (lane >> 3)] = V2{ pr[0], pi[0] };
    }
}

// Tile pass over the units of one problem: block (run b, vector v) takes the
// units run_ptr[b] .. run_ptr[b+1]-1 in turn (a barrier between units: the
// LDS buffers of the column sums restart at parity 0).  At most 256 VGPRs:
// two blocks per CU.
template <typename M, typename T, bool CONJ, bool PREFETCH, bool NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_sym_tiles(const M *__restrict__ Zp, int64_t N, int64_t nT,
                                                   const int32_t *__restrict__ units,
                                                   const int32_t *__restrict__ unit_ptr,
                                                   const int32_t *__restrict__ run_ptr,
                                                   const int64_t *__restrict__ seg, int64_t nslots,
                                                   const T *__restrict__ X, int64_t ldx, T *__restrict__ part,
                                                   const int *__restrict__ skip, int64_t sks)
{
    using V2 = typename Cx<T>::type;
    const int64_t v = blockIdx.y;
    if (skip && skip[v * sks]) return;
    const int32_t u0 = run_ptr[blockIdx.x], u1 = run_ptr[blockIdx.x + 1];
    for (int32_t u = u0; u < u1; ++u) {
        if (u > u0) __syncthreads();
        const int32_t I = units[3 * u], J0 = units[3 * u + 1], J1 = units[3 * u + 2];
        tile_pass<M, T, CONJ, PREFETCH, NT>(Zp, N, nT, I, J0, J1, u - unit_ptr[I], seg,
                                        reinterpret_cast<const V2 *>(X) + v * ldx,
                                        reinterpret_cast<V2 *>(part) + v * nslots * TB);
    }
}

// a value known to be the same in every lane, moved to scalar registers
__device__ inline int64_t uniform64(int64_t v)
{
    const uint64_t u = uint64_t(v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(u)), hi = __builtin_amdgcn_readfirstlane(uint32_t(u >> 32));
    return int64_t((uint64_t(hi) << 32) | lo);
}

// Grouped tile pass over several problems: block b is the work item (problem
// p, unit u, column group g) and goes through columns c0 + gG .. of p in turn,
// skipping finished ones; the unit's tiles come from memory for the first
// column and from the caches for the others.  A barrier separates the columns:
// the column-sum buffers of the tile pass start again at parity 0, and the
// last tile's buffer may still be read by another wave.  Items are ordered
// longest first.
template <typename M, typename T, bool PREFETCH>
__global__ __launch_bounds__(256) void k_sym_tiles_g(const GProb *__restrict__ probs, GCols gc,
                                                     const int32_t *__restrict__ items, int G, const T *__restrict__ X,
                                                     T *__restrict__ part, const int *__restrict__ skip, int64_t sks)
{
    using V2 = typename Cx<T>::type;
    const int64_t b = blockIdx.x;
    const int32_t p = items[3 * b], u = items[3 * b + 1], g = items[3 * b + 2];
    const GProb P = probs[p];
    // values read through the tables' pointers are the same in every lane:
    // made scalar so that the tile pass keeps its row indices and x of the
    // tile rows in scalar registers, as in the single-operator pass
    const int32_t I = __builtin_amdgcn_readfirstlane(P.units[3 * u]);
    const int32_t J0 = __builtin_amdgcn_readfirstlane(P.units[3 * u + 1]);
    const int32_t J1 = __builtin_amdgcn_readfirstlane(P.units[3 * u + 2]);
    const int32_t uo = __builtin_amdgcn_readfirstlane(u - P.unit_ptr[I]);
    const int32_t cb = P.c0 + g * G, ce = min(P.c1, cb + G);
    bool first = true;
    for (int32_t c = cb; c < ce; ++c) {
        if (skip && skip[int64_t(c) * sks]) continue;   // uniform over the block
        if (!first) __syncthreads();
        first = false;
        const int64_t xo = uniform64(gc.xoff[c] + gc.xstep * P.N), po = uniform64(gc.poff[c] * TB);
        tile_pass<M, T, false, PREFETCH, false>(static_cast<const M *>(P.Z), P.N, P.nT, I, J0, J1, uo, P.seg,
                                                reinterpret_cast<const V2 *>(X) + xo,
                                                reinterpret_cast<V2 *>(part) + po);
    }
}

// Grouped tile pass on the FP32 matrix cores (batches certified by FP64
// residuals): block b is the work item (problem p, unit u, column group g of
// at most 32 columns, padded with zeros to 32).  Per tile (I, J) of the unit
// the complex products Y_I += Z X_J (rows of block I, accumulated over the
// unit) and, for J != I, Y_J = Z^T X_I (written per tile) are four real
// 32 x 32 x 2 chains of v_mfma_f32_32x32x2f32 per wave: wave w = 2 h + part
// computes rows (or tile columns) 32 h .. 32 h + 31 of the real (part 0) or the
// imaginary (part 1) output.  The tile (rows padded to 65 entries) and the two
// vector blocks are staged in LDS in FP32 (the vectors rounded from FP64);
// accumulation is FP32 within the unit; the partial vectors go to the same
// FP64 slots as the VALU tile pass's, so the same reduction sums them.
typedef float f32x16g __attribute__((ext_vector_type(16)));
typedef float f32x4g __attribute__((ext_vector_type(4)));
// Loads that name the global address space.  Pointers read from the problem
// table are generic, and a generic (flat) load also counts against the LDS wait
// counter: the waits for the LDS fragment reads would then wait for the next
// tile's prefetch as well.
typedef float gf2v __attribute__((ext_vector_type(2)));
typedef double gd2v __attribute__((ext_vector_type(2)));
__device__ inline float2 gload_f2(const float2 *p, int64_t i)
{
    const gf2v v = ((const __attribute__((address_space(1))) gf2v *)p)[i];
    return make_float2(v[0], v[1]);
}
__device__ inline double2 gload_d2(const double2 *p, int64_t i)
{
    const gd2v v = ((const __attribute__((address_space(1))) gd2v *)p)[i];
    return make_double2(v[0], v[1]);
}
__device__ inline int64_t gload_i64(const int64_t *p, int64_t i)
{
    return ((const __attribute__((address_space(1))) int64_t *)p)[i];
}

__global__ __launch_bounds__(256) void k_sym_tiles_gm(const GProb *__restrict__ probs, GCols gc,
                                                      const int32_t *__restrict__ items, int G,
                                                      const double *__restrict__ X, float *__restrict__ part,
                                                      const int *__restrict__ skip, int64_t sks)
{
    __shared__ float2 sZ[TB][TB + 1];
    __shared__ float2 sXI[TB][32];
    __shared__ float2 sXJ[TB][32];
    __shared__ int32_t live[32];
    const int64_t b = blockIdx.x;
    const int32_t p = items[3 * b], u = items[3 * b + 1], g = items[3 * b + 2];
    const GProb P = probs[p];
    const int32_t I = __builtin_amdgcn_readfirstlane(P.units[3 * u]);
    const int32_t J0 = __builtin_amdgcn_readfirstlane(P.units[3 * u + 1]);
    const int32_t J1 = __builtin_amdgcn_readfirstlane(P.units[3 * u + 2]);
    const int32_t uo = __builtin_amdgcn_readfirstlane(u - P.unit_ptr[I]);
    const int32_t cb = P.c0 + g * G, ce = min(min(P.c1, cb + G), cb + 32);
    const int nc = ce - cb;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, h = w >> 1, prt = w & 1, li = lane & 31, lk = lane >> 5;
    if (t < 32) live[t] = (t < nc && !(skip && skip[int64_t(cb + t) * sks])) ? 1 : 0;
    __syncthreads();
    int hi = 0;   // one past the last live column
    for (int c = 0; c < nc; ++c)
        if (live[c]) hi = c + 1;
    if (hi == 0) return;   // uniform over the block
    // at most 16 live leading columns: 16 x 16 products (half the matrix-core work)
    const bool narrow = hi <= 16;
    const float2 *Z = static_cast<const float2 *>(P.Z);
    const double2 *Xc = reinterpret_cast<const double2 *>(X);
    // staging: thread t always moves column t & 31 of the vectors (rows t/32 + 8 i)
    // and entries t + 256 i of the tile (row t/64 + 4 i, column t & 63)
    const int sc = t & 31, sr = t >> 5;
    const bool slive = live[sc] != 0;
    const int64_t sxo = slive ? gc.xoff[cb + sc] + gc.xstep * P.N : 0;
    auto load_x = [&](double2 (&xv)[8], int32_t blk) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t row = int64_t(blk) * TB + sr + 8 * q;
            xv[q] = (slive && row < P.N) ? gload_d2(Xc, sxo + row) : make_double2(0.0, 0.0);
        }
    };
    auto put_x = [&](float2 (*dst)[32], const double2 (&xv)[8]) {
#pragma unroll
        for (int q = 0; q < 8; ++q) dst[sr + 8 * q][sc] = make_float2(float(xv[q].x), float(xv[q].y));
    };
    auto load_z = [&](float2 (&zv)[16], int32_t J) {
        const float2 *tile = Z + tile_of(I, J, P.nT) * TB * TB + t;
#pragma unroll
        for (int q = 0; q < 16; ++q) zv[q] = gload_f2(tile, 256 * q);
    };
    auto put_z = [&](const float2 (&zv)[16]) {
#pragma unroll
        for (int q = 0; q < 16; ++q) sZ[(t >> 6) + 4 * q][t & 63] = zv[q];
    };
    // one real 32 x 32 output of the complex product over the 64 entries of k
    auto chain = [&](f32x16g acc, bool transposed, float2 (*xs)[32]) {
#pragma unroll 8
        for (int k0 = 0; k0 < TB; k0 += 2) {
            const float2 z = transposed ? sZ[k0 + lk][32 * h + li] : sZ[32 * h + li][k0 + lk];
            const float2 x = xs[k0 + lk][li];
            if (prt == 0) {
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(z.x, x.x, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(-z.y, x.y, acc, 0, 0, 0);
            } else {
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(z.x, x.y, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(z.y, x.x, acc, 0, 0, 0);
            }
        }
        return acc;
    };
    // value q of lane l: row 32 h + 8 (q / 4) + 4 (l / 32) + q % 4, column l % 32
    const bool olive = live[li] != 0;
    const int64_t opo = olive ? gc.poff[cb + li] * TB : 0;
    auto store = [&](const f32x16g &acc, int64_t slot) {
        if (!olive) return;
        float *pv = part + (opo + slot * TB) * 2 + prt;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int r = 32 * h + 8 * (q >> 2) + 4 * lk + (q & 3);
            pv[2 * r] = acc[q];
        }
    };
    // narrow form: wave w takes rows 16 w .. + 15 of the tile and both parts;
    // v_mfma_f32_16x16x4f32: A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k,
    // output value q of lane l at row 4 (l / 16) + q, column l % 16
    const int ni = lane & 15, nk = lane >> 4;
    auto chain16 = [&](f32x4g &ar, f32x4g &ai, bool transposed, float2 (*xs)[32]) {
#pragma unroll 4
        for (int k0 = 0; k0 < TB; k0 += 4) {
            const float2 z = transposed ? sZ[k0 + nk][16 * w + ni] : sZ[16 * w + ni][k0 + nk];
            const float2 x = xs[k0 + nk][ni];
            ar = __builtin_amdgcn_mfma_f32_16x16x4f32(z.x, x.x, ar, 0, 0, 0);
            ar = __builtin_amdgcn_mfma_f32_16x16x4f32(-z.y, x.y, ar, 0, 0, 0);
            ai = __builtin_amdgcn_mfma_f32_16x16x4f32(z.x, x.y, ai, 0, 0, 0);
            ai = __builtin_amdgcn_mfma_f32_16x16x4f32(z.y, x.x, ai, 0, 0, 0);
        }
    };
    const bool nlive = live[ni] != 0;
    const int64_t npo = nlive ? gc.poff[cb + ni] * TB : 0;
    auto store16 = [&](const f32x4g &ar, const f32x4g &ai, int64_t slot) {
        if (!nlive) return;
        float *pv = part + (npo + slot * TB) * 2;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = 16 * w + 4 * nk + q;
            pv[2 * r] = ar[q];
            pv[2 * r + 1] = ai[q];
        }
    };
    double2 xv[8];
    float2 zv[16];
    load_x(xv, I);
    put_x(sXI, xv);
    load_z(zv, J0);
    load_x(xv, J0);
    f32x16g arow;
    f32x4g nrr, nri;
#pragma unroll
    for (int q = 0; q < 16; ++q) arow[q] = 0.f;
#pragma unroll
    for (int q = 0; q < 4; ++q) nrr[q] = nri[q] = 0.f;
    for (int32_t J = J0; J < J1; ++J) {
        __syncthreads();   // the previous tile's LDS reads are done
        put_z(zv);
        put_x(sXJ, xv);
        __syncthreads();
        if (J + 1 < J1) {   // the next tile's loads go out before this tile's products
            load_z(zv, J + 1);
            load_x(xv, J + 1);
        }
        if (narrow) {
            chain16(nrr, nri, false, sXJ);
            if (J != I) {
                f32x4g cr, ci;
#pragma unroll
                for (int q = 0; q < 4; ++q) cr[q] = ci[q] = 0.f;
                chain16(cr, ci, true, sXI);
                store16(cr, ci, gload_i64(P.seg, J) + I);
            }
        } else {
            arow = chain(arow, false, sXJ);
            if (J != I) {
                f32x16g acol;
#pragma unroll
                for (int q = 0; q < 16; ++q) acol[q] = 0.f;
                acol = chain(acol, true, sXI);
                store(acol, gload_i64(P.seg, J) + I);
            }
        }
    }
    if (narrow) store16(nrr, nri, gload_i64(P.seg, I) + I + uo);
    else store(arow, gload_i64(P.seg, I) + I + uo);
}

// The same grouped pass on FP64 tiles with the FP64 matrix cores
// (v_mfma_f64_16x16x4f64: A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k,
// output value q of lane l at row l / 16 + 4 q, column l % 16 -- rows
// interleaved, unlike the FP32 16 x 16 x 4 form): wave w takes
// rows 16 w .. + 15 of the tile, both parts, and the item's columns in halves of
// 16 (one half when the live columns fit in it).  The tile (64 KB) and the two
// vector blocks stay FP64 in LDS; FP64 accumulation throughout.
typedef double f64x4g __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_sym_tiles_gm64(const GProb *__restrict__ probs, GCols gc,
                                                        const int32_t *__restrict__ items, int G,
                                                        const double *__restrict__ X, double *__restrict__ part,
                                                        const int *__restrict__ skip, int64_t sks)
{
    __shared__ double2 sZ[TB][TB + 1];
    __shared__ double2 sXI[TB][32];
    __shared__ double2 sXJ[TB][32];
    __shared__ int32_t live[32];
    const int64_t b = blockIdx.x;
    const int32_t p = items[3 * b], u = items[3 * b + 1], g = items[3 * b + 2];
    const GProb P = probs[p];
    const int32_t I = __builtin_amdgcn_readfirstlane(P.units[3 * u]);
    const int32_t J0 = __builtin_amdgcn_readfirstlane(P.units[3 * u + 1]);
    const int32_t J1 = __builtin_amdgcn_readfirstlane(P.units[3 * u + 2]);
    const int32_t uo = __builtin_amdgcn_readfirstlane(u - P.unit_ptr[I]);
    const int32_t cb = P.c0 + g * G, ce = min(min(P.c1, cb + G), cb + 32);
    const int nc = ce - cb;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, ni = lane & 15, nk = lane >> 4;
    if (t < 32) live[t] = (t < nc && !(skip && skip[int64_t(cb + t) * sks])) ? 1 : 0;
    __syncthreads();
    int hi = 0;
    for (int c = 0; c < nc; ++c)
        if (live[c]) hi = c + 1;
    if (hi == 0) return;   // uniform over the block
    const int halves = hi <= 16 ? 1 : 2;
    const double2 *Z = static_cast<const double2 *>(P.Z);
    const double2 *Xc = reinterpret_cast<const double2 *>(X);
    // staging as in the FP32 pass: column t & 31 of the vectors (rows t/32 + 8 i),
    // entries t + 256 i of the tile
    const int sc = t & 31, sr = t >> 5;
    const bool slive = live[sc] != 0;
    const int64_t sxo = slive ? gc.xoff[cb + sc] + gc.xstep * P.N : 0;
    auto load_x = [&](double2 (&xv)[8], int32_t blk) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t row = int64_t(blk) * TB + sr + 8 * q;
            xv[q] = (slive && row < P.N) ? gload_d2(Xc, sxo + row) : make_double2(0.0, 0.0);
        }
    };
    auto put_x = [&](double2 (*dst)[32], const double2 (&xv)[8]) {
#pragma unroll
        for (int q = 0; q < 8; ++q) dst[sr + 8 * q][sc] = xv[q];
    };
    auto load_z = [&](double2 (&zv)[16], int32_t J) {
        const double2 *tile = Z + tile_of(I, J, P.nT) * TB * TB + t;
#pragma unroll
        for (int q = 0; q < 16; ++q) zv[q] = gload_d2(tile, 256 * q);
    };
    auto put_z = [&](const double2 (&zv)[16]) {
#pragma unroll
        for (int q = 0; q < 16; ++q) sZ[(t >> 6) + 4 * q][t & 63] = zv[q];
    };
    auto chain = [&](f64x4g (&ar)[2], f64x4g (&ai)[2], bool transposed, double2 (*xs)[32]) {
        for (int k0 = 0; k0 < TB; k0 += 4) {
            const double2 z = transposed ? sZ[k0 + nk][16 * w + ni] : sZ[16 * w + ni][k0 + nk];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                if (c >= halves) break;
                const double2 x = xs[k0 + nk][16 * c + ni];
                ar[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(z.x, x.x, ar[c], 0, 0, 0);
                ar[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(-z.y, x.y, ar[c], 0, 0, 0);
                ai[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(z.x, x.y, ai[c], 0, 0, 0);
                ai[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(z.y, x.x, ai[c], 0, 0, 0);
            }
        }
    };
    auto store = [&](const f64x4g (&ar)[2], const f64x4g (&ai)[2], int64_t slot) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            if (c >= halves) break;
            const int col = 16 * c + ni;
            if (!live[col]) continue;
            double *pv = part + (gc.poff[cb + col] * TB + slot * TB) * 2;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = 16 * w + nk + 4 * q;
                pv[2 * r] = ar[c][q];
                pv[2 * r + 1] = ai[c][q];
            }
        }
    };
    double2 xv[8];
    double2 zv[16];
    load_x(xv, I);
    put_x(sXI, xv);
    load_z(zv, J0);
    load_x(xv, J0);
    f64x4g rr[2], ri[2];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int q = 0; q < 4; ++q) rr[c][q] = ri[c][q] = 0.0;
    for (int32_t J = J0; J < J1; ++J) {
        __syncthreads();   // the previous tile's LDS reads are done
        put_z(zv);
        put_x(sXJ, xv);
        __syncthreads();
        if (J + 1 < J1) {   // the next tile's loads go out before this tile's products
            load_z(zv, J + 1);
            load_x(xv, J + 1);
        }
        chain(rr, ri, false, sXJ);
        if (J != I) {
            f64x4g cr[2], ci[2];
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int q = 0; q < 4; ++q) cr[c][q] = ci[c][q] = 0.0;
            chain(cr, ci, true, sXI);
            store(cr, ci, gload_i64(P.seg, J) + I);
        }
    }
    store(rr, ri, gload_i64(P.seg, I) + I + uo);
}

// y_I = sum of the partial vectors of row block I (column sums of tiles
// (J < I, I), then row sums of the units of tile row I), stored contiguously.
// Eight waves split the vectors (every eighth one) and their sums are added in
// wave order (deterministic).
template <typename T, bool SUB>
__device__ inline void reduce_rows(int64_t N, const int64_t *__restrict__ seg, int64_t I,
                                   const typename Cx<T>::type *__restrict__ pv, typename Cx<T>::type *__restrict__ y,
                                   const typename Cx<T>::type *__restrict__ b)
{
    using V2 = typename Cx<T>::type;
    const int r = threadIdx.x & 63, w = threadIdx.x >> 6;
    pv += seg[I] * TB;
    const int64_t K = seg[I + 1] - seg[I];
    V2 a = { 0, 0 };
#pragma unroll 4
    for (int64_t q = w; q < K; q += 8) a += pv[q * TB + r];
    __shared__ V2 red[8][TB];
    red[w][r] = a;
    __syncthreads();
    if (w != 0) return;
    a = red[0][r];
#pragma unroll
    for (int q = 1; q < 8; ++q) a += red[q][r];
    const int64_t m = I * TB + r;
    if (m < N) {
        if (SUB) y[m] = b[m] - a;
        else y[m] = a;
    }
}

// The same with FP32 partial sums (the matrix-core pass stores its FP32
// accumulators as they are), added in FP64.
template <bool SUB>
__device__ inline void reduce_rows_f(int64_t N, const int64_t *__restrict__ seg, int64_t I,
                                     const float2 *__restrict__ pv, double2 *__restrict__ y,
                                     const double2 *__restrict__ b)
{
    const int r = threadIdx.x & 63, w = threadIdx.x >> 6;
    pv += seg[I] * TB;
    const int64_t K = seg[I + 1] - seg[I];
    double2 a = { 0, 0 };
#pragma unroll 4
    for (int64_t q = w; q < K; q += 8) {
        const float2 v = pv[q * TB + r];
        a.x += double(v.x);
        a.y += double(v.y);
    }
    __shared__ double2 red[8][TB];
    red[w][r] = a;
    __syncthreads();
    if (w != 0) return;
    a = red[0][r];
#pragma unroll
    for (int q = 1; q < 8; ++q) a += red[q][r];
    const int64_t m = I * TB + r;
    if (m < N) {
        if (SUB) y[m] = b[m] - a;
        else y[m] = a;
    }
}

template <typename T, bool SUB>
__global__ __launch_bounds__(512) void k_sym_reduce(int64_t N, const int64_t *__restrict__ seg, int64_t nslots,
                                                    const T *__restrict__ part, T *__restrict__ Y, int64_t ldy,
                                                    const T *__restrict__ B, int64_t ldb,
                                                    const int *__restrict__ skip, int64_t sks)
{
    using V2 = typename Cx<T>::type;
    const int64_t I = blockIdx.x, v = blockIdx.y;
    if (skip && skip[v * sks]) return;
    reduce_rows<T, SUB>(N, seg, I, reinterpret_cast<const V2 *>(part) + v * nslots * TB,
                        reinterpret_cast<V2 *>(Y) + v * ldy, SUB ? reinterpret_cast<const V2 *>(B) + v * ldb : nullptr);
}

// Grouped reduce: block b is the item (column c, row block I).
template <typename T, bool SUB>
__global__ __launch_bounds__(512) void k_sym_reduce_g(const GProb *__restrict__ probs, GCols gc,
                                                      const int32_t *__restrict__ items, const T *__restrict__ part,
                                                      T *__restrict__ Y, const T *__restrict__ B,
                                                      const int *__restrict__ skip, int64_t sks)
{
    using V2 = typename Cx<T>::type;
    const int64_t b = blockIdx.x;
    const int32_t c = items[2 * b], I = items[2 * b + 1];
    if (skip && skip[int64_t(c) * sks]) return;
    const GProb P = probs[gc.prob[c]];
    reduce_rows<T, SUB>(P.N, P.seg, I, reinterpret_cast<const V2 *>(part) + gc.poff[c] * TB,
                        reinterpret_cast<V2 *>(Y) + gc.yoff[c],
                        SUB ? reinterpret_cast<const V2 *>(B) + gc.yoff[c] : nullptr);
}

// Grouped reduce of the matrix-core pass's FP32 partial sums (FP64 sums, FP64 vectors)
template <bool SUB>
__global__ __launch_bounds__(512) void k_sym_reduce_gf(const GProb *__restrict__ probs, GCols gc,
                                                       const int32_t *__restrict__ items, const float *__restrict__ part,
                                                       double *__restrict__ Y, const double *__restrict__ B,
                                                       const int *__restrict__ skip, int64_t sks)
{
    const int64_t b = blockIdx.x;
    const int32_t c = items[2 * b], I = items[2 * b + 1];
    if (skip && skip[int64_t(c) * sks]) return;
    const GProb P = probs[gc.prob[c]];
    reduce_rows_f<SUB>(P.N, P.seg, I, reinterpret_cast<const float2 *>(part) + gc.poff[c] * TB,
                       reinterpret_cast<double2 *>(Y) + gc.yoff[c], SUB ? reinterpret_cast<const double2 *>(B) + gc.yoff[c] : nullptr);
}

template <typename T>
__global__ __launch_bounds__(256) void k_unpack(const T *__restrict__ Zp, int64_t N, int64_t nT,
                                                double2 *__restrict__ out)
{
    using V2 = typename Cx<T>::type;
    const int64_t n = int64_t(blockIdx.x) * 256 + threadIdx.x;
    const int64_t m = blockIdx.y;
    if (n >= N) return;
    const int64_t I = m / TB, J = n / TB;
    const V2 *Z = reinterpret_cast<const V2 *>(Zp);
    const V2 z = I <= J ? Z[tile_of(I, J, nT) * TB * TB + (m % TB) * TB + (n % TB)]
                        : Z[tile_of(J, I, nT) * TB * TB + (n % TB) * TB + (m % TB)];
    out[m * N + n] = make_double2(double(z.x), double(z.y));
}

// One wave per sampled row i: (T x)_i from the packed tiles (row i of tiles
// (I, J >= I), column i of tiles (J < I, I)), then |b_i - (T x)_i|^2.
__global__ __launch_bounds__(256) void k_sampled_rows(const double2 *__restrict__ Zp, int64_t N, int64_t nT,
                                                      int64_t S, const int64_t *__restrict__ rows,
                                                      const double2 *__restrict__ B, const double2 *__restrict__ X,
                                                      double *__restrict__ out, const int *__restrict__ mask)
{
    const int64_t v = blockIdx.y;
    if (!mask[v]) return;
    const int lane = threadIdx.x & 63;
    const int64_t s = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (s >= S) return;
    const int64_t i = rows[v * S + s];
    const int64_t I = i / TB, rr = i % TB;
    const double2 *x = X + v * N;
    double ar = 0.0, ai = 0.0;
    for (int64_t J = 0; J < nT; ++J) {
        const int64_t n = J * TB + lane;
        if (n >= N) continue;
        const double2 z = J >= I ? Zp[tile_of(I, J, nT) * TB * TB + rr * TB + lane]
                                 : Zp[tile_of(J, I, nT) * TB * TB + lane * TB + rr];
        const double2 xv = x[n];
        ar += z.x * xv.x - z.y * xv.y;
        ai += z.x * xv.y + z.y * xv.x;
    }
    ar = wsum(ar);
    ai = wsum(ai);
    if (lane == 0) {
        const double2 b = B[v * N + i];
        const double dr = b.x - ar, di = b.y - ai;
        out[v * S + s] = dr * dr + di * di;
    }
}

__global__ void k_convert_d2f(const double *__restrict__ a, float *__restrict__ b, int64_t n)
{
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        b[i] = float(a[i]);
}
__global__ void k_convert_f2d(const float *__restrict__ a, double *__restrict__ b, int64_t n)
{
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        b[i] = double(a[i]);
}
__global__ void k_nonfinite(const double *__restrict__ a, int64_t n, int *__restrict__ flag)
{
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        if (!isfinite(a[i])) *flag = 1;
}

// Tile-pass variant: register double buffering of the next tile (default) or
// not; BIE_SYM_PREFETCH=0 selects the plain form (kept for measurement).
int sym_prefetch()
{
    static int v = [] {
        const char *e = getenv("BIE_SYM_PREFETCH");
        return e ? atoi(e) : 1;
    }();
    return v;
}

// Star-split product (Sec. VI-A): T x = T_A' x + Sigma V' Sigma^T x.
// u = Sigma^T x: u_p = sum over the three edges m of triangle p of s x_m.
template <typename T>
__global__ __launch_bounds__(256) void k_star_gather(int64_t F, const int32_t *__restrict__ slot_m,
                                                     const int8_t *__restrict__ sgn, const T *__restrict__ X,
                                                     int64_t ldx, T *__restrict__ U, const int *__restrict__ skip,
                                                     int64_t sks)
{
    using V2 = typename Cx<T>::type;
    const int64_t v = blockIdx.y;
    if (skip && skip[v * sks]) return;
    const V2 *x = reinterpret_cast<const V2 *>(X) + v * ldx;
    V2 *u = reinterpret_cast<V2 *>(U) + v * F;
    for (int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x; p < F; p += int64_t(gridDim.x) * 256) {
        V2 a = { 0, 0 };
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            const V2 xm = x[slot_m[3 * p + e]];
            if (sgn[3 * p + e] > 0) a += xm;
            else a -= xm;
        }
        u[p] = a;
    }
}

// y_m += w_{c+(m)} - w_{c-(m)} (SUB: -=), w = V' u
template <typename T, bool SUB>
__global__ __launch_bounds__(256) void k_star_scatter(int64_t N, int64_t F, const int4 *__restrict__ rwg4,
                                                      const T *__restrict__ W, T *__restrict__ Y, int64_t ldy,
                                                      const int *__restrict__ skip, int64_t sks)
{
    using V2 = typename Cx<T>::type;
    const int64_t v = blockIdx.y;
    if (skip && skip[v * sks]) return;
    const V2 *w = reinterpret_cast<const V2 *>(W) + v * F;
    V2 *y = reinterpret_cast<V2 *>(Y) + v * ldy;
    for (int64_t m = int64_t(blockIdx.x) * 256 + threadIdx.x; m < N; m += int64_t(gridDim.x) * 256) {
        const int4 e = rwg4[m];
        const V2 d = w[e.x] - w[e.y];
        if (SUB) y[m] -= d;
        else y[m] += d;
    }
}

template <typename M, typename T, bool CONJ, bool SUB>
void launch_product(const Packed &pk, void *part, const void *Z, const void *X, int64_t ldx, void *Y, int64_t ldy,
                    const void *B, int64_t ldb, int64_t R, const int *skip, int64_t sks, hipStream_t s,
                    bool profile = true)
{
    const dim3 grid(unsigned(pk.nruns), unsigned(R));
    if (profile) prof::begin(0, s, R);
    // non-temporal tile loads for the FP64 matrix, cached loads for the FP32
    // one (measured: 92 vs 144 us, 52 vs 47 us at N = 7680)
    constexpr bool NT = sizeof(M) == 8;
    if (sym_prefetch())
        hipLaunchKernelGGL((k_sym_tiles<M, T, CONJ, true, NT>), grid, dim3(256), 0, s, (const M *)Z, pk.N, pk.nT,
                           pk.units, pk.unit_ptr, pk.run_ptr, pk.seg, pk.nslots, (const T *)X, ldx, (T *)part,
                           skip, sks);
    else
        hipLaunchKernelGGL((k_sym_tiles<M, T, CONJ, false, NT>), grid, dim3(256), 0, s, (const M *)Z, pk.N, pk.nT,
                           pk.units, pk.unit_ptr, pk.run_ptr, pk.seg, pk.nslots, (const T *)X, ldx, (T *)part,
                           skip, sks);
    if (profile) {
        prof::end(0, s);
        prof::begin(3, s, R);
    }
    hipLaunchKernelGGL((k_sym_reduce<T, SUB>), dim3(unsigned(pk.nT), unsigned(R)), dim3(512), 0, s, pk.N, pk.seg,
                       pk.nslots, (const T *)part, (T *)Y, ldy, (const T *)B, ldb, skip, sks);
    BIE_HIP(hipGetLastError());
    if (profile) prof::end(3, s);
}

}  // namespace

// Row pointers and partial-slot segments of a unit table sorted by tile row:
// row block I owns the column sums of tiles (J < I, I), then one row-sum slot
// per unit of tile row I.
static void unit_rows(int64_t nT, const std::vector<int32_t> &units, std::vector<int32_t> &uptr,
                      std::vector<int64_t> &seg)
{
    const int64_t nu = int64_t(units.size() / 3);
    uptr.assign(nT + 1, int32_t(nu));
    for (int64_t u = nu - 1; u >= 0; --u) uptr[units[3 * u]] = int32_t(u);
    for (int64_t I = nT - 1; I >= 0; --I) uptr[I] = std::min(uptr[I], uptr[I + 1]);
    seg.assign(nT + 1, 0);
    for (int64_t I = 0; I < nT; ++I) seg[I + 1] = seg[I] + I + (uptr[I + 1] - uptr[I]);
}

void build_units(int64_t nT, int U, std::vector<int32_t> &units, std::vector<int32_t> &uptr,
                 std::vector<int64_t> &seg)
{
    units.clear();
    for (int64_t I = 0; I < nT; ++I)
        for (int64_t J0 = I; J0 < nT; J0 += U) {
            units.push_back(int32_t(I));
            units.push_back(int32_t(J0));
            units.push_back(int32_t(std::min<int64_t>(nT, J0 + U)));
        }
    unit_rows(nT, units, uptr, seg);
}

// Balanced runs: the T = nT (nT + 1) / 2 stored tiles in row-major order
// (I, J >= I) are cut into nb runs [T b / nb, T (b+1) / nb) of equal length
// to within one tile, and each run into units at the ends of tile rows; run b
// is units rptr[b] .. rptr[b+1]-1.  With nb = 512 (two 4-wave blocks on each of
// the 256 CUs) every block of a single-vector product has the same work and
// all are resident at once; small matrices take fewer runs (at least 8 tiles
// each: a run's fixed cost is loading x and writing its row sums).  Selected
// with BIE_SYM_UNIT=0.
void build_runs(int64_t nT, int64_t nb, std::vector<int32_t> &units, std::vector<int32_t> &uptr,
                std::vector<int64_t> &seg, std::vector<int32_t> &rptr)
{
    const int64_t T = nT * (nT + 1) / 2;
    nb = std::max<int64_t>(1, std::min(nb, T));
    units.clear();
    rptr.assign(nb + 1, 0);
    int64_t I = 0, J = 0, t = 0;
    for (int64_t b = 0; b < nb; ++b) {
        rptr[b] = int32_t(units.size() / 3);
        const int64_t t1 = T * (b + 1) / nb;
        while (t < t1) {
            const int64_t take = std::min(nT - J, t1 - t);
            units.push_back(int32_t(I));
            units.push_back(int32_t(J));
            units.push_back(int32_t(J + take));
            t += take;
            J += take;
            if (J == nT) J = ++I;
        }
    }
    rptr[nb] = int32_t(units.size() / 3);
    unit_rows(nT, units, uptr, seg);
}

// Tables of the packed n x n tiles with units of U tiles (U >= 1) or balanced
// runs (U = 0).
static void packed_setup_units(Packed &pk, int64_t n, int U)
{
    pk.N = n;
    pk.nT = (pk.N + TB - 1) / TB;
    pk.ntiles = pk.nT * (pk.nT + 1) / 2;
    pk.unit_len = U;
    std::vector<int32_t> units, uptr, rptr;
    std::vector<int64_t> seg;
    if (U > 0) {
        build_units(pk.nT, U, units, uptr, seg);
        rptr.resize(units.size() / 3 + 1);
        for (size_t b = 0; b < rptr.size(); ++b) rptr[b] = int32_t(b);
    } else {   // 512 runs, or fewer for small matrices: at least 8 tiles per run
        build_runs(pk.nT, std::max<int64_t>(1, std::min<int64_t>(512, pk.ntiles / 8)), units, uptr, seg, rptr);
    }
    pk.nunits = int64_t(units.size() / 3);
    pk.nruns = int64_t(rptr.size()) - 1;
    pk.nslots = seg[pk.nT];
    BIE_HIP(hipMalloc(&pk.seg, seg.size() * sizeof(int64_t)));
    BIE_HIP(hipMemcpy(pk.seg, seg.data(), seg.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    BIE_HIP(hipMalloc(&pk.units, units.size() * sizeof(int32_t)));
    BIE_HIP(hipMalloc(&pk.unit_ptr, uptr.size() * sizeof(int32_t)));
    BIE_HIP(hipMalloc(&pk.run_ptr, rptr.size() * sizeof(int32_t)));
    BIE_HIP(hipMemcpy(pk.units, units.data(), units.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    BIE_HIP(hipMemcpy(pk.unit_ptr, uptr.data(), uptr.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    BIE_HIP(hipMemcpy(pk.run_ptr, rptr.data(), rptr.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    pk.h_units = std::move(units);
    pk.h_unit_ptr = std::move(uptr);
    pk.h_seg = std::move(seg);
}

void packed_setup(Packed &pk, int64_t n) { packed_setup_units(pk, n, unit_tiles()); }

void packed_free(Packed &pk)
{
    if (pk.units) (void)hipFree(pk.units);
    if (pk.unit_ptr) (void)hipFree(pk.unit_ptr);
    if (pk.run_ptr) (void)hipFree(pk.run_ptr);
    pk.run_ptr = nullptr;
    if (pk.seg) (void)hipFree(pk.seg);
    pk.seg = nullptr;
    if (pk.part) (void)hipFree(pk.part);
    pk.units = pk.unit_ptr = nullptr;
    pk.part = nullptr;
    pk.part_R = 0;
}

// part: the partial sums, R x nslots x 64 complex T (the operator's buffer, or
// the static scratch of the allocation-free entry point, which also skips the
// profiling events)
template <typename M, typename T>
void dispatch(const Packed &pk, const void *Z, const void *X, int64_t ldx, void *Y, int64_t ldy, const void *B,
              int64_t ldb, int64_t R, const int *skip, int64_t sks, bool conj, hipStream_t s, void *part = nullptr)
{
    const bool profile = part == nullptr;
    if (!part) part = pk.part;
    if (B) launch_product<M, T, false, true>(pk, part, Z, X, ldx, Y, ldy, B, ldb, R, skip, sks, s, profile);
    else if (conj) launch_product<M, T, true, false>(pk, part, Z, X, ldx, Y, ldy, nullptr, 0, R, skip, sks, s, profile);
    else launch_product<M, T, false, false>(pk, part, Z, X, ldx, Y, ldy, nullptr, 0, R, skip, sks, s, profile);
}

// partial-sum buffer of a packed product for R vectors (sized for complex128)
static void ensure_part(Packed &pk, int64_t R, hipStream_t s)
{
    if (pk.part_R >= R) return;
    BIE_HIP(hipStreamSynchronize(s));
    if (pk.part) (void)hipFree(pk.part);
    pk.part = nullptr;
    pk.part_R = 0;
    BIE_HIP(hipMalloc(&pk.part, size_t(R) * size_t(pk.nslots) * TB * 16));
    pk.part_R = R;
}

// The packed product's work units for this operator: the autotuner's choice
// for (N, matrix precision) among units of 4, 8, 16 tiles and balanced runs,
// timed (tile pass and reduction of one vector) the first time the size
// occurs; the operator's tables are rebuilt if the choice is not the default.
// Fixed by BIE_SYM_UNIT (measurement) or with tuning off.
void tune_packed(bie_op *op, hipStream_t s)
{
    if (op->star || getenv("BIE_SYM_UNIT") || !tune_enabled() || stream_capturing(s)) return;
    const bool mat64 = op->Z64 != nullptr;
    const void *Z = mat64 ? op->Z64 : op->Z32;
    if (!Z) return;
    const int64_t N = op->mesh.N;
    const std::string key = "sym:" + std::to_string(N) + (mat64 ? ":f64" : ":f32");
    std::vector<int> v;
    if (!tune_get(key, v) || v.size() != 1 || v[0] < 0 || v[0] > 64) {
        void *x = nullptr, *y = nullptr;
        BIE_HIP(hipMalloc(&x, size_t(N) * 16));
        try {
            BIE_HIP(hipMalloc(&y, size_t(N) * 16));
            BIE_HIP(hipMemsetAsync(x, 0, size_t(N) * 16, s));
            float best = 0.f;
            v = { unit_tiles() };
            for (int U : { 8, 0, 4, 16 }) {
                Packed c;
                try {
                    packed_setup_units(c, N, U);
                    ensure_part(c, 1, s);
                    const float ms = time_launches(s, 3, [&]() {
                        if (mat64)
                            launch_product<double, double, false, false>(c, c.part, Z, x, N, y, N, nullptr, 0, 1,
                                                                         nullptr, 1, s, false);
                        else
                            launch_product<float, double, false, false>(c, c.part, Z, x, N, y, N, nullptr, 0, 1,
                                                                        nullptr, 1, s, false);
                    });
                    if (best == 0.f || ms < best) {
                        best = ms;
                        v = { U };
                    }
                } catch (...) {
                    packed_free(c);
                    throw;
                }
                packed_free(c);
            }
        } catch (...) {
            (void)hipFree(x);
            if (y) (void)hipFree(y);
            throw;
        }
        BIE_HIP(hipStreamSynchronize(s));
        (void)hipFree(x);
        (void)hipFree(y);
        tune_put(key, v);
    }
    if (v[0] != op->pk.unit_len) {
        BIE_HIP(hipStreamSynchronize(s));
        packed_free(op->pk);
        packed_setup_units(op->pk, N, v[0]);
    }
}

// T x (conj: conj(T) x; B: B - T x) for the star-split operator: u = Sigma^T x,
// w = V' u, y = T_A' x (or B - T_A' x), y += Sigma w (or -=).
template <typename M, typename T>
static void star_product(bie_op *op, const void *Za, const void *Vm, const void *X, int64_t ldx, void *Y,
                         int64_t ldy, const void *B, int64_t ldb, int64_t R, const int *skip, int64_t sks, bool conj,
                         hipStream_t s)
{
    const int64_t N = op->mesh.N, F = op->mesh.F;
    if (op->star_R < R) {
        BIE_HIP(hipStreamSynchronize(s));
        if (op->star_buf) (void)hipFree(op->star_buf);
        op->star_buf = nullptr;
        op->star_R = 0;
        BIE_HIP(hipMalloc(&op->star_buf, 2 * size_t(R) * size_t(F) * 16));
        op->star_R = R;
    }
    T *U = static_cast<T *>(op->star_buf), *W = U + 2 * R * F;
    const unsigned gx = unsigned(std::min<int64_t>((std::max(N, F) + 255) / 256, 1024));
    hipLaunchKernelGGL(k_star_gather<T>, dim3(gx, unsigned(R)), dim3(256), 0, s, F, op->tri.slot_m, op->tri.sgn,
                       (const T *)X, ldx, U, skip, sks);
    dispatch<M, T>(op->pkv, Vm, U, F, W, F, nullptr, 0, R, skip, sks, conj, s);
    dispatch<M, T>(op->pk, Za, X, ldx, Y, ldy, B, ldb, R, skip, sks, conj, s);
    if (B) hipLaunchKernelGGL((k_star_scatter<T, true>), dim3(gx, unsigned(R)), dim3(256), 0, s, N, F,
                              (const int4 *)op->tri.edges, W, (T *)Y, ldy, skip, sks);
    else hipLaunchKernelGGL((k_star_scatter<T, false>), dim3(gx, unsigned(R)), dim3(256), 0, s, N, F,
                            (const int4 *)op->tri.edges, W, (T *)Y, ldy, skip, sks);
    BIE_HIP(hipGetLastError());
}

void product(const bie_op *opc, int mat, bool vec64, const void *X, int64_t ldx, void *Y, int64_t ldy,
             const void *B, int64_t ldb, int64_t R, const int *skip, int64_t sks, bool conj, hipStream_t s)
{
    bie_op *op = const_cast<bie_op *>(opc);
    if (op->fast) {   // near entries + multilevel far field; every vector computed (no skip)
        if (!vec64 || conj) throw Error(BIE_EINVAL, "the fast operator takes complex128 vectors, no conjugate");
        fast_product(op, X, ldx, Y, ldy, B, ldb, R, s);
        return;
    }
    if (mat == MATBF16) {
        if (!op->Abf) throw Error(BIE_EINVAL, "no split-BF16 matrix stored");
        if (!vec64 || conj) throw Error(BIE_EINVAL, "the block product takes complex128 vectors, no conjugate");
        gemm_product(op, X, ldx, VEC_C128, Y, ldy, B, ldb, R, nullptr, s);
        return;
    }
    const bool mat64 = mat == MAT64;
    const void *Z = mat64 ? op->Z64 : op->Z32;
    if (!Z) throw Error(BIE_EINVAL, "matrix not stored in the requested precision");
    if (mat64 && !vec64) throw Error(BIE_EINVAL, "complex64 vectors need the FP32 matrix");
    ensure_part(op->pk, R, s);
    if (op->star) {
        const void *Vm = mat64 ? op->V64 : op->V32;
        ensure_part(op->pkv, R, s);
        if (mat64) star_product<double, double>(op, Z, Vm, X, ldx, Y, ldy, B, ldb, R, skip, sks, conj, s);
        else if (vec64) star_product<float, double>(op, Z, Vm, X, ldx, Y, ldy, B, ldb, R, skip, sks, conj, s);
        else star_product<float, float>(op, Z, Vm, X, ldx, Y, ldy, B, ldb, R, skip, sks, conj, s);
        return;
    }
    if (mat64) dispatch<double, double>(op->pk, Z, X, ldx, Y, ldy, B, ldb, R, skip, sks, conj, s);
    else if (vec64) dispatch<float, double>(op->pk, Z, X, ldx, Y, ldy, B, ldb, R, skip, sks, conj, s);
    else dispatch<float, float>(op->pk, Z, X, ldx, Y, ldy, B, ldb, R, skip, sks, conj, s);
}

// ----------------------------------------------------------------------------- allocation-free product
// For callers that cannot allocate (graph capture, serving loops): the
// partial sums live in this static array instead of the operator's buffer.
// Each device holds its own copy for the life of the process; host code
// reaches it only through the address hipGetSymbolAddress returns on that
// device (kept in scratch_dev), never through the array's name.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_dev[MAX_DEVICES] = { nullptr };

// device address of the current device's scratch, looked up once per device
void *noalloc_scratch(int dev)
{
    if (dev < 0 || dev >= MAX_DEVICES) throw Error(BIE_EDEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> g(scratch_mu);
    if (!scratch_dev[dev]) {
        void *p = nullptr;
        BIE_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw Error(BIE_EDEVICE, "hipGetSymbolAddress returned no address for the scratch array");
        scratch_dev[dev] = p;
    }
    return scratch_dev[dev];
}
}  // namespace

void product_noalloc(const bie_op *op, bool vec64, const void *X, void *Y, int64_t R, bool conj, hipStream_t s)
{
    if (op->star) throw Error(BIE_EINVAL, "the allocation-free product takes an assembled operator");
    const Packed &pk = op->pk;
    const size_t need = size_t(R) * size_t(pk.nslots) * TB * (vec64 ? 16 : 8);
    if (need > NOALLOC_SCRATCH_BYTES)
        throw Error(BIE_EINVAL, "partial sums of " + std::to_string(need) + " bytes exceed the " +
                                    std::to_string(NOALLOC_SCRATCH_BYTES) + "-byte scratch of the allocation-free "
                                    "product: use fewer vectors per call");
    int dev = -1;
    BIE_HIP(hipGetDevice(&dev));
    if (dev != op->device) throw Error(BIE_EINVAL, "the operator's device must be current");
    void *part = noalloc_scratch(dev);
    if (vec64) {
        if (op->Z64) dispatch<double, double>(pk, op->Z64, X, pk.N, Y, pk.N, nullptr, 0, R, nullptr, 1, conj, s, part);
        else if (op->Z32) dispatch<float, double>(pk, op->Z32, X, pk.N, Y, pk.N, nullptr, 0, R, nullptr, 1, conj, s, part);
        else throw Error(BIE_EINVAL, "no packed matrix stored");
    } else {
        if (!op->Z32) throw Error(BIE_EINVAL, "complex64 vectors need the FP32 matrix");
        dispatch<float, float>(pk, op->Z32, X, pk.N, Y, pk.N, nullptr, 0, R, nullptr, 1, conj, s, part);
    }
}

void grouped_product(bool mat64, const GProb *probs, const GCols &gc, const int32_t *items, int64_t nitems, int G,
                     const int32_t *ritems, int64_t nritems, const void *X, void *part, void *Y, const void *B,
                     const int *skip, int64_t sks, hipStream_t s, bool mfma)
{
    if (nitems == 0) return;
    const bool pf = sym_prefetch() != 0;
    if (mfma) {
        if (G > 32) throw Error(BIE_EINVAL, "the matrix-core grouped pass takes at most 32 columns per item");
        if (mat64)
            hipLaunchKernelGGL(k_sym_tiles_gm64, dim3(unsigned(nitems)), dim3(256), 0, s, probs, gc, items, G,
                               (const double *)X, (double *)part, skip, sks);
        else {   // FP32 partial sums, reduced here
            hipLaunchKernelGGL(k_sym_tiles_gm, dim3(unsigned(nitems)), dim3(256), 0, s, probs, gc, items, G,
                               (const double *)X, (float *)part, skip, sks);
            if (B) hipLaunchKernelGGL(k_sym_reduce_gf<true>, dim3(unsigned(nritems)), dim3(512), 0, s, probs, gc, ritems,
                                      (const float *)part, (double *)Y, (const double *)B, skip, sks);
            else hipLaunchKernelGGL(k_sym_reduce_gf<false>, dim3(unsigned(nritems)), dim3(512), 0, s, probs, gc, ritems,
                                    (const float *)part, (double *)Y, nullptr, skip, sks);
            BIE_HIP(hipGetLastError());
            return;
        }
    } else if (mat64) {
        if (pf) hipLaunchKernelGGL((k_sym_tiles_g<double, double, true>), dim3(unsigned(nitems)), dim3(256), 0, s, probs,
                                   gc, items, G, (const double *)X, (double *)part, skip, sks);
        else hipLaunchKernelGGL((k_sym_tiles_g<double, double, false>), dim3(unsigned(nitems)), dim3(256), 0, s,
                                probs, gc, items, G, (const double *)X, (double *)part, skip, sks);
    } else {
        if (pf) hipLaunchKernelGGL((k_sym_tiles_g<float, double, true>), dim3(unsigned(nitems)), dim3(256), 0, s, probs,
                                   gc, items, G, (const double *)X, (double *)part, skip, sks);
        else hipLaunchKernelGGL((k_sym_tiles_g<float, double, false>), dim3(unsigned(nitems)), dim3(256), 0, s, probs,
                                gc, items, G, (const double *)X, (double *)part, skip, sks);
    }
    if (B) hipLaunchKernelGGL((k_sym_reduce_g<double, true>), dim3(unsigned(nritems)), dim3(512), 0, s, probs, gc,
                              ritems, (const double *)part, (double *)Y, (const double *)B, skip, sks);
    else hipLaunchKernelGGL((k_sym_reduce_g<double, false>), dim3(unsigned(nritems)), dim3(512), 0, s, probs, gc,
                            ritems, (const double *)part, (double *)Y, nullptr, skip, sks);
    BIE_HIP(hipGetLastError());
}

void unpack_c128(const bie_op *op, bool from64, void *dst, hipStream_t s)
{
    const Packed &pk = op->pk;
    const dim3 grid(unsigned((pk.N + 255) / 256), unsigned(pk.N));
    if (from64) hipLaunchKernelGGL(k_unpack<double>, grid, dim3(256), 0, s, (const double *)op->Z64, pk.N, pk.nT,
                                   (double2 *)dst);
    else hipLaunchKernelGGL(k_unpack<float>, grid, dim3(256), 0, s, (const float *)op->Z32, pk.N, pk.nT,
                            (double2 *)dst);
    BIE_HIP(hipGetLastError());
}

void sampled_residual(const bie_op *op, const void *B, const void *X, int64_t R, int64_t S, const int64_t *rows,
                      double *out, const int *mask, hipStream_t s)
{
    if (!op->Z64) throw Error(BIE_EINVAL, "the random-sampling criterion needs the FP64 matrix");
    const Packed &pk = op->pk;
    hipLaunchKernelGGL(k_sampled_rows, dim3(unsigned((S + 3) / 4), unsigned(R)), dim3(256), 0, s,
                       (const double2 *)op->Z64, pk.N, pk.nT, S, rows, (const double2 *)B, (const double2 *)X, out,
                       mask);
    BIE_HIP(hipGetLastError());
}

void convert_c128_to_c64(const void *src, void *dst, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_convert_d2f, dim3(2048), dim3(256), 0, s, (const double *)src, (float *)dst, 2 * n);
    BIE_HIP(hipGetLastError());
}

void convert_c64_to_c128(const void *src, void *dst, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_convert_f2d, dim3(2048), dim3(256), 0, s, (const float *)src, (double *)dst, 2 * n);
    BIE_HIP(hipGetLastError());
}

bool has_nonfinite(const void *x, int64_t n_doubles, hipStream_t s)
{
    int *flag = nullptr;
    BIE_HIP(hipMalloc(&flag, sizeof(int)));
    BIE_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_nonfinite, dim3(1024), dim3(256), 0, s, (const double *)x, n_doubles, flag);
    int h = 0;
    BIE_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    BIE_HIP(hipStreamSynchronize(s));
    (void)hipFree(flag);
    return h != 0;
}

}  // namespace bie
