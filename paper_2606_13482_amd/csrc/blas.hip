// Dense complex matrix-vector products with the impedance matrix.
//
// The matrix-vector product is the O(N^2) operation of every Krylov
// iteration (Sec. I and II: dense storage and MVP cost).  T is stored
// row-major, N x N, interleaved complex (FP64: 16 B, FP32: 8 B per entry).
// The product streams T from HBM exactly once per call: every lane issues
// 16-byte loads of consecutive columns (a wave covers 1 KiB of a row per
// step), ROWS rows per wave share each load of x (x stays in L2), NV vectors
// share each load of T, and each row's partial sums are combined with wave
// shuffles.  Y = T X, Y = T^H X = conj(T conj X) (T = T^T), or Y = B - T X.
#include <hip/hip_runtime.h>

#include <utility>
#include <vector>

#include "bie_internal.hpp"

namespace bie {

// Optional timing of the product kernel: events recorded on the launch stream.
namespace prof {
bool on = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
size_t used = 0;

void begin(hipStream_t s)
{
    if (!on) return;
    if (used == ev.size()) {
        hipEvent_t a, b;
        BIE_HIP(hipEventCreate(&a));
        BIE_HIP(hipEventCreate(&b));
        ev.emplace_back(a, b);
    }
    BIE_HIP(hipEventRecord(ev[used].first, s));
}
void end(hipStream_t s)
{
    if (!on) return;
    BIE_HIP(hipEventRecord(ev[used].second, s));
    ++used;
}
}  // namespace prof

void prof_enable(bool enable) { prof::on = enable; }

void prof_read(int64_t *launches, double *total_ms)
{
    double t = 0.0;
    for (size_t i = 0; i < prof::used; ++i) {
        BIE_HIP(hipEventSynchronize(prof::ev[i].second));
        float ms = 0.f;
        BIE_HIP(hipEventElapsedTime(&ms, prof::ev[i].first, prof::ev[i].second));
        t += ms;
    }
    *launches = int64_t(prof::used);
    *total_ms = t;
    prof::used = 0;
}

namespace {

typedef double nd2 __attribute__((ext_vector_type(2)));
typedef float nf4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Packet;   // 16-byte load unit (native vector type)
template <>
struct Packet<double> {
    using type = nd2;       // one complex128
    static constexpr int C = 1;
};
template <>
struct Packet<float> {
    using type = nf4;       // two complex64
    static constexpr int C = 2;
};

template <typename T>
__device__ inline T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <typename T>
__device__ inline void unpack(const typename Packet<T>::type &p, T re[], T im[]);
template <>
__device__ inline void unpack<double>(const nd2 &p, double re[], double im[])
{
    re[0] = p.x; im[0] = p.y;
}
template <>
__device__ inline void unpack<float>(const nf4 &p, float re[], float im[])
{
    re[0] = p.x; im[0] = p.y; re[1] = p.z; im[1] = p.w;
}

// One wave: ROWS consecutive rows x NV vectors.  Block: 4 waves.
// X, Y: vector v at offset v*ld (complex elements); B (optional): Y = B - T X.
template <typename T, int ROWS, int NV, bool CONJ, bool SUB>
__global__ __launch_bounds__(256) void k_gemv(const T *__restrict__ Z, int64_t N, const T *__restrict__ X,
                                              int64_t ldx, T *__restrict__ Y, int64_t ldy,
                                              const T *__restrict__ B, int64_t ldb, int64_t R,
                                              const int *__restrict__ skip, int64_t sks)
{
    using P = typename Packet<T>::type;
    constexpr int C = Packet<T>::C;
    const int lane = threadIdx.x & 63;
    const int64_t row0 = (int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6)) * ROWS;
    const int64_t v0 = int64_t(blockIdx.y) * NV;
    if (row0 >= N) return;
    if (skip) {
        bool any = false;
        for (int v = 0; v < NV; ++v)
            if (v0 + v < R && !skip[(v0 + v) * sks]) any = true;
        if (!any) return;
    }
    int64_t rows[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) rows[r] = (row0 + r < N) ? row0 + r : N - 1;
    const T *xs[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) xs[v] = X + 2 * ((v0 + v < R ? v0 + v : R - 1) * ldx);

    T ar[ROWS][NV], ai[ROWS][NV];
#pragma unroll
    for (int r = 0; r < ROWS; ++r)
#pragma unroll
        for (int v = 0; v < NV; ++v) { ar[r][v] = 0; ai[r][v] = 0; }

    for (int64_t c = int64_t(lane) * C; c < N; c += 64 * C) {
        T xr[NV][C], xi[NV][C];
#pragma unroll
        for (int v = 0; v < NV; ++v) unpack<T>(*reinterpret_cast<const P *>(xs[v] + 2 * c), xr[v], xi[v]);
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            T zr[C], zi[C];
            unpack<T>(__builtin_nontemporal_load(reinterpret_cast<const P *>(Z + 2 * (rows[r] * N + c))), zr, zi);
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int e = 0; e < C; ++e) {
                    if (!CONJ) {
                        ar[r][v] += zr[e] * xr[v][e] - zi[e] * xi[v][e];
                        ai[r][v] += zr[e] * xi[v][e] + zi[e] * xr[v][e];
                    } else {
                        ar[r][v] += zr[e] * xr[v][e] + zi[e] * xi[v][e];
                        ai[r][v] += zr[e] * xi[v][e] - zi[e] * xr[v][e];
                    }
                }
        }
    }
#pragma unroll
    for (int r = 0; r < ROWS; ++r)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            ar[r][v] = wave_sum(ar[r][v]);
            ai[r][v] = wave_sum(ai[r][v]);
        }
    if (lane == 0) {
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            if (row0 + r >= N) continue;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const int64_t vv = v0 + v;
                if (vv >= R || (skip && skip[vv * sks])) continue;
                T yr = ar[r][v], yi = ai[r][v];
                if (SUB) {
                    yr = B[2 * (vv * ldb + row0 + r)] - yr;
                    yi = B[2 * (vv * ldb + row0 + r) + 1] - yi;
                }
                Y[2 * (vv * ldy + row0 + r)] = yr;
                Y[2 * (vv * ldy + row0 + r) + 1] = yi;
            }
        }
    }
}

template <typename T, bool CONJ, bool SUB>
void launch_gemv(const void *Z, int64_t N, const void *X, int64_t ldx, void *Y, int64_t ldy, const void *B,
                 int64_t ldb, int64_t R, const int *skip, int64_t sks, hipStream_t s)
{
    // Rows per wave / vectors per pass chosen for enough loads in flight per CU.
    constexpr int ROWS = 4;
    prof::begin(s);
    if (R >= 4) {
        constexpr int NV = 4;
        dim3 grid(unsigned((N + 4 * ROWS - 1) / (4 * ROWS)), unsigned((R + NV - 1) / NV));
        hipLaunchKernelGGL((k_gemv<T, ROWS, NV, CONJ, SUB>), grid, dim3(256), 0, s, (const T *)Z, N, (const T *)X,
                           ldx, (T *)Y, ldy, (const T *)B, ldb, R, skip, sks);
    } else {
        constexpr int NV = 1;
        dim3 grid(unsigned((N + 4 * ROWS - 1) / (4 * ROWS)), unsigned(R));
        hipLaunchKernelGGL((k_gemv<T, ROWS, NV, CONJ, SUB>), grid, dim3(256), 0, s, (const T *)Z, N, (const T *)X,
                           ldx, (T *)Y, ldy, (const T *)B, ldb, R, skip, sks);
    }
    BIE_HIP(hipGetLastError());
    prof::end(s);
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

}  // namespace

void gemv_c128(const void *Z, int64_t N, const void *X, void *Y, int64_t R, bool conj, hipStream_t s)
{
    if (conj) launch_gemv<double, true, false>(Z, N, X, N, Y, N, nullptr, 0, R, nullptr, 1, s);
    else launch_gemv<double, false, false>(Z, N, X, N, Y, N, nullptr, 0, R, nullptr, 1, s);
}

void gemv_c64(const void *Z, int64_t N, const void *X, void *Y, int64_t R, bool conj, hipStream_t s)
{
    if (conj) launch_gemv<float, true, false>(Z, N, X, N, Y, N, nullptr, 0, R, nullptr, 1, s);
    else launch_gemv<float, false, false>(Z, N, X, N, Y, N, nullptr, 0, R, nullptr, 1, s);
}

// Strided forms used by the solvers (declared in krylov.hip).
void gemv_strided(bool fp64, const void *Z, int64_t N, const void *X, int64_t ldx, void *Y, int64_t ldy,
                  const void *B, int64_t ldb, int64_t R, const int *skip, int64_t sks, bool conj, hipStream_t s)
{
    if (fp64) {
        if (B) launch_gemv<double, false, true>(Z, N, X, ldx, Y, ldy, B, ldb, R, skip, sks, s);
        else if (conj) launch_gemv<double, true, false>(Z, N, X, ldx, Y, ldy, nullptr, 0, R, skip, sks, s);
        else launch_gemv<double, false, false>(Z, N, X, ldx, Y, ldy, nullptr, 0, R, skip, sks, s);
    } else {
        if (B) launch_gemv<float, false, true>(Z, N, X, ldx, Y, ldy, B, ldb, R, skip, sks, s);
        else if (conj) launch_gemv<float, true, false>(Z, N, X, ldx, Y, ldy, nullptr, 0, R, skip, sks, s);
        else launch_gemv<float, false, false>(Z, N, X, ldx, Y, ldy, nullptr, 0, R, skip, sks, s);
    }
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
