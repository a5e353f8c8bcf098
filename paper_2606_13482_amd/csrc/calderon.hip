// Multiplicative Calderon preconditioner of the EFIE (Andriulli et al., IEEE TAP
// 56(8), 2008), which the paper uses in all of its simulations (Sec. VI-A, remark
// on the star-split operator; Sec. VII, setup of the results) without restating it.
//
// M = -G^{-1} T_BC G^{-T}, stored like T in packed symmetric FP64 tiles (M is
// complex symmetric because T_BC is), so that one preconditioned product costs
// two packed products.  Pieces:
//   * barycentric refinement (host): each triangle cut into six by its centroid
//     and edge midpoints; vertices = original, then the midpoint of RWG edge m at
//     nv + m, then the centroid of triangle t at nv + N + t;
//   * BC functions (host): b_m is the combination of refined RWG functions on
//     the dual cells (refined triangles around a vertex) of the two ends of edge
//     m with charge +1/A(hi) spread uniformly over the cell of the higher vertex
//     and -1/A(lo) over the lower one's, flux 1/2 through each of the two refined
//     edges from the midpoint of m to the centroids of c+ and c-, and no flux
//     through the two halves of edge m.  Walking around a cell from the child
//     next to one half of the dual edge, the flux through each radial edge is
//     the previous one plus the child's share of the charge;
//   * mixed Gram matrix G_mn = <n x b_m, f_n> (host, CSR): exact with the
//     three-edge-midpoint rule on each refined triangle (quadratic integrand);
//   * T_BC = C Z_b C^T (device): Z_b from the FP64 fill of the refined mesh; in
//     column chunks, each BC function's column of Z_b C^T gathered from the rows
//     of Z_b's dense FP64 copy (Z_b is symmetric) that its coefficients name, then
//     the sparse map C on the left;
//   * G^{-1} applied to all N columns at once by Chebyshev iteration on the
//     interval that holds G's spectrum (CG on the normal equations if it fails),
//     twice with a transpose in between, on row-major blocks so that the sparse
//     products read whole rows of 64 columns.
#include <algorithm>
#include <cstdlib>
#include <chrono>
#include <map>
#include <memory>
#include <mutex>
#include <unordered_map>

#include "bie_internal.hpp"

struct bie_calderon {
    const bie_op *op = nullptr;   // operator it was built for (mesh and k)
    bie_op *view = nullptr;       // N x N packed FP64 tiles of M, products through the packed kernels
    bie_op *tm = nullptr;         // T M (dense, split-BF16 copy only) for the preconditioned block products
    void *tmp = nullptr;          // 2 x tmp_R x N complex128 for the preconditioned solve
    int64_t tmp_R = 0;
    bie_calderon_info info{};
    bool counted = false;         // holds a reference on the setup pool
};

namespace bie {
namespace {

constexpr int CT = 256;

// Setup pool: freeing tens of GB costs about 30 ms per GB on this runtime once
// many buffers have come and gone, so the three largest transient buffers of a
// setup are kept (per device) for the next one while any preconditioner lives.
// Setups are serialised: they share these buffers.
struct SetupPool {
    void *buf[3] = {};
    size_t cap[3] = {};
};
std::mutex g_setup_mu;        // one setup at a time
std::mutex g_pool_mu;
std::map<int, SetupPool> g_pool;
int g_live = 0;               // live preconditioners
thread_local bool g_pool_on = false;

// frees one slot of this device's pool (the next setup that needs it allocates it again)
void setup_pool_drop(int slot)
{
    std::lock_guard<std::mutex> lk(g_pool_mu);
    int dev = 0;
    BIE_HIP(hipGetDevice(&dev));
    auto it = g_pool.find(dev);
    if (it == g_pool.end() || !it->second.buf[slot]) return;
    (void)hipFree(it->second.buf[slot]);
    it->second.buf[slot] = nullptr;
    it->second.cap[slot] = 0;
}

void setup_pool_release()
{
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (auto &kv : g_pool)
        for (int i = 0; i < 3; ++i)
            if (kv.second.buf[i]) (void)hipFree(kv.second.buf[i]);
    g_pool.clear();
}

struct Csr {
    std::vector<int64_t> ptr;
    std::vector<int32_t> idx;
    std::vector<double> val;
};

struct CsrDev {
    int64_t rows = 0;
    int64_t *ptr = nullptr;
    int32_t *idx = nullptr;
    double *val = nullptr;
    void upload(const Csr &c)
    {
        rows = int64_t(c.ptr.size()) - 1;
        BIE_HIP(hipMalloc(&ptr, c.ptr.size() * sizeof(int64_t)));
        BIE_HIP(hipMalloc(&idx, std::max<size_t>(1, c.idx.size()) * sizeof(int32_t)));
        BIE_HIP(hipMalloc(&val, std::max<size_t>(1, c.val.size()) * sizeof(double)));
        BIE_HIP(hipMemcpy(ptr, c.ptr.data(), c.ptr.size() * sizeof(int64_t), hipMemcpyHostToDevice));
        BIE_HIP(hipMemcpy(idx, c.idx.data(), c.idx.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        BIE_HIP(hipMemcpy(val, c.val.data(), c.val.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    ~CsrDev()
    {
        if (ptr) (void)hipFree(ptr);
        if (idx) (void)hipFree(idx);
        if (val) (void)hipFree(val);
    }
};

// ----------------------------------------------------------------------------- kernels

// Y[:, c] = A X[:, c] for a real CSR matrix A and complex columns (grid.y = columns).
__global__ __launch_bounds__(CT) void k_csr_cols(int64_t rows, const int64_t *__restrict__ ptr,
                                                 const int32_t *__restrict__ idx, const double *__restrict__ val,
                                                 const double2 *__restrict__ X, int64_t ldx, double2 *__restrict__ Y,
                                                 int64_t ldy)
{
    const int64_t i = int64_t(blockIdx.x) * CT + threadIdx.x;
    if (i >= rows) return;
    const double2 *x = X + int64_t(blockIdx.y) * ldx;
    double re = 0.0, im = 0.0;
    for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
        const double a = val[k];
        const double2 v = x[idx[k]];
        re += a * v.x;
        im += a * v.y;
    }
    Y[int64_t(blockIdx.y) * ldy + i] = make_double2(re, im);
}

// Y = A X for a real CSR matrix A and n x nc complex matrices stored row-major
// (entry (i, c) at i nc + c): a wave takes 64 consecutive columns of one row, so
// each nonzero reads 1 KiB contiguously.  Grid: rows x column blocks, rows
// fastest, so that the workgroups in flight share one column slice of X (kept in
// the last-level cache while they walk the rows).
__global__ __launch_bounds__(CT) void k_csr_rm(const int64_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                                               const double *__restrict__ val, int64_t nc, const double2 *__restrict__ X,
                                               double2 *__restrict__ Y)
{
    const int64_t c = int64_t(blockIdx.y) * CT + threadIdx.x, i = blockIdx.x;
    if (c >= nc) return;
    double re = 0.0, im = 0.0;
    for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
        const double a = val[k];
        const double2 v = X[int64_t(idx[k]) * nc + c];
        re += a * v.x;
        im += a * v.y;
    }
    Y[i * nc + c] = make_double2(re, im);
}

// Column c of Yc = Z_b (row j0 + c of C)^T for the symmetric refined matrix Z_b, from
// its dense FP64 operand (row e at e Kp, (Re, Im) pairs): the combination of the
// rows e of the BC map's nonzeros, read contiguously (grid: row blocks x columns).
__global__ __launch_bounds__(CT) void k_bc_gather(const double *__restrict__ A64, int64_t Kp, int64_t Nb,
                                                  const int64_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                                                  const double *__restrict__ val, int64_t j0, double2 *__restrict__ Yc,
                                                  int64_t ld)
{
    const int64_t i = int64_t(blockIdx.x) * CT + threadIdx.x, c = blockIdx.y;
    if (i >= Nb) return;
    double re = 0.0, im = 0.0;
    for (int64_t k = ptr[j0 + c]; k < ptr[j0 + c + 1]; ++k) {
        const double a = val[k];
        const double2 z = *reinterpret_cast<const double2 *>(A64 + int64_t(idx[k]) * Kp + 2 * i);
        re += a * z.x;
        im += a * z.y;
    }
    Yc[c * ld + i] = make_double2(re, im);
}

__global__ void k_fill0(int64_t n, double2 *__restrict__ a)
{
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x)
        a[e] = make_double2(0.0, 0.0);
}

// Row-major n x n: partial sums over the rows i = s, s + S, ... of |X(i, c)|^2
// (grid: column blocks x S slices), then their sum per column.
__global__ __launch_bounds__(CT) void k_colsq_part(int64_t n, const double2 *__restrict__ X, double *__restrict__ part)
{
    const int64_t c = int64_t(blockIdx.x) * CT + threadIdx.x;
    if (c >= n) return;
    double s = 0.0;
    for (int64_t i = blockIdx.y; i < n; i += gridDim.y) {
        const double2 v = X[i * n + c];
        s += v.x * v.x + v.y * v.y;
    }
    part[int64_t(blockIdx.y) * n + c] = s;
}

__global__ __launch_bounds__(CT) void k_colsq_fin(int64_t n, int S, const double *__restrict__ part,
                                                  double *__restrict__ out)
{
    const int64_t c = int64_t(blockIdx.x) * CT + threadIdx.x;
    if (c >= n) return;
    double s = 0.0;
    for (int k = 0; k < S; ++k) s += part[int64_t(k) * n + c];
    out[c] = s;
}

// CGNR step, per column c of row-major n x n blocks: alpha = zz / ww; X += alpha P;
// R -= alpha W (grid-stride over the entries).
__global__ __launch_bounds__(CT) void k_cg_xr(int64_t n, const double *__restrict__ zz, const double *__restrict__ ww,
                                              const double2 *__restrict__ P, const double2 *__restrict__ W,
                                              double2 *__restrict__ X, double2 *__restrict__ Rr)
{
    for (int64_t e = int64_t(blockIdx.x) * CT + threadIdx.x; e < n * n; e += int64_t(gridDim.x) * CT) {
        const int64_t c = e % n;
        const double a = ww[c] > 0.0 ? zz[c] / ww[c] : 0.0;
        const double2 p = P[e], w = W[e];
        double2 x = X[e], r = Rr[e];
        x.x += a * p.x;
        x.y += a * p.y;
        r.x -= a * w.x;
        r.y -= a * w.y;
        X[e] = x;
        Rr[e] = r;
    }
}

// Chebyshev step on row-major blocks (coefficients shared by every column):
// X += D; R -= W (W = G D); D = c1 D + c2 R.
__global__ __launch_bounds__(CT) void k_cheb(int64_t nn, double c1, double c2, const double2 *__restrict__ W,
                                             double2 *__restrict__ D, double2 *__restrict__ X, double2 *__restrict__ Rr)
{
    for (int64_t e = int64_t(blockIdx.x) * CT + threadIdx.x; e < nn; e += int64_t(gridDim.x) * CT) {
        const double2 d = D[e], w = W[e];
        double2 x = X[e], r = Rr[e];
        x.x += d.x;
        x.y += d.y;
        r.x -= w.x;
        r.y -= w.y;
        X[e] = x;
        Rr[e] = r;
        D[e] = make_double2(c1 * d.x + c2 * r.x, c1 * d.y + c2 * r.y);
    }
}

__global__ __launch_bounds__(CT) void k_scale_copy(int64_t nn, double a, const double2 *__restrict__ Xs,
                                                   double2 *__restrict__ Y)
{
    for (int64_t e = int64_t(blockIdx.x) * CT + threadIdx.x; e < nn; e += int64_t(gridDim.x) * CT) {
        const double2 v = Xs[e];
        Y[e] = make_double2(a * v.x, a * v.y);
    }
}

// CGNR direction, per column c of row-major blocks: beta = zn / zz; P = Z + beta P.
__global__ __launch_bounds__(CT) void k_cg_p(int64_t n, const double *__restrict__ zn, const double *__restrict__ zz,
                                             const double2 *__restrict__ Zv, double2 *__restrict__ P)
{
    for (int64_t e = int64_t(blockIdx.x) * CT + threadIdx.x; e < n * n; e += int64_t(gridDim.x) * CT) {
        const int64_t c = e % n;
        const double b = zz[c] > 0.0 ? zn[c] / zz[c] : 0.0;
        const double2 z = Zv[e], p = P[e];
        P[e] = make_double2(z.x + b * p.x, z.y + b * p.y);
    }
}

// B = A^T for column-major n x n complex matrices (32 x 32 tiles through LDS).
__global__ __launch_bounds__(256) void k_transpose(int64_t n, const double2 *__restrict__ A, double2 *__restrict__ B)
{
    __shared__ double2 t[32][33];
    const int64_t c0 = int64_t(blockIdx.y) * 32, r0 = int64_t(blockIdx.x) * 32;
    for (int k = threadIdx.y; k < 32; k += 8) {
        const int64_t r = r0 + threadIdx.x, c = c0 + k;
        if (r < n && c < n) t[k][threadIdx.x] = A[c * n + r];
    }
    __syncthreads();
    for (int k = threadIdx.y; k < 32; k += 8) {
        const int64_t r = c0 + threadIdx.x, c = r0 + k;   // B(r, c) = A(c, r)
        if (r < n && c < n) B[c * n + r] = t[threadIdx.x][k];
    }
}

// Packed symmetric tiles (I <= J, row-major tiles of TB x TB, row-major over the
// upper triangle) of s (A + A^T)/2 for a dense column-major n x n matrix A.
__global__ __launch_bounds__(256) void k_pack_sym(int64_t n, int64_t nT, const double2 *__restrict__ A, double s,
                                                  double2 *__restrict__ Zp)
{
    const int64_t I = blockIdx.y, J = blockIdx.x;
    if (J < I) return;
    double2 *tile = Zp + (I * nT - I * (I - 1) / 2 + (J - I)) * int64_t(TB * TB);
    for (int e = threadIdx.x; e < TB * TB; e += 256) {
        const int64_t i = I * TB + e / TB, j = J * TB + e % TB;
        double2 v = make_double2(0.0, 0.0);
        if (i < n && j < n) {
            const double2 a = A[j * n + i], b = A[i * n + j];
            v = make_double2(0.5 * s * (a.x + b.x), 0.5 * s * (a.y + b.y));
        }
        tile[e] = v;
    }
}

// Columns j0 .. j0 + nc - 1 of the n x n identity, dense (n entries per column).
__global__ __launch_bounds__(256) void k_unit_cols(int64_t n, int64_t j0, int64_t nc, double2 *__restrict__ X)
{
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n * nc; e += int64_t(gridDim.x) * blockDim.x)
        X[e] = make_double2(e % n == j0 + e / n ? 1.0 : 0.0, 0.0);
}

__global__ __launch_bounds__(256) void k_add_cols(int64_t n, const double2 *__restrict__ a, double2 *__restrict__ x)
{
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x) {
        const double2 v = a[e];
        double2 y = x[e];
        y.x += v.x;
        y.y += v.y;
        x[e] = y;
    }
}

// ----------------------------------------------------------------------------- host geometry

struct V3 {
    double x, y, z;
};
inline V3 vsub(V3 a, V3 b) { return { a.x - b.x, a.y - b.y, a.z - b.z }; }
inline V3 vmid(V3 a, V3 b) { return { 0.5 * (a.x + b.x), 0.5 * (a.y + b.y), 0.5 * (a.z + b.z) }; }
inline V3 vcross(V3 a, V3 b) { return { a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x }; }
inline double vdot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 vscale(V3 a, double s) { return { a.x * s, a.y * s, a.z * s }; }

// Barycentric refinement of a validated closed mesh.
void refine(const Mesh &M, std::vector<double> &Vb, std::vector<int32_t> &Tb)
{
    const int64_t nv = M.nv, N = M.N, F = M.F;
    Vb.assign(3 * (nv + N + F), 0.0);
    std::copy(M.V.begin(), M.V.end(), Vb.begin());
    for (int64_t m = 0; m < N; ++m)
        for (int d = 0; d < 3; ++d)
            Vb[3 * (nv + m) + d] = 0.5 * (M.V[3 * M.edges[4 * m] + d] + M.V[3 * M.edges[4 * m + 1] + d]);
    for (int64_t t = 0; t < F; ++t)
        for (int d = 0; d < 3; ++d)
            Vb[3 * (nv + N + t) + d] =
                (M.V[3 * M.T[3 * t] + d] + M.V[3 * M.T[3 * t + 1] + d] + M.V[3 * M.T[3 * t + 2] + d]) / 3.0;
    Tb.assign(18 * F, 0);
    for (int64_t t = 0; t < F; ++t) {
        const int32_t g = int32_t(nv + N + t);
        for (int k = 0; k < 3; ++k) {
            const int32_t a = M.T[3 * t + k], b = M.T[3 * t + (k + 1) % 3];
            const int32_t mab = int32_t(nv + M.slot_m[3 * t + (k + 2) % 3]);   // edge a-b is opposite vertex k+2
            int32_t *c0 = &Tb[3 * (6 * t + 2 * k)];
            c0[0] = a; c0[1] = mab; c0[2] = g;
            c0[3] = mab; c0[4] = b; c0[5] = g;
        }
    }
}

// BC coefficients (CSR, N rows over the refined RWG functions) and the mixed Gram
// matrix (CSR, N x N) and its transpose.
void bc_and_gram(const Mesh &M, const Mesh &B, Csr &C, Csr &G, Csr &Gt)
{
    const int64_t nv = M.nv, N = M.N, nvb = B.nv;
    std::unordered_map<uint64_t, int32_t> eid;
    eid.reserve(size_t(B.N) * 2);
    for (int64_t e = 0; e < B.N; ++e) eid[uint64_t(B.edges[4 * e]) * uint64_t(nvb) + uint64_t(B.edges[4 * e + 1])] = int32_t(e);
    auto edge_of = [&](int32_t a, int32_t b) -> int32_t {
        const auto it = eid.find(uint64_t(std::min(a, b)) * uint64_t(nvb) + uint64_t(std::max(a, b)));
        if (it == eid.end()) throw Error(BIE_EMESH, "refined mesh lacks an expected edge");
        return it->second;
    };
    auto sigma = [&](int32_t e, int32_t t) { return B.edges[4 * e + 2] == t ? 1.0 : -1.0; };
    auto across = [&](int32_t e, int32_t t) { return B.edges[4 * e + 2] == t ? B.edges[4 * e + 3] : B.edges[4 * e + 2]; };
    auto Vb = [&](int32_t v) { return V3{ B.V[3 * v], B.V[3 * v + 1], B.V[3 * v + 2] }; };
    // the radial edge of child t (corner v) other than e
    auto other_radial = [&](int32_t t, int32_t v, int32_t e) {
        int32_t x[2], n = 0;
        for (int k = 0; k < 3; ++k)
            if (B.T[3 * t + k] != v) x[n++] = B.T[3 * t + k];
        const int32_t e1 = edge_of(v, x[0]), e2 = edge_of(v, x[1]);
        return e1 == e ? e2 : e1;
    };

    C.ptr.assign(1, 0);
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t m = 0; m < N; ++m) {
        row.clear();
        const int32_t lo = M.edges[4 * m], hi = M.edges[4 * m + 1], cp = M.edges[4 * m + 2], cm = M.edges[4 * m + 3];
        const int32_t mid = int32_t(nv + m);
        const int32_t half_p = edge_of(mid, int32_t(nv + N + cp)), half_m = edge_of(mid, int32_t(nv + N + cm));
        for (int side = 0; side < 2; ++side) {
            const int32_t v = side == 0 ? hi : lo;
            const double charge = side == 0 ? 1.0 : -1.0;
            const int32_t e0 = edge_of(v, mid);
            const int32_t t1 = B.edges[4 * e0 + 2] / 6 == cp ? B.edges[4 * e0 + 2] : B.edges[4 * e0 + 3];
            std::vector<int32_t> ts, es;
            int32_t t = t1, prev = e0;
            while (true) {
                ts.push_back(t);
                const int32_t nx = other_radial(t, v, prev);
                if (nx == e0) break;
                es.push_back(nx);
                t = across(nx, t);
                prev = nx;
                if (ts.size() > 256) throw Error(BIE_EMESH, "dual cell walk did not close");
            }
            double Ac = 0.0;
            for (int32_t c : ts) Ac += B.area[c];
            double phi = 0.0;   // flux through the half of edge m: none
            for (size_t i = 0; i + 1 < ts.size(); ++i) {
                const double out_dual = i == 0 ? 0.5 * charge : 0.0;
                phi += charge * B.area[ts[i]] / Ac - out_dual;
                row.emplace_back(es[i], phi * sigma(es[i], ts[i]));
            }
            if (side == 0) {
                row.emplace_back(half_p, 0.5 * sigma(half_p, ts.front()));
                row.emplace_back(half_m, 0.5 * sigma(half_m, ts.back()));
            }
        }
        std::sort(row.begin(), row.end());
        for (auto &p : row) {
            C.idx.push_back(p.first);
            C.val.push_back(p.second);
        }
        C.ptr.push_back(int64_t(C.idx.size()));
    }

    // G_mn = <n x b_m, f_n>
    G.ptr.assign(1, 0);
    std::vector<double> acc(N, 0.0);
    std::vector<char> seen(N, 0);
    std::vector<int32_t> touched;
    for (int64_t m = 0; m < N; ++m) {
        touched.clear();
        for (int64_t k = C.ptr[m]; k < C.ptr[m + 1]; ++k) {
            const int32_t e = C.idx[k];
            const double ce = C.val[k];
            for (int side = 0; side < 2; ++side) {
                const int32_t t = B.edges[4 * e + 2 + side], T = t / 6;
                const V3 a = { M.V[3 * M.T[3 * T]], M.V[3 * M.T[3 * T] + 1], M.V[3 * M.T[3 * T] + 2] };
                const V3 b = { M.V[3 * M.T[3 * T + 1]], M.V[3 * M.T[3 * T + 1] + 1], M.V[3 * M.T[3 * T + 1] + 2] };
                const V3 c = { M.V[3 * M.T[3 * T + 2]], M.V[3 * M.T[3 * T + 2] + 1], M.V[3 * M.T[3 * T + 2] + 2] };
                V3 nrm = vcross(vsub(b, a), vsub(c, a));
                nrm = vscale(nrm, 1.0 / std::sqrt(vdot(nrm, nrm)));
                int32_t fb = -1;
                for (int q = 0; q < 3; ++q)
                    if (B.T[3 * t + q] != B.edges[4 * e] && B.T[3 * t + q] != B.edges[4 * e + 1]) fb = B.T[3 * t + q];
                const V3 p0 = Vb(B.T[3 * t]), p1 = Vb(B.T[3 * t + 1]), p2 = Vb(B.T[3 * t + 2]);
                const V3 xq[3] = { vmid(p0, p1), vmid(p1, p2), vmid(p2, p0) };
                const double sb = sigma(e, t) / (2.0 * B.area[t]);
                for (int sl = 0; sl < 3; ++sl) {
                    const int32_t n = M.slot_m[3 * T + sl];
                    const V3 vf = { M.V[3 * M.T[3 * T + sl]], M.V[3 * M.T[3 * T + sl] + 1], M.V[3 * M.T[3 * T + sl] + 2] };
                    const double sf = double(M.slot_s[3 * T + sl]) / (2.0 * M.area[T]);
                    double s = 0.0;
                    for (int q = 0; q < 3; ++q) {
                        const V3 rb = vcross(nrm, vscale(vsub(xq[q], Vb(fb)), sb));
                        s += vdot(rb, vscale(vsub(xq[q], vf), sf));
                    }
                    if (!seen[n]) {
                        seen[n] = 1;
                        touched.push_back(n);
                    }
                    acc[n] += ce * B.area[t] / 3.0 * s;
                }
            }
        }
        std::sort(touched.begin(), touched.end());
        for (int32_t n : touched) {
            G.idx.push_back(n);
            G.val.push_back(acc[n]);
            acc[n] = 0.0;
            seen[n] = 0;
        }
        G.ptr.push_back(int64_t(G.idx.size()));
    }
    // transpose
    Gt.ptr.assign(N + 1, 0);
    for (int32_t n : G.idx) Gt.ptr[n + 1] += 1;
    for (int64_t i = 0; i < N; ++i) Gt.ptr[i + 1] += Gt.ptr[i];
    Gt.idx.assign(G.idx.size(), 0);
    Gt.val.assign(G.val.size(), 0.0);
    std::vector<int64_t> fillp(Gt.ptr.begin(), Gt.ptr.end() - 1);
    for (int64_t m = 0; m < N; ++m)
        for (int64_t k = G.ptr[m]; k < G.ptr[m + 1]; ++k) {
            const int64_t d = fillp[G.idx[k]]++;
            Gt.idx[d] = int32_t(m);
            Gt.val[d] = G.val[k];
        }
}

// G X = B for the n columns of B by CG on the normal equations G^T G X = G^T B.
// R (input B, overwritten by the residual), X, P, W are n x n row-major (entry
// (i, c) at i n + c; column c is one right-hand side); sc holds 5 n + NSLICE n doubles.
constexpr int NSLICE = 64;

void gram_solve(const CsrDev &G, const CsrDev &Gt, int64_t n, double2 *Rr, double2 *X, double2 *P, double2 *W,
                double *sc, hipStream_t s, int64_t &iters, double &relres)
{
    const int64_t nn = n * n;
    double *zz = sc, *zn = sc + n, *ww = sc + 2 * n, *rr = sc + 3 * n, *bb = sc + 4 * n, *part = sc + 5 * n;
    const unsigned cb = unsigned((n + CT - 1) / CT);
    const dim3 mm(unsigned(n), cb);                               // sparse products: rows x column blocks
    const unsigned ew = unsigned(std::min<int64_t>((nn + CT - 1) / CT, 16384));
    auto colsq = [&](const double2 *A, double *out) {
        hipLaunchKernelGGL(k_colsq_part, dim3(cb, NSLICE), dim3(CT), 0, s, n, A, part);
        hipLaunchKernelGGL(k_colsq_fin, dim3(cb), dim3(CT), 0, s, n, NSLICE, (const double *)part, out);
    };
    hipLaunchKernelGGL(k_fill0, dim3(2048), dim3(256), 0, s, nn, X);
    colsq(Rr, bb);
    hipLaunchKernelGGL(k_csr_rm, mm, dim3(CT), 0, s, Gt.ptr, Gt.idx, Gt.val, n, Rr, P);   // z = G^T r
    colsq(P, zz);
    BIE_HIP(hipGetLastError());
    std::vector<double> hb(n), hr(n);
    BIE_HIP(hipMemcpyAsync(hb.data(), bb, n * sizeof(double), hipMemcpyDeviceToHost, s));
    BIE_HIP(hipStreamSynchronize(s));
    const double target = 1e-13;
    const int64_t maxit = 2000;
    relres = 1.0;
    for (iters = 1; iters <= maxit; ++iters) {
        hipLaunchKernelGGL(k_csr_rm, mm, dim3(CT), 0, s, G.ptr, G.idx, G.val, n, P, W);      // w = G p
        colsq(W, ww);
        hipLaunchKernelGGL(k_cg_xr, dim3(ew), dim3(CT), 0, s, n, zz, ww, P, W, X, Rr);
        hipLaunchKernelGGL(k_csr_rm, mm, dim3(CT), 0, s, Gt.ptr, Gt.idx, Gt.val, n, Rr, W);  // z = G^T r
        colsq(W, zn);
        hipLaunchKernelGGL(k_cg_p, dim3(ew), dim3(CT), 0, s, n, zn, zz, W, P);
        BIE_HIP(hipGetLastError());
        std::swap(zz, zn);
        if (iters % 8 == 0 || iters == maxit) {
            colsq(Rr, rr);
            BIE_HIP(hipMemcpyAsync(hr.data(), rr, n * sizeof(double), hipMemcpyDeviceToHost, s));
            BIE_HIP(hipStreamSynchronize(s));
            relres = 0.0;
            for (int64_t c = 0; c < n; ++c)
                if (hb[c] > 0.0) relres = std::max(relres, std::sqrt(hr[c] / hb[c]));
            if (relres <= target) break;
        }
    }
    if (relres > target) throw Error(BIE_ENUMERIC, "Gram solve of the Calderon preconditioner did not converge");
    iters = std::min(iters, maxit);
}

// G X = B by Chebyshev iteration on the interval [GA, GB] of the real axis (Saad,
// Iterative Methods for Sparse Linear Systems, Sec. 12.3).  The spectrum of the
// mixed Gram matrix lies in [1/3, 1) up to imaginary parts near 1e-3 on every mesh
// tried (spheres, ellipsoids up to 1:2:3, rounded cubes, area ratios up to 6):
// one sparse product per step and no reductions, about 0.3 per step.  The residual
// is checked every 4 steps; if it has not fallen by half since the last check (a
// spectrum outside the interval), false is returned and R, X are undefined.
constexpr double GA = 0.30, GB = 1.05;

bool gram_solve_cheb(const CsrDev &G, int64_t n, double2 *Rr, double2 *X, double2 *D, double2 *W, double *sc,
                     hipStream_t s, int64_t &iters, double &relres)
{
    const int64_t nn = n * n;
    double *rr = sc + 3 * n, *bb = sc + 4 * n, *part = sc + 5 * n;
    const unsigned cb = unsigned((n + CT - 1) / CT);
    const dim3 mm(unsigned(n), cb);
    const unsigned ew = unsigned(std::min<int64_t>((nn + CT - 1) / CT, 16384));
    auto colsq = [&](const double2 *A, double *out) {
        hipLaunchKernelGGL(k_colsq_part, dim3(cb, NSLICE), dim3(CT), 0, s, n, A, part);
        hipLaunchKernelGGL(k_colsq_fin, dim3(cb), dim3(CT), 0, s, n, NSLICE, (const double *)part, out);
    };
    const double theta = 0.5 * (GB + GA), delta = 0.5 * (GB - GA), sigma = theta / delta;
    hipLaunchKernelGGL(k_fill0, dim3(2048), dim3(256), 0, s, nn, X);
    colsq(Rr, bb);
    hipLaunchKernelGGL(k_scale_copy, dim3(ew), dim3(CT), 0, s, nn, 1.0 / theta, (const double2 *)Rr, D);
    BIE_HIP(hipGetLastError());
    std::vector<double> hb(n), hr(n);
    BIE_HIP(hipMemcpyAsync(hb.data(), bb, n * sizeof(double), hipMemcpyDeviceToHost, s));
    BIE_HIP(hipStreamSynchronize(s));
    const double target = 1e-13;
    double rho = 1.0 / sigma, last = 1.0;
    relres = 1.0;
    for (iters = 1; iters <= 200; ++iters) {
        const double rhon = 1.0 / (2.0 * sigma - rho);
        hipLaunchKernelGGL(k_csr_rm, mm, dim3(CT), 0, s, G.ptr, G.idx, G.val, n, D, W);   // W = G D
        hipLaunchKernelGGL(k_cheb, dim3(ew), dim3(CT), 0, s, nn, rhon * rho, 2.0 * rhon / delta, W, D, X, Rr);
        BIE_HIP(hipGetLastError());
        rho = rhon;
        if (iters % 4 == 0) {
            colsq(Rr, rr);
            BIE_HIP(hipMemcpyAsync(hr.data(), rr, n * sizeof(double), hipMemcpyDeviceToHost, s));
            BIE_HIP(hipStreamSynchronize(s));
            relres = 0.0;
            for (int64_t c = 0; c < n; ++c)
                if (hb[c] > 0.0) relres = std::max(relres, std::sqrt(hr[c] / hb[c]));
            if (relres <= target) return true;
            if (!(relres < 0.5 * last)) return false;
            last = relres;
        }
    }
    return false;
}

// G X = B: Chebyshev, or CG on the normal equations from the saved B if it fails.
void gram_solve_any(const CsrDev &G, const CsrDev &Gt, int64_t n, double2 *Rr, double2 *X, double2 *P, double2 *W,
                    double2 *Bs, double *sc, hipStream_t s, int64_t &iters, double &relres)
{
    const int64_t nn = n * n;
    const unsigned ew = unsigned(std::min<int64_t>((nn + CT - 1) / CT, 16384));
    const char *env = getenv("BIE_CALDERON_GRAM");
    if (env && std::string(env) == "cgnr") {
        gram_solve(G, Gt, n, Rr, X, P, W, sc, s, iters, relres);
        return;
    }
    hipLaunchKernelGGL(k_scale_copy, dim3(ew), dim3(CT), 0, s, nn, 1.0, (const double2 *)Rr, Bs);
    BIE_HIP(hipGetLastError());
    if (gram_solve_cheb(G, n, Rr, X, P, W, sc, s, iters, relres)) return;
    int64_t it2 = 0;
    hipLaunchKernelGGL(k_scale_copy, dim3(ew), dim3(CT), 0, s, nn, 1.0, (const double2 *)Bs, Rr);
    gram_solve(G, Gt, n, Rr, X, P, W, sc, s, it2, relres);
    iters += it2;
}

}  // namespace

// Largest N for which the preconditioner is built.  The refined mesh has 6 N
// unknowns and 4 N triangles: its fill's pair scratch (144 B per triangle pair,
// 1152 N^2 bytes) beside its packed FP64 matrix (288 N^2) is the peak of the
// fill, 217 GB at this N; then the packed matrix and its dense copy (864 N^2)
// with five N x N work matrices (80 N^2).  The pool keeps the pair scratch for
// the next setup only while the rest of the setup fits beside it (checked with
// hipMemGetInfo after the fill); otherwise it is freed first, so the peak stays
// max(1440, 944) N^2 bytes.
constexpr int64_t CALDERON_MAX_N = 12288;

bool setup_pool_active() { return g_pool_on; }

void *setup_pool_get(int slot, size_t bytes)
{
    std::lock_guard<std::mutex> lk(g_pool_mu);
    int dev = 0;
    BIE_HIP(hipGetDevice(&dev));
    SetupPool &p = g_pool[dev];
    if (p.cap[slot] < bytes) {
        if (p.buf[slot]) (void)hipFree(p.buf[slot]);
        p.buf[slot] = nullptr;
        p.cap[slot] = 0;
        BIE_HIP(hipMalloc(&p.buf[slot], bytes));
        p.cap[slot] = bytes;
    }
    return p.buf[slot];
}

bie_calderon *calderon_create(const bie_op *op, hipStream_t s)
{
    std::lock_guard<std::mutex> serial(g_setup_mu);
    struct PoolScope {
        PoolScope() { g_pool_on = true; }
        ~PoolScope()
        {
            g_pool_on = false;
            bool none;
            {
                std::lock_guard<std::mutex> lk(g_pool_mu);
                none = g_live == 0;
            }
            if (none) setup_pool_release();   // a failed first setup keeps nothing
        }
    } scope;
    const auto t0 = std::chrono::steady_clock::now();
    const Mesh &M = op->mesh;
    const int64_t N = M.N;
    if (N > CALDERON_MAX_N) throw Error(BIE_EINVAL, "Calderon preconditioner: N above 12288 (refined dense matrix too large)");
    if (op->star) throw Error(BIE_EINVAL, "Calderon preconditioner: needs an assembled operator");
    std::vector<double> Vb;
    std::vector<int32_t> Tb;
    refine(M, Vb, Tb);
    bie_op *opb = nullptr;
    bie_fill_opts fo{};
    fo.storage = BIE_C128;
    fo.near_factor = 2.0;
    int rc = bie_op_create(Vb.data(), int64_t(Vb.size() / 3), Tb.data(), int64_t(Tb.size() / 3), op->k, &fo, s, &opb);
    if (rc != BIE_OK) throw Error(rc, std::string("Calderon preconditioner, refined mesh: ") + bie_last_error());
    std::unique_ptr<bie_op, void (*)(bie_op *)> hold(opb, bie_op_destroy);
    const int64_t Nb = opb->mesh.N;
    if (Nb != 9 * M.F) throw Error(BIE_EMESH, "refined mesh has an unexpected edge count");
    {
        // the fill's pair scratch (pool slot 0) is not read again in this setup:
        // keep it for the next one only if the refined matrix's dense copy, the
        // work matrices and M's storage still fit beside it
        size_t freeb = 0, totb = 0;
        BIE_HIP(hipMemGetInfo(&freeb, &totb));
        const double n2 = double(N) * double(N);
        const double later = 16.0 * double(Nb) * double(Nb) + (5 * 16 + 8 + 16 + 8 + 16) * n2 + double(size_t(4) << 30);
        if (double(freeb) < later) setup_pool_drop(0);
    }

    Csr C, G, Gt;
    bc_and_gram(M, opb->mesh, C, G, Gt);
    CsrDev dC, dG, dGt;
    dC.upload(C);
    dG.upload(G);
    dGt.upload(Gt);

    std::unique_ptr<bie_calderon, void (*)(bie_calderon *)> pc(new bie_calderon(), calderon_destroy);
    pc->op = op;
    pc->info.N = N;
    pc->info.Nb = Nb;
    pc->info.nnz_bc = int64_t(C.idx.size());
    pc->info.nnz_gram = int64_t(G.idx.size());

    // dense work, n x n each: T_BC / residual, X, P (Chebyshev direction), W, and the
    // saved right-hand side for the fallback; column scalars and partial sums
    const int64_t nn = N * N;
    double2 *buf[5] = {};
    double *scal = nullptr;
    struct Free {
        double2 **b;
        double **sc;
        ~Free()
        {
            for (int i = 0; i < 5; ++i)
                if (b[i]) (void)hipFree(b[i]);
            if (*sc) (void)hipFree(*sc);
        }
    } guard{ buf, &scal };
    for (int i = 0; i < 5; ++i) BIE_HIP(hipMalloc(&buf[i], size_t(nn) * sizeof(double2)));
    BIE_HIP(hipMalloc(&scal, size_t((5 + NSLICE) * N) * sizeof(double)));

    // T_BC in column chunks: Yc = Z_b C^T[:, chunk] gathered from the rows of the
    // refined matrix's dense FP64 operand (Z_b symmetric: column e = row e), then
    // T_BC[:, chunk] = C Yc
    {
        dense64_setup(opb, s);
        const int64_t ch = std::min<int64_t>(N, 512);
        double2 *Yc = nullptr;
        BIE_HIP(hipMalloc(&Yc, size_t(Nb * ch) * sizeof(double2)));
        struct F2 {
            double2 *p;
            ~F2() { if (p) (void)hipFree(p); }
        } fy{ Yc };
        for (int64_t j0 = 0; j0 < N; j0 += ch) {
            const int64_t nc = std::min(ch, N - j0);
            hipLaunchKernelGGL(k_bc_gather, dim3(unsigned((Nb + CT - 1) / CT), unsigned(nc)), dim3(CT), 0, s,
                               (const double *)opb->A64, opb->d64_Kp, Nb, dC.ptr, dC.idx, dC.val, j0, Yc, Nb);
            BIE_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_csr_cols, dim3(unsigned((N + CT - 1) / CT), unsigned(nc)), dim3(CT), 0, s, N, dC.ptr,
                               dC.idx, dC.val, Yc, Nb, buf[0] + j0 * N, N);
            BIE_HIP(hipGetLastError());
        }
        BIE_HIP(hipStreamSynchronize(s));
    }
    hold.reset();   // the refined operator is no longer needed

    // A1 = G^{-1} T_BC (into buf1); M' = G^{-1} A1^T (into buf1 again, A1^T in buf0)
    gram_solve_any(dG, dGt, N, buf[0], buf[1], buf[2], buf[3], buf[4], scal, s, pc->info.cg_iters[0],
                   pc->info.cg_relres[0]);
    hipLaunchKernelGGL(k_transpose, dim3(unsigned((N + 31) / 32), unsigned((N + 31) / 32)), dim3(32, 8), 0, s, N,
                       buf[1], buf[0]);
    BIE_HIP(hipGetLastError());
    gram_solve_any(dG, dGt, N, buf[0], buf[1], buf[2], buf[3], buf[4], scal, s, pc->info.cg_iters[1],
                   pc->info.cg_relres[1]);

    // M = -(M' + M'^T)/2 in packed tiles
    bie_op *v = new bie_op();
    pc->view = v;
    v->device = op->device;
    v->k = op->k;
    v->storage = BIE_C128;
    v->mesh.N = N;
    packed_setup(v->pk, N);
    BIE_HIP(hipMalloc(&v->Z64, size_t(v->pk.ntiles) * TB * TB * sizeof(double2)));
    hipLaunchKernelGGL(k_pack_sym, dim3(unsigned(v->pk.nT), unsigned(v->pk.nT)), dim3(256), 0, s, N, v->pk.nT,
                       buf[1], -1.0, (double2 *)v->Z64);
    BIE_HIP(hipGetLastError());
    BIE_HIP(hipStreamSynchronize(s));
    if (op->Abf) calderon_tm(pc.get(), s);   // block products of the preconditioned mixed solves
    pc->info.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        ++g_live;
        pc->counted = true;
    }
    return pc.release();
}

bie_op *calderon_tm(const bie_calderon *pcc, hipStream_t s)
{
    bie_calderon *pc = const_cast<bie_calderon *>(pcc);
    if (pc->tm) return pc->tm;
    const bie_op *op = pc->op;
    if (!op->Z64) throw Error(BIE_EINVAL, "Calderon preconditioner: T M needs the FP64 matrix");
    const int64_t N = pc->info.N, ch = std::min<int64_t>(N, 512);
    double2 *A = nullptr, *I = nullptr, *Mc = nullptr;
    struct F3 {
        double2 **p[3];
        ~F3()
        {
            for (auto q : p)
                if (*q) (void)hipFree(*q);
        }
    } guard{ { &A, &I, &Mc } };
    BIE_HIP(hipMalloc(&A, size_t(N) * N * sizeof(double2)));
    BIE_HIP(hipMalloc(&I, size_t(N) * ch * sizeof(double2)));
    BIE_HIP(hipMalloc(&Mc, size_t(N) * ch * sizeof(double2)));
    // column chunk of T M: unit vectors, M on the FP64 matrix cores, then T
    for (int64_t j0 = 0; j0 < N; j0 += ch) {
        const int64_t nc = std::min(ch, N - j0);
        hipLaunchKernelGGL(k_unit_cols, dim3(2048), dim3(256), 0, s, N, j0, nc, I);
        BIE_HIP(hipGetLastError());
        gemm64_product(pc->view, I, N, Mc, N, nullptr, 0, nc, nullptr, s);
        gemm64_product(op, Mc, N, A + j0 * N, N, nullptr, 0, nc, nullptr, s);
    }
    std::unique_ptr<bie_op, void (*)(bie_op *)> t(new bie_op(), bie_op_destroy);
    t->device = op->device;
    t->k = op->k;
    t->storage = BIE_SPLIT_BF16;
    t->mesh.N = N;
    split_dense(t.get(), A, s);   // synchronises
    pc->tm = t.release();
    return pc->tm;
}

void calderon_destroy(bie_calderon *pc)
{
    if (!pc) return;
    if (pc->view) bie_op_destroy(pc->view);   // every buffer the products made on it too
    if (pc->tm) bie_op_destroy(pc->tm);
    if (pc->tmp) (void)hipFree(pc->tmp);
    bool last = false;
    if (pc->counted) {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        last = --g_live == 0;
    }
    delete pc;
    if (last) {   // wait for a setup in progress on another thread, which may be using the pool
        std::lock_guard<std::mutex> serial(g_setup_mu);
        bool none;
        {
            std::lock_guard<std::mutex> lk(g_pool_mu);
            none = g_live == 0;
        }
        if (none) setup_pool_release();
    }
}

const bie_op *calderon_operator(const bie_calderon *pc) { return pc->op; }
const bie_calderon_info &calderon_info(const bie_calderon *pc) { return pc->info; }

// The operator holding M (packed FP64 tiles); split: also its split-BF16 copy for
// the block product (made on first use).
bie_op *calderon_view(const bie_calderon *pc, bool split, hipStream_t s)
{
    if (split && !pc->view->Abf) split_matrix(pc->view, s);
    return pc->view;
}

// The operator holding M with an FP32 copy of its packed tiles as well (made on
// first use, freed with the preconditioner), for products in FP32 storage.
bie_op *calderon_view32(const bie_calderon *pc, hipStream_t s)
{
    bie_op *v = pc->view;
    if (!v->Z32) {
        const int64_t n = v->pk.ntiles * TB * TB;
        void *z = nullptr;
        BIE_HIP(hipMalloc(&z, size_t(n) * sizeof(float2)));
        convert_c128_to_c64(v->Z64, z, n, s);
        BIE_HIP(hipStreamSynchronize(s));
        v->Z32 = z;
    }
    return v;
}

// Two R x N complex128 scratch blocks for the preconditioned solve.
double2 *calderon_scratch(const bie_calderon *pcc, int64_t R, hipStream_t s)
{
    bie_calderon *pc = const_cast<bie_calderon *>(pcc);
    if (pc->tmp_R < R) {
        BIE_HIP(hipStreamSynchronize(s));
        if (pc->tmp) (void)hipFree(pc->tmp);
        pc->tmp = nullptr;
        pc->tmp_R = 0;
        BIE_HIP(hipMalloc(&pc->tmp, size_t(2 * R * pc->info.N) * sizeof(double2)));
        pc->tmp_R = R;
    }
    return static_cast<double2 *>(pc->tmp);
}

void calderon_apply(const bie_calderon *pc, const void *X, int64_t ldx, void *Y, int64_t ldy, int64_t R,
                    const int *skip, int64_t sks, hipStream_t s)
{
    product(pc->view, MAT64, true, X, ldx, Y, ldy, nullptr, 0, R, skip, sks, false, s);
}

// x += a for n complex entries.
void add_into(int64_t n, const void *a, void *x, hipStream_t s)
{
    hipLaunchKernelGGL(k_add_cols, dim3(unsigned(std::min<int64_t>((n + 255) / 256, 4096))), dim3(256), 0, s, n,
                       (const double2 *)a, (double2 *)x);
    BIE_HIP(hipGetLastError());
}

void zero_into(int64_t n, void *x, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill0, dim3(unsigned(std::min<int64_t>((n + 255) / 256, 4096))), dim3(256), 0, s, n,
                       (double2 *)x);
    BIE_HIP(hipGetLastError());
}

}  // namespace bie
