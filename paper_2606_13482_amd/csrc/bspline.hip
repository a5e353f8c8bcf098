// Single-level far field by tensor-product B-spline interpolation of the
// Green's function (the paper's Sec. III; stabilised knots of Sec. V-B; knot
// insertion of Sec. IV-B; buffer knots of Sec. III-B).
//
// Boxes: a uniform grid of cubes of side a; an RWG function belongs to the box
// holding the mean of its two triangle centroids; two boxes are far when their
// indices differ by more than one along some axis.  Along each axis a box
// carries degree-p splines on an open equidistant knot vector of s splines
// (knot spacing du = 1/(s - p) in box units) extended by sb buffer knots per
// side so that every support of its functions lies inside; r = (p - 1)/2
// interior knots are removed next to each end (the paper's table for odd p),
// and the stabilised splines interpolate at their n' equispaced points.  For
// odd p these points fall on the knots: every box's points lie on one lattice
// of spacing h = a du, so g between any two points of any two boxes is a value
// of g at a lattice vector and one table holds them all.
//
// Product y = Z~_far x for R columns:
//   moments (once):   m~[m][c][k] = sum_q coef_c(q) b~_k1(t1) b~_k2(t2) b~_k3(t3)
//                     at the 14 quadrature points of the two triangles of m,
//                     b~ = A b_eq with A = B_stab^-1 C (C by knot insertion),
//                     coef = s w (x - v)/2 for c = x, y, z and s w for the
//                     divergence (the fill's rule, areas cancelled);
//   aggregate:        M_Y[c][k] = sum_{n in Y} x_n m~[n][c][k];
//   translate:        L_X[c][i] = sum_{Y far} sum_k g(h (D_XY + i - k)) M_Y[c][k]
//                     (partial sums per chunk of far boxes);
//   disaggregate:     y_m = jk sum_{c<3} m~[m][c] . L_X[c] + m~[m][3] . L_X[3] / (jk).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "bie_internal.hpp"

namespace {

constexpr int NPT = 2 * bie::QPTS;   // quadrature points of one RWG function
constexpr int MAXP = 5;             // highest degree (odd: 1, 3, 5)
constexpr int MAXN = 24;            // most splines per axis (buffer included)
constexpr int FAR_CHUNK = 8;        // far source boxes per translation item

struct BsConst {
    int p, n, nst, npts;       // degree, equidistant splines, stabilised splines, nst^3
    double a;                  // box side
    double lo, hi;             // parameter interval of the interpolation domain (box = [0, 1])
    const double *knots;       // device: the n + p + 1 equidistant knots (buffer included)
    const double *A;           // device: nst x n, row-major (B_stab^-1 C)
};

// Nonzero B-splines at x: N[0..p] of splines span-p .. span (u[span] <= x < u[span+1],
// the last non-empty interval closed on the right); returns span.
__host__ __device__ inline int nonzero_splines(const double *u, int n, int p, double x, double *N)
{
    int span = p;
    while (span < n - 1 && x >= u[span + 1]) ++span;
    double left[MAXP + 1], right[MAXP + 1];
    N[0] = 1.0;
    for (int j = 1; j <= p; ++j) {
        left[j] = x - u[span + 1 - j];
        right[j] = u[span + j] - x;
        double carry = 0.0;
        for (int q = 0; q < j; ++q) {
            const double tmp = N[q] / (right[q + 1] + left[j - q]);
            N[q] = carry + right[q + 1] * tmp;
            carry = left[j - q] * tmp;
        }
        N[j] = carry;
    }
    return span;
}

// Transformed moments of one RWG function per block.
__global__ __launch_bounds__(256) void k_bs_moments(BsConst c, int64_t N, const int4 *__restrict__ rwg4,
                                                    const double *__restrict__ cent, const double *__restrict__ loc,
                                                    const double *__restrict__ vfree, const double *__restrict__ qw,
                                                    const double *__restrict__ box_lo, const int32_t *__restrict__ box_of,
                                                    double *__restrict__ mt)
{
    const int64_t m = blockIdx.x;
    if (m >= N) return;
    __shared__ double bt[NPT][3][MAXN];
    __shared__ double coef[NPT][4];
    const int4 e = rwg4[m];
    const double *lo = box_lo + 3 * int64_t(box_of[m]);
    const int tid = threadIdx.x;
    if (tid < NPT * 3) {
        const int q = tid / 3, ax = tid % 3;
        const int t = q < bie::QPTS ? e.x : e.y;
        const int qq = q % bie::QPTS;
        const double x = cent[3 * t + ax] + loc[(int64_t(t) * bie::QPTS + qq) * 3 + ax];
        const double tp = (x - lo[ax]) / c.a;
        double Nv[MAXP + 1];
        const int span = nonzero_splines(c.knots, c.n, c.p, fmin(fmax(tp, c.lo), c.hi), Nv);
        for (int k = 0; k < c.nst; ++k) {
            double v = 0.0;
            for (int l = 0; l <= c.p; ++l) v += c.A[k * c.n + span - c.p + l] * Nv[l];
            bt[q][ax][k] = v;
        }
    } else if (tid >= 64 && tid < 64 + NPT) {
        const int q = tid - 64;
        const bool plus = q < bie::QPTS;
        const int t = plus ? e.x : e.y, slot = plus ? e.z : e.w, qq = q % bie::QPTS;
        const double sw = (plus ? 1.0 : -1.0) * qw[qq];
        for (int d = 0; d < 3; ++d)
            coef[q][d] = 0.5 * sw * (loc[(int64_t(t) * bie::QPTS + qq) * 3 + d] - vfree[int64_t(t) * 9 + slot * 3 + d]);
        coef[q][3] = sw;
    }
    __syncthreads();
    const int n2 = c.nst * c.nst;
    for (int k = tid; k < c.npts; k += 256) {
        const int k1 = k / n2, k2 = (k / c.nst) % c.nst, k3 = k % c.nst;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        for (int q = 0; q < NPT; ++q) {
            const double b = bt[q][0][k1] * bt[q][1][k2] * bt[q][2][k3];
            s0 += coef[q][0] * b;
            s1 += coef[q][1] * b;
            s2 += coef[q][2] * b;
            s3 += coef[q][3] * b;
        }
        double *o = mt + m * 4 * int64_t(c.npts);
        o[k] = s0;
        o[c.npts + k] = s1;
        o[2 * c.npts + k] = s2;
        o[3 * c.npts + k] = s3;
    }
}

// g(h |d|) on the lattice vectors d in [-Q, Q] (per axis), z fastest.
__global__ __launch_bounds__(256) void k_bs_gtable(int qx, int qy, int qz, double h, double k, double2 *__restrict__ tab)
{
    const int64_t ny = 2 * qy + 1, nz = 2 * qz + 1;
    const int64_t total = (2 * qx + 1) * ny * nz;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < total; i += int64_t(gridDim.x) * 256) {
        const int64_t dz = i % nz - qz, dy = (i / nz) % ny - qy, dx = i / (ny * nz) - qx;
        const double r = h * sqrt(double(dx * dx + dy * dy + dz * dz));
        double2 g = make_double2(0.0, 0.0);
        if (r > 0.0) {
            double sn, cs;
            sincos(k * r, &sn, &cs);
            const double f = 1.0 / (4.0 * M_PI * r);
            g = make_double2(f * cs, -f * sn);
        }
        tab[i] = g;
    }
}

// M_Y[r][c][k] = sum_{n in box Y} x_r[n] m~[n][c][k]
__global__ __launch_bounds__(256) void k_bs_aggregate(int npts, int64_t N, int64_t nbox,
                                                      const int32_t *__restrict__ mem_ptr,
                                                      const int32_t *__restrict__ mem, const double *__restrict__ mt,
                                                      const double2 *__restrict__ X, double2 *__restrict__ agg)
{
    const int64_t Yb = blockIdx.x, r = blockIdx.y;
    const int32_t b0 = mem_ptr[Yb], b1 = mem_ptr[Yb + 1];
    const double2 *x = X + r * N;
    double2 *out = agg + (r * nbox + Yb) * 4 * int64_t(npts);
    for (int k = threadIdx.x; k < npts; k += 256) {
        double2 acc[4] = { { 0, 0 }, { 0, 0 }, { 0, 0 }, { 0, 0 } };
        for (int32_t t = b0; t < b1; ++t) {
            const int32_t n = mem[t];
            const double2 xv = x[n];
            const double *mn = mt + int64_t(n) * 4 * npts;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double v = mn[c * npts + k];
                acc[c].x += v * xv.x;
                acc[c].y += v * xv.y;
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) out[c * int64_t(npts) + k] = acc[c];
    }
}

constexpr int UPT = 4;   // target points per thread (n'^3 <= 1024)

// One item = (target box X, far source boxes far[f0 .. f1)): partial L.
__global__ __launch_bounds__(256) void k_bs_translate(int nst, int npts, int shift, int qx, int qy, int qz,
                                                      int64_t nbox, int64_t nitems, const int4 *__restrict__ items,
                                                      const int32_t *__restrict__ far, const int32_t *__restrict__ box_ijk,
                                                      const double2 *__restrict__ tab, const double2 *__restrict__ agg,
                                                      double2 *__restrict__ lpart)
{
    extern __shared__ double2 src[];   // 4 x npts
    const int64_t it = blockIdx.x, r = blockIdx.y;
    const int4 item = items[it];        // (X, f0, f1, -)
    const int tid = threadIdx.x;
    const int64_t sy = 2 * qz + 1, sx = (2 * qy + 1) * sy;
    const int n2 = nst * nst;
    double2 acc[UPT][4];
    int ti[UPT][3];
#pragma unroll
    for (int u = 0; u < UPT; ++u) {
        const int i = tid + 256 * u;
        ti[u][0] = i / n2;
        ti[u][1] = (i / nst) % nst;
        ti[u][2] = i % nst;
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[u][c] = make_double2(0.0, 0.0);
    }
    const int *bx = box_ijk + 3 * int64_t(item.x);
    for (int f = item.y; f < item.z; ++f) {
        const int32_t Yb = far[f];
        const int *by = box_ijk + 3 * int64_t(Yb);
        const int D0 = shift * (bx[0] - by[0]), D1 = shift * (bx[1] - by[1]), D2 = shift * (bx[2] - by[2]);
        __syncthreads();
        const double2 *A = agg + (r * nbox + Yb) * 4 * int64_t(npts);
        for (int e = tid; e < 4 * npts; e += 256) src[e] = A[e];
        __syncthreads();
        for (int j = 0; j < npts; ++j) {
            const int j1 = j / n2, j2 = (j / nst) % nst, j3 = j % nst;
            const double2 s0 = src[j], s1 = src[npts + j], s2 = src[2 * npts + j], s3 = src[3 * npts + j];
#pragma unroll
            for (int u = 0; u < UPT; ++u) {
                if (tid + 256 * u >= npts) continue;
                const int64_t idx = int64_t(D0 + ti[u][0] - j1 + qx) * sx + int64_t(D1 + ti[u][1] - j2 + qy) * sy +
                                    (D2 + ti[u][2] - j3 + qz);
                const double2 g = tab[idx];
                acc[u][0].x += g.x * s0.x - g.y * s0.y;
                acc[u][0].y += g.x * s0.y + g.y * s0.x;
                acc[u][1].x += g.x * s1.x - g.y * s1.y;
                acc[u][1].y += g.x * s1.y + g.y * s1.x;
                acc[u][2].x += g.x * s2.x - g.y * s2.y;
                acc[u][2].y += g.x * s2.y + g.y * s2.x;
                acc[u][3].x += g.x * s3.x - g.y * s3.y;
                acc[u][3].y += g.x * s3.y + g.y * s3.x;
            }
        }
    }
    double2 *out = lpart + (r * nitems + it) * 4 * int64_t(npts);
#pragma unroll
    for (int u = 0; u < UPT; ++u) {
        const int i = tid + 256 * u;
        if (i >= npts) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) out[c * int64_t(npts) + i] = acc[u][c];
    }
}

// y_r[m] = jk sum_{c<3} m~[m][c] . L_X[c] + m~[m][3] . L_X[3] / (jk), L_X summed
// over the items of X in order.
__global__ __launch_bounds__(256) void k_bs_disaggregate(int npts, int64_t N, int64_t nitems, double k,
                                                         const int32_t *__restrict__ box_of,
                                                         const int32_t *__restrict__ item_ptr,
                                                         const double *__restrict__ mt, const double2 *__restrict__ lpart,
                                                         double2 *__restrict__ Y)
{
    const int64_t m = blockIdx.x, r = blockIdx.y;
    const int32_t X = box_of[m];
    const int32_t i0 = item_ptr[X], i1 = item_ptr[X + 1];
    const double *mm = mt + m * 4 * int64_t(npts);
    double2 sv = make_double2(0.0, 0.0), ss = make_double2(0.0, 0.0);   // vector and scalar parts
    for (int kk = threadIdx.x; kk < npts; kk += 256) {
        double2 L[4] = { { 0, 0 }, { 0, 0 }, { 0, 0 }, { 0, 0 } };
        for (int32_t it = i0; it < i1; ++it) {
            const double2 *lp = lpart + (r * nitems + it) * 4 * int64_t(npts);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double2 v = lp[c * int64_t(npts) + kk];
                L[c].x += v.x;
                L[c].y += v.y;
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            sv.x += mm[c * npts + kk] * L[c].x;
            sv.y += mm[c * npts + kk] * L[c].y;
        }
        ss.x += mm[3 * npts + kk] * L[3].x;
        ss.y += mm[3 * npts + kk] * L[3].y;
    }
    __shared__ double red[4][256];
    red[0][threadIdx.x] = sv.x;
    red[1][threadIdx.x] = sv.y;
    red[2][threadIdx.x] = ss.x;
    red[3][threadIdx.x] = ss.y;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (int(threadIdx.x) < o)
            for (int c = 0; c < 4; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        // jk (a + jb) = -k b + j k a;  (a + jb) / (jk) = b / k - j a / k
        Y[r * N + m] = make_double2(-k * red[1][0] + red[3][0] / k, k * red[0][0] - red[2][0] / k);
    }
}

// ----------------------------------------------------------------------------- host: 1D spline algebra
std::vector<double> open_knots(int n, int p, double lo, double hi)
{
    std::vector<double> u(size_t(n + p + 1));
    for (int i = 0; i <= p; ++i) {
        u[i] = lo;
        u[n + i] = hi;
    }
    for (int i = p + 1; i < n; ++i) u[i] = lo + (hi - lo) * double(i - p) / double(n - p);
    return u;
}

// values of all n splines at x
std::vector<double> all_splines(const std::vector<double> &u, int p, double x)
{
    const int n = int(u.size()) - p - 1;
    std::vector<double> v(size_t(n), 0.0);
    double N[MAXP + 1];
    const int span = nonzero_splines(u.data(), n, p, x, N);
    for (int l = 0; l <= p; ++l) v[span - p + l] = N[l];
    return v;
}

// Boehm: insert ub into (u, w)
void insert_one(std::vector<double> &u, int p, std::vector<double> &w, double ub)
{
    const int n = int(w.size());
    int k = 0;
    while (k + 1 < int(u.size()) && u[k + 1] <= ub) ++k;
    std::vector<double> nw(size_t(n + 1));
    for (int i = 0; i <= n; ++i) {
        const double al = i <= k - p ? 1.0 : (i <= k ? (ub - u[i]) / (u[i + p] - u[i]) : 0.0);
        nw[i] = (i < n ? al * w[i] : 0.0) + (i >= 1 ? (1.0 - al) * w[i - 1] : 0.0);
    }
    u.insert(u.begin() + k + 1, ub);
    w.swap(nw);
}

// inverse of a small dense matrix (Gauss-Jordan, partial pivoting)
std::vector<double> invert(std::vector<double> A, int n)
{
    std::vector<double> I(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i) I[size_t(i) * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int pr = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[size_t(r) * n + c]) > std::fabs(A[size_t(pr) * n + c])) pr = r;
        if (!(std::fabs(A[size_t(pr) * n + c]) > 0.0)) throw bie::Error(BIE_ENUMERIC, "singular spline sampling matrix");
        for (int j = 0; j < n; ++j) {
            std::swap(A[size_t(c) * n + j], A[size_t(pr) * n + j]);
            std::swap(I[size_t(c) * n + j], I[size_t(pr) * n + j]);
        }
        const double d = A[size_t(c) * n + c];
        for (int j = 0; j < n; ++j) {
            A[size_t(c) * n + j] /= d;
            I[size_t(c) * n + j] /= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double f = A[size_t(r) * n + c];
            if (f == 0.0) continue;
            for (int j = 0; j < n; ++j) {
                A[size_t(r) * n + j] -= f * A[size_t(c) * n + j];
                I[size_t(r) * n + j] -= f * I[size_t(c) * n + j];
            }
        }
    }
    return I;
}

// The spline spaces of one box level along an axis (parameter coordinate, box
// = [0, 1]): the equidistant knots of n = s + 2 sb splines on [lo, hi], and
// A = B_stab^-1 C (nst x n, row-major): C writes the stabilised splines (r
// interior knots removed per side) in the equidistant ones by knot insertion,
// B_stab samples the stabilised splines at their nst equispaced points.
struct SplineMap {
    int n = 0, nst = 0;
    double lo = 0.0, hi = 1.0;
    std::vector<double> ueq, A;
};

SplineMap spline_map(int s, int p, int sb, int r)
{
    SplineMap m;
    const double du = 1.0 / double(s - p);
    m.n = s + 2 * sb;
    m.nst = m.n - 2 * r;
    m.lo = -sb * du;
    m.hi = 1.0 + sb * du;
    m.ueq = open_knots(m.n, p, m.lo, m.hi);
    const std::vector<double> &ueq = m.ueq;
    std::vector<double> ust(ueq.begin(), ueq.begin() + p + 1);
    for (int i = p + 1 + r; i < m.n - r; ++i) ust.push_back(ueq[i]);
    for (int i = 0; i <= p; ++i) ust.push_back(m.hi);
    // stabilised sampling matrix B[i][m] = b_i(t_m) at nst equispaced points
    std::vector<double> tpt(m.nst), B(size_t(m.nst) * m.nst);
    for (int q = 0; q < m.nst; ++q) tpt[q] = q == m.nst - 1 ? m.hi : m.lo + (m.hi - m.lo) * q / double(m.nst - 1);
    for (int q = 0; q < m.nst; ++q) {
        const std::vector<double> v = all_splines(ust, p, tpt[q]);
        for (int i = 0; i < m.nst; ++i) B[size_t(i) * m.nst + q] = v[i];
    }
    const std::vector<double> Bi = invert(B, m.nst);
    // C: stabilised spline j in the equidistant splines (insert the removed knots)
    std::vector<double> removed;
    for (int i = p + 1; i < p + 1 + r; ++i) removed.push_back(ueq[i]);
    for (int i = m.n - r; i < m.n; ++i) removed.push_back(ueq[i]);
    std::vector<double> Cm(size_t(m.nst) * m.n);
    for (int j = 0; j < m.nst; ++j) {
        std::vector<double> u = ust, w(size_t(m.nst), 0.0);
        w[j] = 1.0;
        for (double ub : removed) insert_one(u, p, w, ub);
        for (int i = 0; i < m.n; ++i) Cm[size_t(j) * m.n + i] = w[i];
    }
    m.A.assign(size_t(m.nst) * m.n, 0.0);
    for (int k = 0; k < m.nst; ++k)
        for (int i = 0; i < m.n; ++i) {
            double v = 0.0;
            for (int j = 0; j < m.nst; ++j) v += Bi[size_t(k) * m.nst + j] * Cm[size_t(j) * m.n + i];
            m.A[size_t(k) * m.n + i] = v;
        }
    return m;
}

template <typename T>
T *dalloc(size_t n)
{
    void *p = nullptr;
    BIE_HIP(hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)));
    return static_cast<T *>(p);
}

}  // namespace

struct bie_far {
    const bie_op *op = nullptr;
    BsConst c{};
    int s = 0, sb = 0, r = 0, shift = 0, q[3] = { 0, 0, 0 };
    double origin[3] = { 0, 0, 0 }, prot = 0.0;
    int64_t nbox = 0, npairs = 0, nitems = 0;
    std::vector<int32_t> h_box_ijk, h_box_of;
    double *mt = nullptr, *box_lo = nullptr, *qw = nullptr;
    int32_t *box_of = nullptr, *box_ijk = nullptr, *mem_ptr = nullptr, *mem = nullptr, *far = nullptr,
            *item_ptr = nullptr;
    int4 *items = nullptr;
    double2 *tab = nullptr, *agg = nullptr, *lpart = nullptr;
    double *knots = nullptr, *A = nullptr;
    int64_t cap_R = 0;
    ~bie_far()
    {
        for (void *p : { (void *)knots, (void *)A, (void *)mt, (void *)box_lo, (void *)qw, (void *)box_of, (void *)box_ijk, (void *)mem_ptr,
                         (void *)mem, (void *)far, (void *)item_ptr, (void *)items, (void *)tab, (void *)agg,
                         (void *)lpart })
            if (p) (void)hipFree(p);
    }
};

namespace bie {

bie_far *far_create(const bie_op *op, double a, int s, int p, hipStream_t st)
{
    if (op->star) throw Error(BIE_EINVAL, "the far field takes an assembled operator");
    if (!(a > 0.0) || !std::isfinite(a)) throw Error(BIE_EINVAL, "box side must be positive");
    if (p != 1 && p != 3 && p != 5) throw Error(BIE_EINVAL, "degree must be 1, 3 or 5");
    const int r = (p - 1) / 2;   // knots removed per side (stabilisation)
    if (s < p + 1 + 2 * r) throw Error(BIE_EINVAL, "too few splines for the degree");
    const Mesh &M = op->mesh;
    const int64_t N = M.N;
    auto f = std::make_unique<bie_far>();
    f->op = op;
    f->s = s;
    f->r = r;
    // boxes and protrusion
    for (int d = 0; d < 3; ++d) {
        double mn = M.V[d];
        for (int64_t v = 1; v < M.nv; ++v) mn = std::min(mn, M.V[3 * v + d]);
        f->origin[d] = mn - 1e-9 * a;
    }
    std::vector<int32_t> ijk(3 * N);
    double prot = 0.0;
    for (int64_t m = 0; m < N; ++m) {
        const int32_t tp = M.edges[4 * m + 2], tm = M.edges[4 * m + 3];
        for (int d = 0; d < 3; ++d) {
            const double c = 0.5 * (M.cent[3 * tp + d] + M.cent[3 * tm + d]);
            ijk[3 * m + d] = int32_t(std::floor((c - f->origin[d]) / a));
        }
        for (int32_t t : { tp, tm })
            for (int v = 0; v < 3; ++v)
                for (int d = 0; d < 3; ++d) {
                    const double x = M.V[3 * M.T[3 * t + v] + d];
                    const double lo = f->origin[d] + a * ijk[3 * m + d];
                    prot = std::max(prot, std::max((lo - x) / a, (x - lo - a) / a));
                }
    }
    f->prot = prot;
    const int sb = prot > 0.0 ? int(std::ceil(prot * (s - p) - 1e-12)) : 0;
    if (2 * sb >= s - p) throw Error(BIE_EINVAL, "buffer knots reach half a box: use larger boxes or more splines");
    f->sb = sb;
    // splines (parameter coordinates, box = [0, 1])
    const double du = 1.0 / double(s - p);
    BsConst &c = f->c;
    const SplineMap sm = spline_map(s, p, sb, r);
    c.p = p;
    c.a = a;
    c.n = sm.n;
    c.lo = sm.lo;
    c.hi = sm.hi;
    c.nst = sm.nst;
    c.npts = c.nst * c.nst * c.nst;
    if (c.n > MAXN || c.npts > 256 * UPT) throw Error(BIE_EINVAL, "too many splines per box");
    const std::vector<double> &ueq = sm.ueq;
    const std::vector<double> &hA = sm.A;
    // interpolation points on the knot lattice: point m of box I at lattice
    // coordinate shift I + m - sb, shift = s - p
    f->shift = s - p;
    // boxes, members, far lists
    std::map<std::array<int32_t, 3>, int32_t> index;
    for (int64_t m = 0; m < N; ++m) index.emplace(std::array<int32_t, 3>{ ijk[3 * m], ijk[3 * m + 1], ijk[3 * m + 2] }, 0);
    int32_t nb = 0;
    for (auto &kv : index) {
        kv.second = nb++;
        f->h_box_ijk.insert(f->h_box_ijk.end(), kv.first.begin(), kv.first.end());
    }
    f->nbox = nb;
    f->h_box_of.resize(N);
    std::vector<int32_t> cnt(nb + 1, 0);
    for (int64_t m = 0; m < N; ++m) {
        f->h_box_of[m] = index[{ ijk[3 * m], ijk[3 * m + 1], ijk[3 * m + 2] }];
        ++cnt[f->h_box_of[m] + 1];
    }
    for (int b = 0; b < nb; ++b) cnt[b + 1] += cnt[b];
    std::vector<int32_t> mem(N), fill(cnt.begin(), cnt.end() - 1);
    for (int64_t m = 0; m < N; ++m) mem[fill[f->h_box_of[m]]++] = int32_t(m);
    std::vector<int32_t> far, iptr(1, 0);
    std::vector<int4> items;
    int span[3] = { 0, 0, 0 };
    for (int32_t X = 0; X < nb; ++X) {
        const int32_t f0 = int32_t(far.size());
        for (int32_t Y = 0; Y < nb; ++Y) {
            int dmax = 0;
            for (int d = 0; d < 3; ++d) {
                const int dd = std::abs(f->h_box_ijk[3 * X + d] - f->h_box_ijk[3 * Y + d]);
                dmax = std::max(dmax, dd);
                span[d] = std::max(span[d], dd);
            }
            if (dmax > 1) far.push_back(Y);
        }
        const int32_t f1 = int32_t(far.size());
        for (int32_t g = f0; g < f1; g += FAR_CHUNK) items.push_back(make_int4(X, g, std::min(f1, g + FAR_CHUNK), 0));
        iptr.push_back(int32_t(items.size()));
    }
    f->npairs = int64_t(far.size());
    f->nitems = int64_t(items.size());
    for (int d = 0; d < 3; ++d) f->q[d] = f->shift * span[d] + c.nst - 1;
    // device tables
    std::vector<double> blo(3 * size_t(nb));
    for (int32_t b = 0; b < nb; ++b)
        for (int d = 0; d < 3; ++d) blo[3 * b + d] = f->origin[d] + a * f->h_box_ijk[3 * b + d];
    double qwh[QPTS];
    quad_weights(qwh);
    f->knots = dalloc<double>(ueq.size());
    f->A = dalloc<double>(hA.size());
    BIE_HIP(hipMemcpy(f->knots, ueq.data(), ueq.size() * sizeof(double), hipMemcpyHostToDevice));
    BIE_HIP(hipMemcpy(f->A, hA.data(), hA.size() * sizeof(double), hipMemcpyHostToDevice));
    c.knots = f->knots;
    c.A = f->A;
    f->box_lo = dalloc<double>(blo.size());
    f->qw = dalloc<double>(QPTS);
    f->box_of = dalloc<int32_t>(N);
    f->box_ijk = dalloc<int32_t>(f->h_box_ijk.size());
    f->mem_ptr = dalloc<int32_t>(cnt.size());
    f->mem = dalloc<int32_t>(N);
    f->far = dalloc<int32_t>(far.size());
    f->item_ptr = dalloc<int32_t>(iptr.size());
    f->items = dalloc<int4>(items.size());
    BIE_HIP(hipMemcpy(f->box_lo, blo.data(), blo.size() * sizeof(double), hipMemcpyHostToDevice));
    BIE_HIP(hipMemcpy(f->qw, qwh, sizeof(qwh), hipMemcpyHostToDevice));
    BIE_HIP(hipMemcpy(f->box_of, f->h_box_of.data(), N * sizeof(int32_t), hipMemcpyHostToDevice));
    BIE_HIP(hipMemcpy(f->box_ijk, f->h_box_ijk.data(), f->h_box_ijk.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    BIE_HIP(hipMemcpy(f->mem_ptr, cnt.data(), cnt.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    BIE_HIP(hipMemcpy(f->mem, mem.data(), N * sizeof(int32_t), hipMemcpyHostToDevice));
    if (!far.empty()) BIE_HIP(hipMemcpy(f->far, far.data(), far.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    BIE_HIP(hipMemcpy(f->item_ptr, iptr.data(), iptr.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    if (!items.empty()) BIE_HIP(hipMemcpy(f->items, items.data(), items.size() * sizeof(int4), hipMemcpyHostToDevice));
    // moments and the lattice table of g
    f->mt = dalloc<double>(size_t(N) * 4 * c.npts);
    const TriDev &D = op->tri;
    hipLaunchKernelGGL(k_bs_moments, dim3(unsigned(N)), dim3(256), 0, st, c, N, (const int4 *)D.edges, D.cent, D.loc,
                       D.vfree, f->qw, f->box_lo, f->box_of, f->mt);
    BIE_HIP(hipGetLastError());
    const int64_t ntab = int64_t(2 * f->q[0] + 1) * (2 * f->q[1] + 1) * (2 * f->q[2] + 1);
    f->tab = dalloc<double2>(size_t(ntab));
    hipLaunchKernelGGL(k_bs_gtable, dim3(unsigned(std::min<int64_t>((ntab + 255) / 256, 4096))), dim3(256), 0, st,
                       f->q[0], f->q[1], f->q[2], a * du, op->k, f->tab);
    BIE_HIP(hipGetLastError());
    BIE_HIP(hipStreamSynchronize(st));
    return f.release();
}

void far_apply(bie_far *f, const void *X, void *Y, int64_t R, hipStream_t st)
{
    const BsConst &c = f->c;
    const int64_t N = f->op->mesh.N;
    if (f->cap_R < R) {
        BIE_HIP(hipStreamSynchronize(st));
        for (double2 **p : { &f->agg, &f->lpart })
            if (*p) {
                (void)hipFree(*p);
                *p = nullptr;
            }
        f->cap_R = 0;
        f->agg = dalloc<double2>(size_t(R) * f->nbox * 4 * c.npts);
        f->lpart = dalloc<double2>(size_t(R) * std::max<int64_t>(1, f->nitems) * 4 * c.npts);
        f->cap_R = R;
    }
    hipLaunchKernelGGL(k_bs_aggregate, dim3(unsigned(f->nbox), unsigned(R)), dim3(256), 0, st, c.npts, N, f->nbox,
                       f->mem_ptr, f->mem, f->mt, (const double2 *)X, f->agg);
    if (f->nitems)
        hipLaunchKernelGGL(k_bs_translate, dim3(unsigned(f->nitems), unsigned(R)), dim3(256),
                           size_t(4) * c.npts * sizeof(double2), st, c.nst, c.npts, f->shift, f->q[0], f->q[1], f->q[2],
                           f->nbox, f->nitems, f->items, f->far, f->box_ijk, f->tab, f->agg, f->lpart);
    hipLaunchKernelGGL(k_bs_disaggregate, dim3(unsigned(N), unsigned(R)), dim3(256), 0, st, c.npts, N, f->nitems,
                       f->op->k, f->box_of, f->item_ptr, f->mt, f->lpart, (double2 *)Y);
    BIE_HIP(hipGetLastError());
}

void far_info(const bie_far *f, bie_far_info *info)
{
    info->boxes = f->nbox;
    info->far_pairs = f->npairs;
    info->buffer_knots = f->sb;
    info->splines = f->c.n;
    info->points_per_axis = f->c.nst;
    info->protrusion = f->prot;
    for (int d = 0; d < 3; ++d) info->origin[d] = f->origin[d];
}

void far_boxes(const bie_far *f, int32_t *out)
{
    for (size_t m = 0; m < f->h_box_of.size(); ++m)
        for (int d = 0; d < 3; ++d) out[3 * m + d] = f->h_box_ijk[3 * size_t(f->h_box_of[m]) + d];
}

void far_destroy(bie_far *f) { delete f; }

}  // namespace bie

// ============================================================================
// Multilevel far field (Sec. IV).  A regular octree over the leaf boxes of
// side a (level 0); the box of level l holding leaf box (i, j, k) is
// (i, j, k) >> l.  Every level carries its own spline space: the parent of a
// level keeps s and takes ceil(sb / 2) buffer knots while its boxes are smaller
// than half a wavelength (Sec. IV-C), and takes 2 s - p splines and the same
// sb otherwise (Sec. IV-D); the knot vectors of a box and of its parent are
// nested, so the parent's equidistant splines restricted to a child's buffered
// interval are exact combinations of the child's (knot insertion, Sec. IV-B):
// the 1D transfer matrices C_0, C_1 (child in the lower / upper half of the
// parent) and their tensor products.
//
// Product y = Z~_far x, Z~_far covering the pairs of far leaf boxes:
//   leaf moments     M_0[X] = sum_{m in X} x_m m_eq[m]  (equidistant splines),
//   upward           M_l[P] = sum_{children X} (C_x (x) C_y (x) C_z) M_l-1[X],
//   transform        M~_l = (A (x) A (x) A) M_l,  A = B_stab^-1 C_stab,
//   translation      Z~_l[X] = w_d sum_{Y in IL_l(X)} G_XY M~_l[Y] by FFT: G_XY
//                    is three-level Toeplitz (Sec. III-C), its symbol K_o one
//                    array per box offset o, so Z^_X = sum_Y K^_o . M^_Y per
//                    frequency (linear convolution in L^3 >= (2 nst - 1)^3),
//   back             L_l[X] = (A^T)^(x)3 Z~_l[X] + (C^T)^(x)3 L_l+1[parent X],
//   test functions   y_m = sum_d m_eq[m][d] . L_0[box m][d].
// IL_l(X): boxes Y with Chebyshev index distance > 1 whose parents are within
// distance 1 (at the top level every far box); w = jk for the three vector
// parts, 1/(jk) for the divergence part.
// ============================================================================
namespace {

constexpr int MLT = 18;                                    // most equidistant splines per axis, any level
constexpr int MLQ = (MLT * MLT * MLT + 255) / 256;         // output entries per thread of k_ml_tensor

// out[ob] (=, or += if acc) sum_{t in ptr[ob] .. ptr[ob+1])
//     (P_bx (x) P_by (x) P_bz) in[box[t]],  P_0 = m0, P_1 = m1 (nout x nin),
// b = the child bits of entry t (x: 4, y: 2, z: 1; none if bits is null);
// per box 4 complex components of nin^3 (nout^3) entries; block (ob, 2 d + part).
__global__ __launch_bounds__(256) void k_ml_tensor(int nin, int nout, const double *__restrict__ m0,
                                                   const double *__restrict__ m1, const int32_t *__restrict__ ptr,
                                                   const int32_t *__restrict__ box, const int32_t *__restrict__ bits,
                                                   const double *__restrict__ in, double *__restrict__ out, int acc)
{
    __shared__ double b0[MLT * MLT * MLT], b1[MLT * MLT * MLT], b2[MLT * MLT * MLT];
    const int64_t ob = blockIdx.x;
    const int d = blockIdx.y >> 1, part = blockIdx.y & 1;
    const int tid = threadIdx.x;
    const int nin2 = nin * nin, nin3 = nin2 * nin, nout3 = nout * nout * nout;
    double a[MLQ];
#pragma unroll
    for (int q = 0; q < MLQ; ++q) a[q] = 0.0;
    for (int32_t t = ptr[ob]; t < ptr[ob + 1]; ++t) {
        const int32_t ib = box[t];
        const int bt = bits ? bits[t] : 0;
        const double *Px = (bt & 4) ? m1 : m0, *Py = (bt & 2) ? m1 : m0, *Pz = (bt & 1) ? m1 : m0;
        __syncthreads();
        const double *src = in + 2 * ((int64_t(ib) * 4 + d) * nin3) + part;
        for (int e = tid; e < nin3; e += 256) b0[e] = src[2 * int64_t(e)];
        __syncthreads();
        for (int e = tid; e < nout * nin2; e += 256) {   // along x
            const int i = e / nin2, rr = e % nin2;
            double v = 0.0;
            for (int q = 0; q < nin; ++q) v += Px[i * nin + q] * b0[q * nin2 + rr];
            b1[e] = v;
        }
        __syncthreads();
        for (int e = tid; e < nout * nout * nin; e += 256) {   // along y
            const int i = e / (nout * nin), j = (e / nin) % nout, z = e % nin;
            double v = 0.0;
            for (int q = 0; q < nin; ++q) v += Py[j * nin + q] * b1[(i * nin + q) * nin + z];
            b2[e] = v;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < MLQ; ++q) {   // along z
            const int e = tid + 256 * q;
            if (e >= nout3) break;
            const int ij = e / nout, k = e % nout;
            double v = 0.0;
            for (int z = 0; z < nin; ++z) v += Pz[k * nin + z] * b2[ij * nin + z];
            a[q] += v;
        }
    }
    double *dst = out + 2 * ((ob * 4 + d) * nout3) + part;
#pragma unroll
    for (int q = 0; q < MLQ; ++q) {
        const int e = tid + 256 * q;
        if (e >= nout3) break;
        dst[2 * int64_t(e)] = acc ? dst[2 * int64_t(e)] + a[q] : a[q];
    }
}

// F[vol] = Mt[vol] (nst^3) zero-padded to L^3.
__global__ __launch_bounds__(256) void k_ml_pad(int nst, int L, int64_t nvol, const double2 *__restrict__ Mt,
                                                double2 *__restrict__ F)
{
    const int64_t L3 = int64_t(L) * L * L, total = nvol * L3;
    for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < total; e += int64_t(gridDim.x) * 256) {
        const int64_t v = e / L3;
        const int r = int(e % L3), i = r / (L * L), j = (r / L) % L, k = r % L;
        F[e] = (i < nst && j < nst && k < nst) ? Mt[v * nst * nst * nst + (i * nst + j) * nst + k]
                                               : make_double2(0.0, 0.0);
    }
}

// Zt[vol][i] = w_d F[vol][i] / L^3 for i in [0, nst)^3 (d = vol % 4).
__global__ __launch_bounds__(256) void k_ml_crop(int nst, int L, int64_t nvol, double k,
                                                 const double2 *__restrict__ F, double2 *__restrict__ Zt)
{
    const int64_t n3 = int64_t(nst) * nst * nst, total = nvol * n3;
    const double sc = 1.0 / (double(L) * L * L);
    for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < total; e += int64_t(gridDim.x) * 256) {
        const int64_t v = e / n3;
        const int r = int(e % n3), i = r / (nst * nst), j = (r / nst) % nst, q = r % nst;
        const double2 f = F[v * L * L * L + (i * L + j) * L + q];
        const double fr = f.x * sc, fi = f.y * sc;
        // jk (a + jb) = -k b + j k a;  (a + jb) / (jk) = b / k - j a / k
        Zt[e] = (v % 4) < 3 ? make_double2(-k * fi, k * fr) : make_double2(fi / k, -fr / k);
    }
}

// In-place 1D FFTs of length L along one axis of nvol L^3 volumes (z fastest),
// one line per thread: radix 2, input in bit-reversed order, twiddles
// tw[j] = exp(-2 pi i j / L) (conjugated for the inverse, unscaled).
template <int L>
__global__ __launch_bounds__(256) void k_ml_fft(double2 *__restrict__ data, int64_t nvol, int axis, int inverse,
                                                const double2 *__restrict__ tw)
{
    const int64_t line = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (line >= nvol * L * L) return;
    const int64_t vol = line / (L * L);
    const int q = int(line % (L * L));
    int64_t base, stride;
    if (axis == 0) {
        base = vol * L * L * L + q;
        stride = L * L;
    } else if (axis == 1) {
        base = vol * L * L * L + int64_t(q / L) * L * L + q % L;
        stride = L;
    } else {
        base = vol * L * L * L + int64_t(q) * L;
        stride = 1;
    }
    constexpr int LB = L == 16 ? 4 : 5;
    double2 v[L];
#pragma unroll
    for (int i = 0; i < L; ++i) {
        int r = 0;
#pragma unroll
        for (int b = 0; b < LB; ++b) r |= ((i >> b) & 1) << (LB - 1 - b);
        v[r] = data[base + i * stride];
    }
    const double sg = inverse ? -1.0 : 1.0;
#pragma unroll
    for (int len = 2; len <= L; len <<= 1) {
        const int half = len / 2;
#pragma unroll
        for (int s0 = 0; s0 < L; s0 += len)
#pragma unroll
            for (int j = 0; j < half; ++j) {
                const double2 w = tw[j * (L / len)];
                const double wr = w.x, wi = sg * w.y;
                const double2 u = v[s0 + j], t0 = v[s0 + j + half];
                const double tr = wr * t0.x - wi * t0.y, ti = wr * t0.y + wi * t0.x;
                v[s0 + j] = make_double2(u.x + tr, u.y + ti);
                v[s0 + j + half] = make_double2(u.x - tr, u.y - ti);
            }
    }
#pragma unroll
    for (int i = 0; i < L; ++i) data[base + i * stride] = v[i];
}

// Fz[X][d][f] = sum_{t in ptr[X] .. ptr[X+1]) Kh[off[t]][f] F[src[t]][d][f]
__global__ __launch_bounds__(256) void k_ml_accum(int64_t L3, const int32_t *__restrict__ ptr,
                                                  const int32_t *__restrict__ src, const int32_t *__restrict__ off,
                                                  const double2 *__restrict__ Kh, const double2 *__restrict__ F,
                                                  double2 *__restrict__ Fz)
{
    const int64_t X = blockIdx.x;
    const int64_t f = int64_t(blockIdx.y) * 256 + threadIdx.x;
    if (f >= L3) return;
    double2 a[4] = { { 0, 0 }, { 0, 0 }, { 0, 0 }, { 0, 0 } };
    for (int32_t t = ptr[X]; t < ptr[X + 1]; ++t) {
        const double2 kk = Kh[int64_t(off[t]) * L3 + f];
        const double2 *m = F + int64_t(src[t]) * 4 * L3 + f;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const double2 v = m[d * L3];
            a[d].x += kk.x * v.x - kk.y * v.y;
            a[d].y += kk.x * v.y + kk.y * v.x;
        }
    }
#pragma unroll
    for (int d = 0; d < 4; ++d) Fz[(X * 4 + d) * L3 + f] = a[d];
}

// K_o on the circular grid: entry (i, j, k) holds g(h |o + (di, dj, dk)|) with
// di = i (i < nst) or i - L (i > L - nst), else 0.
__global__ __launch_bounds__(256) void k_ml_ktab(int L, int nst, int64_t noff, const int32_t *__restrict__ offs,
                                                 double h, double k, double2 *__restrict__ K)
{
    const int64_t L3 = int64_t(L) * L * L, total = noff * L3;
    for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < total; e += int64_t(gridDim.x) * 256) {
        const int64_t o = e / L3;
        const int r = int(e % L3), idx[3] = { r / (L * L), (r / L) % L, r % L };
        double2 val = make_double2(0.0, 0.0);
        bool ok = true;
        double dd[3];
        for (int a = 0; a < 3; ++a) {
            const int i = idx[a];
            const int di = i < nst ? i : (i > L - nst ? i - L : 0);
            ok = ok && (i < nst || i > L - nst);
            dd[a] = double(offs[3 * o + a] + di);
        }
        if (ok) {
            const double R = h * sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
            double sn, cs;
            sincos(k * R, &sn, &cs);
            const double g = 1.0 / (4.0 * M_PI * R);
            val = make_double2(g * cs, -g * sn);
        }
        K[e] = val;
    }
}

// y_m = sum_d sum_e m_eq[m][d][e] L_0[box m][d][e]
__global__ __launch_bounds__(256) void k_ml_disaggregate(int n3, int64_t N, const int32_t *__restrict__ box_of,
                                                         const double *__restrict__ meq, const double2 *__restrict__ Lq,
                                                         double2 *__restrict__ Y)
{
    const int64_t m = blockIdx.x;
    const double *mm = meq + m * 4 * int64_t(n3);
    const double2 *l = Lq + int64_t(box_of[m]) * 4 * n3;
    double sr = 0.0, si = 0.0;
    for (int e = threadIdx.x; e < 4 * n3; e += 256) {
        const double v = mm[e];
        const double2 w = l[e];
        sr += v * w.x;
        si += v * w.y;
    }
    __shared__ double red[2][256];
    red[0][threadIdx.x] = sr;
    red[1][threadIdx.x] = si;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (int(threadIdx.x) < o) {
            red[0][threadIdx.x] += red[0][threadIdx.x + o];
            red[1][threadIdx.x] += red[1][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) Y[m] = make_double2(red[0][0], red[1][0]);
}

// Restriction of the parent's splines (knots u_par) to the child's interval
// [u_ch.front(), u_ch.back()] in the child's splines: the knots of u_ch that
// u_par lacks, the ends up to multiplicity p + 1, inserted into the unit
// curve of parent spline j; row j = the coefficients of the refined splines on
// the interval (n_par x n_ch, row-major).
std::vector<double> restrict_splines(const std::vector<double> &u_par, int p, const std::vector<double> &u_ch)
{
    const double tol = 1e-12;
    const double a = u_ch.front(), b = u_ch.back();
    std::vector<double> pool, extra;
    for (double v : u_par)
        if (v > a - tol && v < b + tol) pool.push_back(v);
    for (double v : u_ch) {
        bool found = false;
        for (size_t t = 0; t < pool.size(); ++t)
            if (std::fabs(pool[t] - v) <= tol) {
                pool.erase(pool.begin() + t);
                found = true;
                break;
            }
        if (!found) extra.push_back(v);
    }
    for (double v : pool)
        if (v > a + tol && v < b - tol) throw bie::Error(BIE_EINVAL, "level knot vectors are not nested");
    std::sort(extra.begin(), extra.end());
    const int np = int(u_par.size()) - p - 1, nc = int(u_ch.size()) - p - 1;
    std::vector<double> C(size_t(np) * nc, 0.0);
    for (int j = 0; j < np; ++j) {
        std::vector<double> u = u_par, w(size_t(np), 0.0);
        w[j] = 1.0;
        for (double e : extra) insert_one(u, p, w, e);
        int k0 = -1;
        for (int i = 0; i < int(u.size()); ++i)
            if (std::fabs(u[i] - a) <= tol) {
                k0 = i;
                break;
            }
        if (k0 < 0 || k0 + nc > int(w.size())) throw bie::Error(BIE_EINVAL, "level knot vectors are not nested");
        for (int i = 0; i < nc; ++i) C[size_t(j) * nc + i] = w[k0 + i];
    }
    return C;
}

template <typename T>
T *upload(const std::vector<T> &v)
{
    T *d = dalloc<T>(v.size());
    if (!v.empty()) BIE_HIP(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return d;
}

std::vector<double> transpose(const std::vector<double> &M, int rows, int cols)
{
    std::vector<double> T(M.size());
    for (int i = 0; i < rows; ++i)
        for (int j = 0; j < cols; ++j) T[size_t(j) * rows + i] = M[size_t(i) * cols + j];
    return T;
}

struct MlLevel {
    int s = 0, sb = 0, n = 0, nst = 0, L = 0;
    double a = 0.0, h = 0.0;
    int64_t nbox = 0, npairs = 0, noff = 0;
    std::vector<int32_t> h_ijk;
    double *A = nullptr, *AT = nullptr, *C[2] = { nullptr, nullptr }, *CT[2] = { nullptr, nullptr };
    int32_t *self_ptr = nullptr, *self_box = nullptr;
    int32_t *kid_ptr = nullptr, *kid_box = nullptr, *kid_bits = nullptr;    // children on the level below
    int32_t *par_ptr = nullptr, *par_box = nullptr, *par_bits = nullptr;    // parent on the level above
    int32_t *il_ptr = nullptr, *il_src = nullptr, *il_off = nullptr;
    double2 *Kh = nullptr, *tw = nullptr;
    double2 *M = nullptr, *Mt = nullptr, *F = nullptr, *Fz = nullptr, *Lq = nullptr;
    void free_all()
    {
        for (void *p : { (void *)A, (void *)AT, (void *)C[0], (void *)C[1], (void *)CT[0], (void *)CT[1],
                         (void *)self_ptr, (void *)self_box, (void *)kid_ptr, (void *)kid_box, (void *)kid_bits,
                         (void *)par_ptr, (void *)par_box, (void *)par_bits, (void *)il_ptr, (void *)il_src,
                         (void *)il_off, (void *)Kh, (void *)tw, (void *)M, (void *)Mt, (void *)F, (void *)Fz,
                         (void *)Lq })
            if (p) (void)hipFree(p);
    }
};

void fft3(const MlLevel &lv, double2 *data, int64_t nvol, bool inverse, hipStream_t st)
{
    const int64_t lines = nvol * lv.L * lv.L;
    const dim3 grid(unsigned((lines + 255) / 256));
    for (int axis = 0; axis < 3; ++axis) {
        if (lv.L == 16)
            hipLaunchKernelGGL(k_ml_fft<16>, grid, dim3(256), 0, st, data, nvol, axis, int(inverse), (const double2 *)lv.tw);
        else
            hipLaunchKernelGGL(k_ml_fft<32>, grid, dim3(256), 0, st, data, nvol, axis, int(inverse), (const double2 *)lv.tw);
    }
    BIE_HIP(hipGetLastError());
}

void tensor(int nin, int nout, const double *m0, const double *m1, const int32_t *ptr, const int32_t *box,
            const int32_t *bits, const double2 *in, double2 *out, int64_t nout_boxes, bool acc, hipStream_t st)
{
    if (nout_boxes == 0) return;
    hipLaunchKernelGGL(k_ml_tensor, dim3(unsigned(nout_boxes), 8), dim3(256), 0, st, nin, nout, m0, m1, ptr, box, bits,
                       (const double *)in, (double *)out, int(acc));
    BIE_HIP(hipGetLastError());
}

}  // namespace

struct bie_farml {
    const bie_op *op = nullptr;
    int p = 0, levels = 0;
    double origin[3] = { 0, 0, 0 }, prot = 0.0;
    std::vector<MlLevel> lv;
    std::vector<int32_t> h_box_of;
    BsConst c0{};                   // leaf moments with the equidistant splines (A = identity)
    double *meq = nullptr, *knots = nullptr, *ident = nullptr, *box_lo = nullptr, *qw = nullptr;
    int32_t *box_of = nullptr, *mem_ptr = nullptr, *mem = nullptr;
    ~bie_farml()
    {
        for (auto &l : lv) l.free_all();
        for (void *q : { (void *)meq, (void *)knots, (void *)ident, (void *)box_lo, (void *)qw, (void *)box_of,
                         (void *)mem_ptr, (void *)mem })
            if (q) (void)hipFree(q);
    }
};

namespace bie {

bie_farml *farml_create(const bie_op *op, double a, int levels, int s, int p, hipStream_t st)
{
    if (op->star) throw Error(BIE_EINVAL, "the far field takes an assembled operator");
    if (!(a > 0.0) || !std::isfinite(a)) throw Error(BIE_EINVAL, "box side must be positive");
    if (p != 1 && p != 3 && p != 5) throw Error(BIE_EINVAL, "degree must be 1, 3 or 5");
    if (levels < 1 || levels > 12) throw Error(BIE_EINVAL, "levels must be 1..12");
    const int r = (p - 1) / 2;
    if (s < p + 1 + 2 * r) throw Error(BIE_EINVAL, "too few splines for the degree");
    const Mesh &Ms = op->mesh;
    const int64_t N = Ms.N;
    auto f = std::make_unique<bie_farml>();
    f->op = op;
    f->p = p;
    f->levels = levels;
    for (int d = 0; d < 3; ++d) {
        double mn = Ms.V[d];
        for (int64_t v = 1; v < Ms.nv; ++v) mn = std::min(mn, Ms.V[3 * v + d]);
        f->origin[d] = mn - 1e-9 * a;
    }
    // leaf boxes and protrusion (as the single-level far field)
    std::vector<int32_t> ijk(3 * N);
    double prot = 0.0;
    for (int64_t m = 0; m < N; ++m) {
        const int32_t tp = Ms.edges[4 * m + 2], tm = Ms.edges[4 * m + 3];
        for (int d = 0; d < 3; ++d) {
            const double cc = 0.5 * (Ms.cent[3 * tp + d] + Ms.cent[3 * tm + d]);
            ijk[3 * m + d] = int32_t(std::floor((cc - f->origin[d]) / a));
        }
        for (int32_t t : { tp, tm })
            for (int v = 0; v < 3; ++v)
                for (int d = 0; d < 3; ++d) {
                    const double x = Ms.V[3 * Ms.T[3 * t + v] + d];
                    const double lo = f->origin[d] + a * ijk[3 * m + d];
                    prot = std::max(prot, std::max((lo - x) / a, (x - lo - a) / a));
                }
    }
    f->prot = prot;
    // spline spaces per level
    const double lam = 2.0 * M_PI / op->k;
    std::vector<SplineMap> maps;
    f->lv.resize(levels);
    for (int l = 0; l < levels; ++l) {
        MlLevel &L = f->lv[l];
        L.a = a * double(1 << l);
        if (l == 0) {
            L.s = s;
            L.sb = prot > 0.0 ? int(std::ceil(prot * (s - p) - 1e-12)) : 0;
        } else if (L.a < 0.5 * lam) {
            L.s = f->lv[l - 1].s;
            L.sb = (f->lv[l - 1].sb + 1) / 2;
        } else {
            L.s = 2 * f->lv[l - 1].s - p;
            L.sb = f->lv[l - 1].sb;
        }
        if (2 * L.sb >= L.s - p) throw Error(BIE_EINVAL, "buffer knots reach half a box: use larger boxes or more splines");
        maps.push_back(spline_map(L.s, p, L.sb, r));
        L.n = maps.back().n;
        L.nst = maps.back().nst;
        if (L.n > MLT) throw Error(BIE_EINVAL, "too many splines per box on level " + std::to_string(l));
        L.L = 2 * L.nst - 1 <= 16 ? 16 : (2 * L.nst - 1 <= 32 ? 32 : 0);
        if (!L.L) throw Error(BIE_EINVAL, "too many interpolation points per box on level " + std::to_string(l));
        L.h = L.a / double(L.s - p);   // odd p: the points lie on the knots
    }
    // boxes per level
    std::vector<std::map<std::array<int32_t, 3>, int32_t>> index(levels);
    for (int64_t m = 0; m < N; ++m)
        for (int l = 0; l < levels; ++l)
            index[l].emplace(std::array<int32_t, 3>{ ijk[3 * m] >> l, ijk[3 * m + 1] >> l, ijk[3 * m + 2] >> l }, 0);
    for (int l = 0; l < levels; ++l) {
        int32_t nb = 0;
        for (auto &kv : index[l]) {
            kv.second = nb++;
            f->lv[l].h_ijk.insert(f->lv[l].h_ijk.end(), kv.first.begin(), kv.first.end());
        }
        f->lv[l].nbox = nb;
    }
    f->h_box_of.resize(N);
    for (int64_t m = 0; m < N; ++m) f->h_box_of[m] = index[0][{ ijk[3 * m], ijk[3 * m + 1], ijk[3 * m + 2] }];
    auto cheb = [](const int32_t *x, const int32_t *y) {
        return std::max(std::abs(x[0] - y[0]), std::max(std::abs(x[1] - y[1]), std::abs(x[2] - y[2])));
    };
    for (int l = 0; l < levels; ++l) {
        MlLevel &L = f->lv[l];
        const int64_t nb = L.nbox;
        const int32_t *B = L.h_ijk.data();
        // identity lists
        std::vector<int32_t> sp(nb + 1), sbx(nb);
        for (int32_t b = 0; b <= nb; ++b) sp[b] = b;
        for (int32_t b = 0; b < nb; ++b) sbx[b] = b;
        L.self_ptr = upload(sp);
        L.self_box = upload(sbx);
        // parent of each box (level above) and children of each box (level below)
        if (l + 1 < levels) {
            std::vector<int32_t> pp(nb + 1), pb(nb), pbits(nb);
            for (int32_t b = 0; b < nb; ++b) {
                pp[b] = b;
                pb[b] = index[l + 1][{ B[3 * b] >> 1, B[3 * b + 1] >> 1, B[3 * b + 2] >> 1 }];
                pbits[b] = ((B[3 * b] & 1) << 2) | ((B[3 * b + 1] & 1) << 1) | (B[3 * b + 2] & 1);
            }
            pp[nb] = int32_t(nb);
            L.par_ptr = upload(pp);
            L.par_box = upload(pb);
            L.par_bits = upload(pbits);
        }
        if (l > 0) {
            const MlLevel &Lc = f->lv[l - 1];
            std::vector<std::vector<int32_t>> kids(nb), kbits(nb);
            for (int32_t c = 0; c < Lc.nbox; ++c) {
                const int32_t *q = Lc.h_ijk.data() + 3 * c;
                const int32_t P = index[l][{ q[0] >> 1, q[1] >> 1, q[2] >> 1 }];
                kids[P].push_back(c);
                kbits[P].push_back(((q[0] & 1) << 2) | ((q[1] & 1) << 1) | (q[2] & 1));
            }
            std::vector<int32_t> kp(1, 0), kb, kt;
            for (int32_t b = 0; b < nb; ++b) {
                kb.insert(kb.end(), kids[b].begin(), kids[b].end());
                kt.insert(kt.end(), kbits[b].begin(), kbits[b].end());
                kp.push_back(int32_t(kb.size()));
            }
            L.kid_ptr = upload(kp);
            L.kid_box = upload(kb);
            L.kid_bits = upload(kt);
            // 1D transfers from the child level: parent splines on each half
            const SplineMap &mp = maps[l], &mc = maps[l - 1];
            for (int c = 0; c < 2; ++c) {
                std::vector<double> uch(mc.ueq.size());
                for (size_t i = 0; i < uch.size(); ++i) uch[i] = 0.5 * c + 0.5 * mc.ueq[i];
                const std::vector<double> Cm = restrict_splines(mp.ueq, p, uch);
                L.C[c] = upload(Cm);
                L.CT[c] = upload(transpose(Cm, mp.n, mc.n));
            }
        }
        L.A = upload(maps[l].A);
        L.AT = upload(transpose(maps[l].A, L.nst, L.n));
        // interaction list by target, box offsets
        std::map<std::array<int32_t, 3>, int32_t> offs;
        std::vector<int32_t> ip(1, 0), isrc, ioff, hoffs;
        for (int32_t X = 0; X < nb; ++X) {
            for (int32_t Y = 0; Y < nb; ++Y) {
                if (cheb(B + 3 * X, B + 3 * Y) <= 1) continue;
                if (l + 1 < levels) {
                    const int32_t px[3] = { B[3 * X] >> 1, B[3 * X + 1] >> 1, B[3 * X + 2] >> 1 };
                    const int32_t py[3] = { B[3 * Y] >> 1, B[3 * Y + 1] >> 1, B[3 * Y + 2] >> 1 };
                    if (cheb(px, py) > 1) continue;
                }
                const std::array<int32_t, 3> o{ B[3 * X] - B[3 * Y], B[3 * X + 1] - B[3 * Y + 1],
                                                B[3 * X + 2] - B[3 * Y + 2] };
                auto it = offs.find(o);
                if (it == offs.end()) {
                    it = offs.emplace(o, int32_t(offs.size())).first;
                    for (int d = 0; d < 3; ++d) hoffs.push_back(o[d] * (L.s - p));   // in lattice steps
                }
                isrc.push_back(Y);
                ioff.push_back(it->second);
            }
            ip.push_back(int32_t(isrc.size()));
        }
        L.npairs = int64_t(isrc.size());
        L.noff = int64_t(offs.size());
        L.il_ptr = upload(ip);
        L.il_src = upload(isrc);
        L.il_off = upload(ioff);
        // FFT twiddles and the kernel symbols of the offsets
        std::vector<double2> tw(L.L / 2);
        for (int j = 0; j < L.L / 2; ++j) {
            const double ang = -2.0 * M_PI * double(j) / double(L.L);
            tw[j] = make_double2(std::cos(ang), std::sin(ang));
        }
        L.tw = upload(tw);
        const int64_t L3 = int64_t(L.L) * L.L * L.L;
        if (L.noff) {
            int32_t *doffs = upload(hoffs);
            L.Kh = dalloc<double2>(size_t(L.noff * L3));
            hipLaunchKernelGGL(k_ml_ktab, dim3(unsigned(std::min<int64_t>((L.noff * L3 + 255) / 256, 65535))), dim3(256),
                               0, st, L.L, L.nst, L.noff, doffs, L.h, op->k, L.Kh);
            BIE_HIP(hipGetLastError());
            fft3(L, L.Kh, L.noff, false, st);
            BIE_HIP(hipStreamSynchronize(st));
            (void)hipFree(doffs);
        }
        // work arrays (one vector)
        L.M = dalloc<double2>(size_t(nb) * 4 * L.n * L.n * L.n);
        L.Lq = dalloc<double2>(size_t(nb) * 4 * L.n * L.n * L.n);
        L.Mt = dalloc<double2>(size_t(nb) * 4 * L.nst * L.nst * L.nst);
        L.F = dalloc<double2>(size_t(nb) * 4 * L3);
        L.Fz = dalloc<double2>(size_t(nb) * 4 * L3);
    }
    // leaf moments with the equidistant splines (A = identity), members of the leaf boxes
    const MlLevel &L0 = f->lv[0];
    const SplineMap &m0 = maps[0];
    std::vector<double> I(size_t(L0.n) * L0.n, 0.0);
    for (int i = 0; i < L0.n; ++i) I[size_t(i) * L0.n + i] = 1.0;
    f->knots = upload(m0.ueq);
    f->ident = upload(I);
    BsConst &c = f->c0;
    c.p = p;
    c.a = a;
    c.n = L0.n;
    c.nst = L0.n;
    c.npts = L0.n * L0.n * L0.n;
    c.lo = m0.lo;
    c.hi = m0.hi;
    c.knots = f->knots;
    c.A = f->ident;
    std::vector<double> blo(3 * size_t(L0.nbox));
    for (int32_t b = 0; b < L0.nbox; ++b)
        for (int d = 0; d < 3; ++d) blo[3 * b + d] = f->origin[d] + a * L0.h_ijk[3 * b + d];
    std::vector<int32_t> cnt(L0.nbox + 1, 0);
    for (int64_t m = 0; m < N; ++m) ++cnt[f->h_box_of[m] + 1];
    for (int64_t b = 0; b < L0.nbox; ++b) cnt[b + 1] += cnt[b];
    std::vector<int32_t> mem(N), fillp(cnt.begin(), cnt.end() - 1);
    for (int64_t m = 0; m < N; ++m) mem[fillp[f->h_box_of[m]]++] = int32_t(m);
    double qwh[QPTS];
    quad_weights(qwh);
    f->box_lo = upload(blo);
    f->qw = dalloc<double>(QPTS);
    BIE_HIP(hipMemcpy(f->qw, qwh, sizeof(qwh), hipMemcpyHostToDevice));
    f->box_of = upload(f->h_box_of);
    f->mem_ptr = upload(cnt);
    f->mem = upload(mem);
    f->meq = dalloc<double>(size_t(N) * 4 * c.npts);
    const TriDev &D = op->tri;
    hipLaunchKernelGGL(k_bs_moments, dim3(unsigned(N)), dim3(256), 0, st, c, N, (const int4 *)D.edges, D.cent, D.loc,
                       D.vfree, f->qw, f->box_lo, f->box_of, f->meq);
    BIE_HIP(hipGetLastError());
    BIE_HIP(hipStreamSynchronize(st));
    return f.release();
}

void farml_apply(bie_farml *f, const void *X, void *Y, int64_t R, hipStream_t st)
{
    const int64_t N = f->op->mesh.N;
    const int top = f->levels - 1;
    for (int64_t r = 0; r < R; ++r) {
        MlLevel &L0 = f->lv[0];
        hipLaunchKernelGGL(k_bs_aggregate, dim3(unsigned(L0.nbox), 1), dim3(256), 0, st, f->c0.npts, N, L0.nbox,
                           f->mem_ptr, f->mem, f->meq, (const double2 *)X + r * N, L0.M);
        BIE_HIP(hipGetLastError());
        for (int l = 1; l <= top; ++l) {
            MlLevel &L = f->lv[l];
            const MlLevel &Lc = f->lv[l - 1];
            tensor(Lc.n, L.n, L.C[0], L.C[1], L.kid_ptr, L.kid_box, L.kid_bits, Lc.M, L.M, L.nbox, false, st);
        }
        for (int l = 0; l <= top; ++l) {
            MlLevel &L = f->lv[l];
            const int64_t nvol = L.nbox * 4, L3 = int64_t(L.L) * L.L * L.L;
            tensor(L.n, L.nst, L.A, L.A, L.self_ptr, L.self_box, nullptr, L.M, L.Mt, L.nbox, false, st);
            hipLaunchKernelGGL(k_ml_pad, dim3(unsigned(std::min<int64_t>((nvol * L3 + 255) / 256, 65535))), dim3(256), 0,
                               st, L.nst, L.L, nvol, L.Mt, L.F);
            fft3(L, L.F, nvol, false, st);
            hipLaunchKernelGGL(k_ml_accum, dim3(unsigned(L.nbox), unsigned((L3 + 255) / 256)), dim3(256), 0, st, L3,
                               L.il_ptr, L.il_src, L.il_off, (const double2 *)L.Kh, (const double2 *)L.F, L.Fz);
            fft3(L, L.Fz, nvol, true, st);
            const int64_t n3 = int64_t(L.nst) * L.nst * L.nst;
            hipLaunchKernelGGL(k_ml_crop, dim3(unsigned(std::min<int64_t>((nvol * n3 + 255) / 256, 65535))), dim3(256), 0,
                               st, L.nst, L.L, nvol, f->op->k, (const double2 *)L.Fz, L.Mt);
            BIE_HIP(hipGetLastError());
            tensor(L.nst, L.n, L.AT, L.AT, L.self_ptr, L.self_box, nullptr, L.Mt, L.Lq, L.nbox, false, st);
        }
        for (int l = top - 1; l >= 0; --l) {
            MlLevel &L = f->lv[l];
            const MlLevel &Lp = f->lv[l + 1];
            tensor(Lp.n, L.n, Lp.CT[0], Lp.CT[1], L.par_ptr, L.par_box, L.par_bits, Lp.Lq, L.Lq, L.nbox, true, st);
        }
        hipLaunchKernelGGL(k_ml_disaggregate, dim3(unsigned(N)), dim3(256), 0, st, f->c0.npts, N, f->box_of, f->meq,
                           (const double2 *)L0.Lq, (double2 *)Y + r * N);
        BIE_HIP(hipGetLastError());
    }
}

void farml_level_info(const bie_farml *f, int level, bie_far_info *info)
{
    if (level < 0 || level >= f->levels) throw Error(BIE_EINVAL, "level out of range");
    const MlLevel &L = f->lv[level];
    info->boxes = L.nbox;
    info->far_pairs = L.npairs;
    info->buffer_knots = L.sb;
    info->splines = L.n;
    info->points_per_axis = L.nst;
    info->protrusion = f->prot;
    for (int d = 0; d < 3; ++d) info->origin[d] = f->origin[d];
}

void farml_leaves(const bie_farml *f, std::vector<int32_t> &box_of, std::vector<int32_t> &ijk)
{
    box_of = f->h_box_of;
    ijk = f->lv[0].h_ijk;
}

void farml_destroy(bie_farml *f) { delete f; }

}  // namespace bie
