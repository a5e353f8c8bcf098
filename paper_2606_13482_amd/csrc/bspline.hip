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
    c.p = p;
    c.a = a;
    c.n = s + 2 * sb;
    c.lo = -sb * du;
    c.hi = 1.0 + sb * du;
    c.nst = c.n - 2 * r;
    c.npts = c.nst * c.nst * c.nst;
    if (c.n > MAXN || c.npts > 256 * UPT) throw Error(BIE_EINVAL, "too many splines per box");
    const std::vector<double> ueq = open_knots(c.n, p, c.lo, c.hi);
    std::vector<double> ust(ueq.begin(), ueq.begin() + p + 1);
    for (int i = p + 1 + r; i < c.n - r; ++i) ust.push_back(ueq[i]);
    for (int i = 0; i <= p; ++i) ust.push_back(c.hi);
    std::vector<double> hA(size_t(c.nst) * c.n);
    // stabilised sampling matrix B[i][m] = b_i(t_m) at n' equispaced points
    std::vector<double> tpt(c.nst), B(size_t(c.nst) * c.nst);
    for (int m = 0; m < c.nst; ++m) tpt[m] = m == c.nst - 1 ? c.hi : c.lo + (c.hi - c.lo) * m / double(c.nst - 1);
    for (int m = 0; m < c.nst; ++m) {
        const std::vector<double> v = all_splines(ust, p, tpt[m]);
        for (int i = 0; i < c.nst; ++i) B[size_t(i) * c.nst + m] = v[i];
    }
    const std::vector<double> Bi = invert(B, c.nst);
    // C: stabilised spline j in the equidistant splines (insert the removed knots)
    std::vector<double> removed;
    for (int i = p + 1; i < p + 1 + r; ++i) removed.push_back(ueq[i]);
    for (int i = c.n - r; i < c.n; ++i) removed.push_back(ueq[i]);
    std::vector<double> Cm(size_t(c.nst) * c.n);
    for (int j = 0; j < c.nst; ++j) {
        std::vector<double> u = ust, w(size_t(c.nst), 0.0);
        w[j] = 1.0;
        for (double ub : removed) insert_one(u, p, w, ub);
        for (int i = 0; i < c.n; ++i) Cm[size_t(j) * c.n + i] = w[i];
    }
    for (int k = 0; k < c.nst; ++k)
        for (int i = 0; i < c.n; ++i) {
            double v = 0.0;
            for (int j = 0; j < c.nst; ++j) v += Bi[size_t(k) * c.nst + j] * Cm[size_t(j) * c.n + i];
            hA[size_t(k) * c.n + i] = v;
        }
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
