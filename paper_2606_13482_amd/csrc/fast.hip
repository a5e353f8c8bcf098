// Fast operator: T x = N x + F x without the dense matrix.
//
// F: the multilevel B-spline far field (Sec. IV, bspline.hip) over the pairs of
// far leaf cubes.  N: the entries T_mn of the RWG functions m, n whose leaf
// cubes are near (Chebyshev index distance <= 1; the complement of F's pairs),
// computed like the dense fill (Sec. II, eq:matTA, eq:matTPhi): for each of the
// four triangle pairs of (m, n) the local value
//     L(p, a, q, b) = s_a s_b [ (jk/4) J_ab + J0/(jk) ]
// with Radon's 7-point rule on both triangles, or, for pairs the mesh flags as
// touching or near, the fill's singular treatment (the flagged pairs' blocks are
// computed once, pair by pair, by the fill's own kernel); then
//     T_mn = (L(+,+) + L(-,-)) + (L(+,-) + L(-,+)).
// N is kept in CSR by row (column indices ascending) and applied one wave per
// row.  Memory: the near entries (16 B + 4 B each), the flagged blocks (144 B
// per pair), the far field's moments and level arrays; nothing of size N^2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <memory>
#include <vector>

#include "bie_internal.hpp"

namespace bie {

struct FastOp {
    bie_farml *far = nullptr;
    int64_t nnz = 0, cubes = 0;
    int levels = 0;
    int64_t *rowptr = nullptr;
    int32_t *cols = nullptr;
    double2 *vals = nullptr;
    double2 *tmp = nullptr;         // far product of one column
    double *qw = nullptr;           // Radon weights
    int32_t *fptr = nullptr, *fq = nullptr;   // flagged partners q >= p of each triangle p, ascending
    double *fblk = nullptr;         // their blocks, 18 doubles per pair (index = position in fq)
    ~FastOp()
    {
        if (far) farml_destroy(far);
        for (void *p : { (void *)rowptr, (void *)cols, (void *)vals, (void *)tmp, (void *)qw, (void *)fptr, (void *)fq,
                         (void *)fblk })
            if (p) (void)hipFree(p);
    }
};

namespace {

constexpr int NQF = QPTS;   // quadrature points per triangle

// L(p, a, q, b) for p <= q (regular rule or the flagged block)
__device__ inline double2 local_block(int32_t p, int32_t a, int32_t q, int32_t b, const double *__restrict__ cent,
                                      const double *__restrict__ loc, const double *__restrict__ vfree,
                                      const int8_t *__restrict__ sgn, const double *__restrict__ qw,
                                      const int32_t *__restrict__ fptr, const int32_t *__restrict__ fq,
                                      const double *__restrict__ fblk, double k)
{
    if (p > q) {   // L(p, a, q, b) = L(q, b, p, a): the kernel is symmetric
        const int32_t t = p;
        p = q;
        q = t;
        const int32_t u = a;
        a = b;
        b = u;
    }
    // flagged?
    int32_t lo = fptr[p], hi = fptr[p + 1];
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (fq[mid] < q) lo = mid + 1;
        else hi = mid;
    }
    if (lo < fptr[p + 1] && fq[lo] == q) {
        const double *bl = fblk + int64_t(lo) * 18 + (a * 3 + b) * 2;
        return make_double2(bl[0], bl[1]);
    }
    const double inv4pi = 1.0 / (4.0 * M_PI);
    double dc[3], va[3], vb[3];
    for (int d = 0; d < 3; ++d) {
        dc[d] = cent[3 * int64_t(p) + d] - cent[3 * int64_t(q) + d];
        va[d] = vfree[9 * int64_t(p) + 3 * a + d];
        vb[d] = vfree[9 * int64_t(q) + 3 * b + d];
    }
    const double *xl = loc + int64_t(p) * NQF * 3, *yl = loc + int64_t(q) * NQF * 3;
    double jr = 0.0, ji = 0.0, s0r = 0.0, s0i = 0.0;
    for (int i = 0; i < NQF; ++i) {
        const double xi[3] = { xl[3 * i], xl[3 * i + 1], xl[3 * i + 2] };
        const double da[3] = { xi[0] - va[0], xi[1] - va[1], xi[2] - va[2] };
        for (int j = 0; j < NQF; ++j) {
            const double d0 = dc[0] + xi[0] - yl[3 * j], d1 = dc[1] + xi[1] - yl[3 * j + 1],
                         d2 = dc[2] + xi[2] - yl[3 * j + 2];
            const double R = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
            double sn, cs;
            sincos(k * R, &sn, &cs);
            const double w = qw[i] * qw[j] * inv4pi / R;
            const double gr = w * cs, gi = -w * sn;
            const double dd = da[0] * (yl[3 * j] - vb[0]) + da[1] * (yl[3 * j + 1] - vb[1]) + da[2] * (yl[3 * j + 2] - vb[2]);
            s0r += gr;
            s0i += gi;
            jr += gr * dd;
            ji += gi * dd;
        }
    }
    const double ss = double(sgn[3 * int64_t(p) + a] * sgn[3 * int64_t(q) + b]);
    const double k4 = 0.25 * k, ik = 1.0 / k;
    return make_double2(ss * (-k4 * ji + ik * s0i), ss * (k4 * jr - ik * s0r));
}

// The near entries of row m (one block per row, threads over its entries).
__global__ __launch_bounds__(256) void k_near_entries(int64_t N, const int64_t *__restrict__ rowptr,
                                                      const int32_t *__restrict__ cols, const int4 *__restrict__ rwg4,
                                                      const double *__restrict__ cent, const double *__restrict__ loc,
                                                      const double *__restrict__ vfree, const int8_t *__restrict__ sgn,
                                                      const double *__restrict__ qw, const int32_t *__restrict__ fptr,
                                                      const int32_t *__restrict__ fq, const double *__restrict__ fblk,
                                                      double k, double2 *__restrict__ vals)
{
    const int64_t m = blockIdx.x;
    if (m >= N) return;
    const int4 em = rwg4[m];
    for (int64_t e = rowptr[m] + threadIdx.x; e < rowptr[m + 1]; e += 256) {
        const int4 en = rwg4[cols[e]];
        const double2 l1 = local_block(em.x, em.z, en.x, en.z, cent, loc, vfree, sgn, qw, fptr, fq, fblk, k);   // (+,+)
        const double2 l2 = local_block(em.y, em.w, en.y, en.w, cent, loc, vfree, sgn, qw, fptr, fq, fblk, k);   // (-,-)
        const double2 l3 = local_block(em.x, em.z, en.y, en.w, cent, loc, vfree, sgn, qw, fptr, fq, fblk, k);   // (+,-)
        const double2 l4 = local_block(em.y, em.w, en.x, en.z, cent, loc, vfree, sgn, qw, fptr, fq, fblk, k);   // (-,+)
        vals[e] = make_double2((l1.x + l2.x) + (l3.x + l4.x), (l1.y + l2.y) + (l3.y + l4.y));
    }
}

// y_m = (B_m -) (sum_e vals[e] x[cols[e]] + far_m), one wave per row.
__global__ __launch_bounds__(256) void k_near_apply(int64_t N, const int64_t *__restrict__ rowptr,
                                                    const int32_t *__restrict__ cols, const double2 *__restrict__ vals,
                                                    const double2 *__restrict__ x, const double2 *__restrict__ far,
                                                    const double2 *__restrict__ B, double2 *__restrict__ y)
{
    const int64_t m = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (m >= N) return;
    double ar = 0.0, ai = 0.0;
    for (int64_t e = rowptr[m] + lane; e < rowptr[m + 1]; e += 64) {
        const double2 v = vals[e], xv = x[cols[e]];
        ar += v.x * xv.x - v.y * xv.y;
        ai += v.x * xv.y + v.y * xv.x;
    }
    for (int o = 32; o > 0; o >>= 1) {
        ar += __shfl_xor(ar, o, 64);
        ai += __shfl_xor(ai, o, 64);
    }
    if (lane == 0) {
        const double2 f = far[m];
        const double tr = ar + f.x, ti = ai + f.y;
        y[m] = B ? make_double2(B[m].x - tr, B[m].y - ti) : make_double2(tr, ti);
    }
}

template <typename T>
T *up(const std::vector<T> &v)
{
    void *d = nullptr;
    BIE_HIP(hipMalloc(&d, std::max<size_t>(v.size(), 1) * sizeof(T)));
    if (!v.empty()) BIE_HIP(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return static_cast<T *>(d);
}

}  // namespace

void fast_setup(bie_op *op, double box, int levels, int s, int p, hipStream_t st)
{
    auto f = std::make_unique<FastOp>();
    f->far = farml_create(op, box, levels, s, p, st);
    f->levels = levels;
    const Mesh &M = op->mesh;
    const int64_t N = M.N, F = M.F;
    std::vector<int32_t> box_of, ijk;
    farml_leaves(f->far, box_of, ijk);
    const int64_t nb = int64_t(ijk.size() / 3);
    f->cubes = nb;
    std::map<std::array<int32_t, 3>, int32_t> index;
    for (int32_t b = 0; b < nb; ++b) index[{ ijk[3 * b], ijk[3 * b + 1], ijk[3 * b + 2] }] = b;
    std::vector<std::vector<int32_t>> members(nb);
    for (int64_t m = 0; m < N; ++m) members[box_of[m]].push_back(int32_t(m));
    // near CSR: every function of the 27 cubes around the row's cube
    std::vector<int64_t> rowptr(N + 1, 0);
    std::vector<int32_t> cols;
    std::vector<std::vector<int32_t>> nearcols(nb);
    for (int32_t b = 0; b < nb; ++b) {
        std::vector<int32_t> &c = nearcols[b];
        for (int dx = -1; dx <= 1; ++dx)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dz = -1; dz <= 1; ++dz) {
                    auto it = index.find({ ijk[3 * b] + dx, ijk[3 * b + 1] + dy, ijk[3 * b + 2] + dz });
                    if (it != index.end()) c.insert(c.end(), members[it->second].begin(), members[it->second].end());
                }
        std::sort(c.begin(), c.end());
    }
    for (int64_t m = 0; m < N; ++m) rowptr[m + 1] = rowptr[m] + int64_t(nearcols[box_of[m]].size());
    cols.reserve(size_t(rowptr[N]));
    for (int64_t m = 0; m < N; ++m) cols.insert(cols.end(), nearcols[box_of[m]].begin(), nearcols[box_of[m]].end());
    f->nnz = rowptr[N];
    // flagged pairs by first triangle, partners ascending
    const int64_t nflag = int64_t(M.near.size() / 2);
    std::vector<std::pair<int32_t, int32_t>> fl(static_cast<size_t>(nflag));
    for (int64_t i = 0; i < nflag; ++i) fl[i] = { M.near[2 * i], M.near[2 * i + 1] };
    std::sort(fl.begin(), fl.end());
    std::vector<int32_t> fptr(F + 1, 0), fq(static_cast<size_t>(nflag)), fpairs(2 * static_cast<size_t>(nflag));
    for (int64_t i = 0; i < nflag; ++i) {
        ++fptr[fl[i].first + 1];
        fq[i] = fl[i].second;
        fpairs[2 * i] = fl[i].first;
        fpairs[2 * i + 1] = fl[i].second;
    }
    for (int64_t t = 0; t < F; ++t) fptr[t + 1] += fptr[t];
    double qwh[QPTS];
    quad_weights(qwh);
    f->qw = up(std::vector<double>(qwh, qwh + QPTS));
    f->fptr = up(fptr);
    f->fq = up(fq);
    f->rowptr = up(rowptr);
    f->cols = up(cols);
    BIE_HIP(hipMalloc(&f->fblk, std::max<int64_t>(nflag, 1) * 18 * sizeof(double)));
    BIE_HIP(hipMalloc(&f->vals, std::max<int64_t>(f->nnz, 1) * sizeof(double2)));
    BIE_HIP(hipMalloc(&f->tmp, std::max<int64_t>(N, 1) * sizeof(double2)));
    int32_t *dpairs = up(fpairs);
    singular_blocks(op, dpairs, nflag, f->fblk, st);
    const TriDev &D = op->tri;
    hipLaunchKernelGGL(k_near_entries, dim3(unsigned(N)), dim3(256), 0, st, N, f->rowptr, f->cols,
                       (const int4 *)D.edges, D.cent, D.loc, D.vfree, D.sgn, f->qw, f->fptr, f->fq, f->fblk, op->k,
                       f->vals);
    BIE_HIP(hipGetLastError());
    BIE_HIP(hipStreamSynchronize(st));
    (void)hipFree(dpairs);
    op->fast = f.release();
}

void fast_product(const bie_op *op, const void *X, int64_t ldx, void *Y, int64_t ldy, const void *B, int64_t ldb,
                  int64_t R, hipStream_t st)
{
    FastOp *f = op->fast;
    const int64_t N = op->mesh.N;
    for (int64_t r = 0; r < R; ++r) {
        const double2 *x = static_cast<const double2 *>(X) + r * ldx;
        farml_apply(f->far, x, f->tmp, 1, st);
        hipLaunchKernelGGL(k_near_apply, dim3(unsigned((N + 3) / 4)), dim3(256), 0, st, N, f->rowptr, f->cols, f->vals,
                           x, (const double2 *)f->tmp, B ? static_cast<const double2 *>(B) + r * ldb : nullptr,
                           static_cast<double2 *>(Y) + r * ldy);
        BIE_HIP(hipGetLastError());
    }
}

void fast_info(const bie_op *op, bie_fast_info *info)
{
    const FastOp *f = op->fast;
    info->near_entries = f->nnz;
    info->leaf_cubes = f->cubes;
    info->levels = f->levels;
}

void fast_destroy(FastOp *f) { delete f; }

}  // namespace bie
