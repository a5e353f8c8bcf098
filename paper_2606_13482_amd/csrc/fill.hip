// Dense EFIE impedance matrix fill, plane-wave excitation and radiation vector.
//
// Operator (Sec. II, eq:efie, eq:matTA, eq:matTPhi) in RWG functions without
// edge-length normalisation.  On triangle p of f_m: f_m = s (r - v)/(2 A_p),
// div f_m = s / A_p.  For a triangle pair (p, q) and local slots a, b the
// contribution to T_{m(p,a), n(q,b)} is
//     L_ab = s_a s_b [ (jk/4) J_ab + J0/(jk) ],
//     J_ab = sum_ij w_i w_j (x_i - v_a).(y_j - v_b) g(|x_i - y_j|),  J0 = sum_ij w_i w_j g
// with area-relative weights (the areas cancel against 1/(A_p A_q)).  The
// minus signs of eq:efie and eq:matTPhi cancel.
//
// Star-split form (Sec. VI-A, star factorisation of the scalar potential):
// with div f_m = +-1/A on c_m^+- the scalar term of T is Sigma V Sigma^T,
// Sigma_mp = s (the sign of triangle p in RWG m) and V_pq = J0 / (jk) the
// piecewise-constant single layer (basis 1/A) scaled by 1/(jk).  In that form
// the local blocks keep only the vector part s_a s_b (jk/4) J_ab (assembled
// into T_A' = jk T_A exactly as T), and J0 / (jk) of every pair p <= q is
// written to its own tile array and assembled into packed F x F tiles of V'.
//
// Pipeline (three launches, no atomics, bitwise symmetric result):
//   1. k_pairs_regular: one thread per ordered triangle pair p <= q of a 16x16
//      triangle tile staged in LDS; 49 kernel evaluations; writes the 3x3
//      local block L into a tile-major scratch array.
//   2. k_pairs_singular: one FP64 thread per flagged pair (touching or near):
//      g = g_r + 1/(4 pi R), g_r on the product rule, the static part with the
//      inner integral in closed form, mean of both orderings; overwrites L.
//   3. k_assemble: T_mn = (L(c+m,c+n) + L(c-m,c-n)) + (L(c+m,c-n) + L(c-m,c+n));
//      the grouping makes T_mn and T_nm the same sum, so T = T^T exactly, and
//      only the upper-triangular 64 x 64 tiles are written (packed storage).
#include <hip/hip_runtime.h>

#include <cmath>

#include "bie_internal.hpp"

namespace bie {

namespace {

constexpr int TT = 16;               // triangles per tile side
constexpr int NQ = 7;                // Radon 7-point rule
constexpr double PI = 3.14159265358979323846;

// Radon's degree-5 rule: centroid, orbits (a,a,1-2a) with a = (6 -+ sqrt(15))/21.
struct Rule {
    double bary[NQ][3];
    double w[NQ];
};

Rule make_rule()
{
    Rule r;
    const double s = std::sqrt(15.0);
    const double a = (6.0 - s) / 21.0, b = (6.0 + s) / 21.0;
    const double wa = (155.0 - s) / 1200.0, wb = (155.0 + s) / 1200.0;
    const double pts[NQ][3] = { { 1.0 / 3, 1.0 / 3, 1.0 / 3 },
                                { a, a, 1 - 2 * a }, { a, 1 - 2 * a, a }, { 1 - 2 * a, a, a },
                                { b, b, 1 - 2 * b }, { b, 1 - 2 * b, b }, { 1 - 2 * b, b, b } };
    const double ws[NQ] = { 9.0 / 40.0, wa, wa, wa, wb, wb, wb };
    for (int i = 0; i < NQ; ++i) {
        for (int d = 0; d < 3; ++d) r.bary[i][d] = pts[i][d];
        r.w[i] = ws[i];
    }
    return r;
}

__constant__ double c_w[NQ];

__host__ __device__ inline int64_t tile_index(int64_t I, int64_t J, int64_t nT)
{
    return I * nT - I * (I - 1) / 2 + (J - I);
}

// ---------------------------------------------------------------------------
// 1. Regular pairs.
template <typename R>
struct TriLDS {
    R loc[NQ][3];
    R vf[3][3];
};
// FP64: one double of padding (31 per triangle), so that the 16 triangles of a
// tile read in one instruction start in 16 different bank pairs (30 doubles put
// triangles 8 apart in the same banks: a two-way conflict on every read).
template <>
struct TriLDS<double> {
    double loc[NQ][3];
    double vf[3][3];
    double pad;
};

template <typename R>
__device__ inline void sincos_t(R x, R *s, R *c);
template <>
__device__ inline void sincos_t<double>(double x, double *s, double *c) { sincos(x, s, c); }
template <>
__device__ inline void sincos_t<float>(float x, float *s, float *c)
{
    // Reduce to [-1/2, 1/2] revolutions, then the hardware sine / cosine.
    const float rev = x * 0.15915494309189533577f;
    const float f = rev - rintf(rev);
    *s = __builtin_amdgcn_sinf(f);
    *c = __builtin_amdgcn_cosf(f);
}

template <typename R>
__device__ inline R rsqrt_t(R x);
template <>
__device__ inline double rsqrt_t<double>(double x) { return 1.0 / sqrt(x); }
template <>
__device__ inline float rsqrt_t<float>(float x) { return rsqrtf(x); }

template <typename R, bool SPLIT>
__global__ __launch_bounds__(256) void k_pairs_regular(int64_t F, int64_t nT, int64_t ntiles,
                                                       const double *__restrict__ cent,
                                                       const double *__restrict__ loc,
                                                       const double *__restrict__ vfree,
                                                       const int8_t *__restrict__ sgn, double k,
                                                       R *__restrict__ LB, R *__restrict__ VS)
{
    __shared__ TriLDS<R> sp[TT], sq[TT];
    __shared__ double scp[TT][3], scq[TT][3];
    __shared__ R sw[NQ];    // w_j / (4 pi)
    __shared__ R swi[NQ];   // w_i
    const int64_t b = blockIdx.x;
    if (b >= ntiles) return;
    // decode b -> (I, J), I <= J, row-major over the upper triangle of tiles
    const double n2 = 2.0 * double(nT) + 1.0;
    int64_t I = int64_t((n2 - sqrt(n2 * n2 - 8.0 * double(b))) * 0.5);
    if (I < 0) I = 0;
    if (I > nT - 1) I = nT - 1;
    while (I > 0 && tile_index(I, I, nT) > b) --I;
    while (I + 1 < nT && tile_index(I + 1, I + 1, nT) <= b) ++I;
    const int64_t J = I + (b - tile_index(I, I, nT));

    const int tid = threadIdx.x;
    // stage the two triangle tiles (local coordinates relative to centroids)
    for (int e = tid; e < TT * (NQ * 3 + 9 + 3); e += 256) {
        const int t = e / (NQ * 3 + 9 + 3), f = e % (NQ * 3 + 9 + 3);
        for (int side = 0; side < 2; ++side) {
            const int64_t tri = (side ? J : I) * TT + t;
            TriLDS<R> *dst = side ? &sq[t] : &sp[t];
            double v = 0.0;
            if (tri < F) {
                if (f < NQ * 3) v = loc[tri * NQ * 3 + f];
                else if (f < NQ * 3 + 9) v = vfree[tri * 9 + (f - NQ * 3)];
                else v = cent[tri * 3 + (f - NQ * 3 - 9)];
            }
            if (f < NQ * 3) dst->loc[f / 3][f % 3] = R(v);
            else if (f < NQ * 3 + 9) dst->vf[(f - NQ * 3) / 3][(f - NQ * 3) % 3] = R(v);
            else (side ? scq : scp)[t][f - NQ * 3 - 9] = v;
        }
    }
    if (tid < NQ) {
        sw[tid] = R(c_w[tid] / (4.0 * PI));
        swi[tid] = R(c_w[tid]);
    }
    __syncthreads();

    const int ti = tid / TT, tj = tid % TT;
    const int64_t p = I * TT + ti, q = J * TT + tj;
    if (p >= F || q >= F || p > q) return;
    const TriLDS<R> &P = sp[ti];
    const TriLDS<R> &Q = sq[tj];
    const R dc[3] = { R(scp[ti][0] - scq[tj][0]), R(scp[ti][1] - scq[tj][1]), R(scp[ti][2] - scq[tj][2]) };
    const R kk = R(k);

    R s0r = 0, s0i = 0, sxr[3] = { 0, 0, 0 }, sxi[3] = { 0, 0, 0 }, syr[3] = { 0, 0, 0 }, syi[3] = { 0, 0, 0 };
    R sxyr = 0, sxyi = 0;
#pragma unroll 1
    for (int i = 0; i < NQ; ++i) {
        const R xi[3] = { P.loc[i][0], P.loc[i][1], P.loc[i][2] };
        const R di[3] = { dc[0] + xi[0], dc[1] + xi[1], dc[2] + xi[2] };
        R t0r = 0, t0i = 0, tyr[3] = { 0, 0, 0 }, tyi[3] = { 0, 0, 0 };
#pragma unroll
        for (int j = 0; j < NQ; ++j) {
            const R d0 = di[0] - Q.loc[j][0], d1 = di[1] - Q.loc[j][1], d2 = di[2] - Q.loc[j][2];
            const R r2 = d0 * d0 + d1 * d1 + d2 * d2;
            const R ri = rsqrt_t<R>(r2);
            R sn, cs;
            sincos_t<R>(kk * (r2 * ri), &sn, &cs);
            const R gw = sw[j] * ri;
            const R gr = gw * cs, gi = -gw * sn;
            t0r += gr;
            t0i += gi;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                tyr[c] += gr * Q.loc[j][c];
                tyi[c] += gi * Q.loc[j][c];
            }
        }
        const R a = swi[i];
        s0r += a * t0r;
        s0i += a * t0i;
        R xtr = 0, xti = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            sxr[c] += a * t0r * xi[c];
            sxi[c] += a * t0i * xi[c];
            syr[c] += a * tyr[c];
            syi[c] += a * tyi[c];
            xtr += xi[c] * tyr[c];
            xti += xi[c] * tyi[c];
        }
        sxyr += a * xtr;
        sxyi += a * xti;
    }
    // J_ab = Sxy - v_b.Sx - v_a.Sy + (v_a.v_b) S0   (local coordinates)
    // L_ab = s_a s_b [ (jk/4) J_ab + S0/(jk) ]
    const int64_t tile = tile_index(I, J, nT);
    R *out = LB + tile * (9 * 256 * 2);
    const R k4 = kk * R(0.25), ik = R(1.0) / kk;
#pragma unroll
    for (int aa = 0; aa < 3; ++aa) {
#pragma unroll
        for (int bb = 0; bb < 3; ++bb) {
            const R *va = P.vf[aa];
            const R *vb = Q.vf[bb];
            R jr = sxyr, ji = sxyi;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                jr -= vb[c] * sxr[c] + va[c] * syr[c];
                ji -= vb[c] * sxi[c] + va[c] * syi[c];
            }
            const R vv = va[0] * vb[0] + va[1] * vb[1] + va[2] * vb[2];
            jr += vv * s0r;
            ji += vv * s0i;
            const R ss = R(sgn[p * 3 + aa] * sgn[q * 3 + bb]);
            const R lr = SPLIT ? ss * (-k4 * ji) : ss * (-k4 * ji + ik * s0i);
            const R li = SPLIT ? ss * (k4 * jr) : ss * (k4 * jr - ik * s0r);
            out[((aa * 3 + bb) * 256 + tid) * 2 + 0] = lr;
            out[((aa * 3 + bb) * 256 + tid) * 2 + 1] = li;
        }
    }
    if (SPLIT) {   // V'_pq = J0 / (jk)
        VS[(tile * 256 + tid) * 2 + 0] = ik * s0i;
        VS[(tile * 256 + tid) * 2 + 1] = -ik * s0r;
    }
}

// ---------------------------------------------------------------------------
// 2. Flagged pairs, FP64.
//
// K0 = int_tri 1/|y-x|, K1 = int_tri (y-x)/|y-x| in closed form (Wilton et al.
// 1984, Graglia 1993): per edge P->Q (CCW about the unit normal n), with
// h = n.(x-P), rho = x - h n, l = (Q-P)/|Q-P|, u = l x n,
// l+- = (Q|P - rho).l, P0 = (P - rho).u, R0^2 = P0^2 + h^2, R+- = sqrt(R0^2 + l+-^2),
// f = ln((R+ + l+)/(R- + l-)) (or ln((R- - l-)/(R+ - l+)) if l+ + l- < 0),
// beta = atan(P0 l+/(R0^2 + |h| R+)) - atan(P0 l-/(R0^2 + |h| R-)):
//   K0 = sum P0 f - |h| beta,  K1 = 1/2 sum u (R0^2 f + l+ R+ - l- R-) - h n K0.
__device__ void static_potentials(const double x[3], const double A[3], const double B[3],
                                  const double C[3], double *K0, double K1[3])
{
    double e1[3], e2[3], n[3];
    for (int d = 0; d < 3; ++d) { e1[d] = B[d] - A[d]; e2[d] = C[d] - A[d]; }
    n[0] = e1[1] * e2[2] - e1[2] * e2[1];
    n[1] = e1[2] * e2[0] - e1[0] * e2[2];
    n[2] = e1[0] * e2[1] - e1[1] * e2[0];
    const double nn = 1.0 / sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    n[0] *= nn; n[1] *= nn; n[2] *= nn;
    const double h = (x[0] - A[0]) * n[0] + (x[1] - A[1]) * n[1] + (x[2] - A[2]) * n[2];
    const double ah = fabs(h);
    const double rho[3] = { x[0] - h * n[0], x[1] - h * n[1], x[2] - h * n[2] };
    const double *Ps[3] = { A, B, C }, *Qs[3] = { B, C, A };
    double k0 = 0.0, kp[3] = { 0.0, 0.0, 0.0 };
    for (int e = 0; e < 3; ++e) {
        const double *P = Ps[e], *Q = Qs[e];
        double l[3] = { Q[0] - P[0], Q[1] - P[1], Q[2] - P[2] };
        const double il = 1.0 / sqrt(l[0] * l[0] + l[1] * l[1] + l[2] * l[2]);
        l[0] *= il; l[1] *= il; l[2] *= il;
        const double u[3] = { l[1] * n[2] - l[2] * n[1], l[2] * n[0] - l[0] * n[2], l[0] * n[1] - l[1] * n[0] };
        const double lp = (Q[0] - rho[0]) * l[0] + (Q[1] - rho[1]) * l[1] + (Q[2] - rho[2]) * l[2];
        const double lm = (P[0] - rho[0]) * l[0] + (P[1] - rho[1]) * l[1] + (P[2] - rho[2]) * l[2];
        const double P0 = (P[0] - rho[0]) * u[0] + (P[1] - rho[1]) * u[1] + (P[2] - rho[2]) * u[2];
        const double R0s = P0 * P0 + h * h;
        const double Rp = sqrt(R0s + lp * lp), Rm = sqrt(R0s + lm * lm);
        double f = 0.0;
        if (R0s > 0.0) f = (lp + lm < 0.0) ? log((Rm - lm) / (Rp - lp)) : log((Rp + lp) / (Rm + lm));
        double beta = 0.0;
        if (ah > 0.0) beta = atan2(P0 * lp, R0s + ah * Rp) - atan2(P0 * lm, R0s + ah * Rm);
        k0 += (R0s > 0.0 ? P0 * f : 0.0) - ah * beta;
        const double c = 0.5 * ((R0s > 0.0 ? R0s * f : 0.0) + lp * Rp - lm * Rm);
        kp[0] += c * u[0]; kp[1] += c * u[1]; kp[2] += c * u[2];
    }
    *K0 = k0;
    for (int d = 0; d < 3; ++d) K1[d] = kp[d] - h * n[d] * k0;
}

template <typename R, bool SPLIT>
__global__ __launch_bounds__(128) void k_pairs_singular(int64_t npairs, int64_t nT,
                                                        const int32_t *__restrict__ pairs,
                                                        const double *__restrict__ cent,
                                                        const double *__restrict__ loc,
                                                        const double *__restrict__ vfree,
                                                        const double *__restrict__ verts,
                                                        const double *__restrict__ area,
                                                        const int8_t *__restrict__ sgn, double k,
                                                        R *__restrict__ LB, R *__restrict__ VS,
                                                        double *__restrict__ compact = nullptr)
{
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= npairs) return;
    const int64_t p = pairs[2 * idx], q = pairs[2 * idx + 1];
    // frames: p-local coordinates relative to c_p, q-local relative to c_q
    double dc[3];
    for (int d = 0; d < 3; ++d) dc[d] = cent[p * 3 + d] - cent[q * 3 + d];
    const double *xl = loc + p * NQ * 3, *yl = loc + q * NQ * 3;
    const double *vp = vfree + p * 9, *vq = vfree + q * 9;
    double trp[9], trq[9];   // vertices relative to own centroid
    for (int v = 0; v < 3; ++v)
        for (int d = 0; d < 3; ++d) {
            trp[v * 3 + d] = verts[p * 9 + v * 3 + d] - cent[p * 3 + d];
            trq[v * 3 + d] = verts[q * 9 + v * 3 + d] - cent[q * 3 + d];
        }
    const double inv4pi = 1.0 / (4.0 * PI);
    double jr[3][3] = { { 0 } }, ji[3][3] = { { 0 } }, j0r = 0.0, j0i = 0.0;
    // regular remainder g_r = (e^{-jkR} - 1)/(4 pi R) = (-2 sin^2(kR/2) - j sin kR)/(4 pi R)
    for (int i = 0; i < NQ; ++i) {
        for (int j = 0; j < NQ; ++j) {
            double d[3];
            for (int c = 0; c < 3; ++c) d[c] = dc[c] + xl[i * 3 + c] - yl[j * 3 + c];
            const double Rr = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            double gr, gi;
            if (Rr > 0.0) {
                const double s = sin(0.5 * k * Rr);
                gr = -2.0 * s * s / Rr * inv4pi;
                gi = -sin(k * Rr) / Rr * inv4pi;
            } else {
                gr = 0.0;
                gi = -k * inv4pi;
            }
            const double w = c_w[i] * c_w[j];
            gr *= w; gi *= w;
            j0r += gr; j0i += gi;
            for (int a = 0; a < 3; ++a) {
                const double da[3] = { xl[i * 3] - vp[a * 3], xl[i * 3 + 1] - vp[a * 3 + 1], xl[i * 3 + 2] - vp[a * 3 + 2] };
                for (int b = 0; b < 3; ++b) {
                    const double db[3] = { yl[j * 3] - vq[b * 3], yl[j * 3 + 1] - vq[b * 3 + 1], yl[j * 3 + 2] - vq[b * 3 + 2] };
                    const double dd = da[0] * db[0] + da[1] * db[1] + da[2] * db[2];
                    jr[a][b] += gr * dd;
                    ji[a][b] += gi * dd;
                }
            }
        }
    }
    // static part, real: p outer / closed form over q, and q outer / over p; mean.
    double sr[3][3] = { { 0 } }, s0 = 0.0;
    const double Ap = area[p], Aq = area[q];
    for (int i = 0; i < NQ; ++i) {
        const double x[3] = { dc[0] + xl[i * 3], dc[1] + xl[i * 3 + 1], dc[2] + xl[i * 3 + 2] };  // in q frame
        double K0, K1[3];
        static_potentials(x, trq, trq + 3, trq + 6, &K0, K1);
        const double f = c_w[i] * inv4pi / Aq;
        s0 += f * K0;
        for (int a = 0; a < 3; ++a) {
            const double da[3] = { xl[i * 3] - vp[a * 3], xl[i * 3 + 1] - vp[a * 3 + 1], xl[i * 3 + 2] - vp[a * 3 + 2] };
            for (int b = 0; b < 3; ++b) {
                // int_q (y - v_b)/R = K1 + (x - v_b) K0, with x and v_b in the q frame
                double iv[3];
                for (int c = 0; c < 3; ++c) iv[c] = K1[c] + (x[c] - vq[b * 3 + c]) * K0;
                sr[a][b] += f * (da[0] * iv[0] + da[1] * iv[1] + da[2] * iv[2]);
            }
        }
    }
    for (int j = 0; j < NQ; ++j) {
        const double y[3] = { yl[j * 3] - dc[0], yl[j * 3 + 1] - dc[1], yl[j * 3 + 2] - dc[2] };  // in p frame
        double K0, K1[3];
        static_potentials(y, trp, trp + 3, trp + 6, &K0, K1);
        const double f = c_w[j] * inv4pi / Ap;
        s0 += f * K0;
        for (int b = 0; b < 3; ++b) {
            const double db[3] = { yl[j * 3] - vq[b * 3], yl[j * 3 + 1] - vq[b * 3 + 1], yl[j * 3 + 2] - vq[b * 3 + 2] };
            for (int a = 0; a < 3; ++a) {
                double iv[3];
                for (int c = 0; c < 3; ++c) iv[c] = K1[c] + (y[c] - vp[a * 3 + c]) * K0;
                sr[a][b] += f * (db[0] * iv[0] + db[1] * iv[1] + db[2] * iv[2]);
            }
        }
    }
    j0r += 0.5 * s0;
    const int64_t I = p / TT, J = q / TT;
    R *out = LB + tile_index(I, J, nT) * (9 * 256 * 2);
    const int tid = int((p % TT) * TT + (q % TT));
    const double k4 = 0.25 * k, ik = 1.0 / k;
    double Jr_[3][3], Ji_[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            Jr_[a][b] = jr[a][b] + 0.5 * sr[a][b];
            Ji_[a][b] = ji[a][b];
        }
    if (p == q) {
        // J_ab = J_ba for a self pair (swap the two integration variables);
        // take the mean so the stored block is symmetric to the last bit.
        for (int a = 0; a < 3; ++a)
            for (int b = a + 1; b < 3; ++b) {
                const double mr = 0.5 * (Jr_[a][b] + Jr_[b][a]), mi = 0.5 * (Ji_[a][b] + Ji_[b][a]);
                Jr_[a][b] = Jr_[b][a] = mr;
                Ji_[a][b] = Ji_[b][a] = mi;
            }
    }
    if (compact) {   // the pair's 3 x 3 block, pair after pair (near field of the fast operator)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                const double ss = double(sgn[p * 3 + a] * sgn[q * 3 + b]);
                compact[idx * 18 + (a * 3 + b) * 2 + 0] = ss * (-k4 * Ji_[a][b] + ik * j0i);
                compact[idx * 18 + (a * 3 + b) * 2 + 1] = ss * (k4 * Jr_[a][b] - ik * j0r);
            }
        return;
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            const double Jr = Jr_[a][b], Ji = Ji_[a][b];
            const double ss = double(sgn[p * 3 + a] * sgn[q * 3 + b]);
            out[((a * 3 + b) * 256 + tid) * 2 + 0] = R(SPLIT ? ss * (-k4 * Ji) : ss * (-k4 * Ji + ik * j0i));
            out[((a * 3 + b) * 256 + tid) * 2 + 1] = R(SPLIT ? ss * (k4 * Jr) : ss * (k4 * Jr - ik * j0r));
        }
    if (SPLIT) {
        const int64_t t = tile_index(I, J, nT);
        VS[(t * 256 + tid) * 2 + 0] = R(ik * j0i);
        VS[(t * 256 + tid) * 2 + 1] = R(-ik * j0r);
    }
}

// ---------------------------------------------------------------------------
// 3. Assembly into the RWG matrix.
template <typename R>
__device__ inline void read_local(const R *__restrict__ LB, int64_t nT, int32_t p, int32_t a, int32_t q,
                                  int32_t b, R &re, R &im)
{
    if (p > q) {   // stored once, for p <= q, transposed
        int32_t t = p; p = q; q = t;
        t = a; a = b; b = t;
    }
    const R *src = LB + tile_index(p / TT, q / TT, nT) * (9 * 256 * 2) +
                   ((a * 3 + b) * 256 + (p % TT) * TT + (q % TT)) * 2;
    re = src[0];
    im = src[1];
}

// rwg4[m] = (c+, c-, slot in c+, slot in c-).  One block per stored tile
// (I, J), I <= J, of the packed symmetric matrix; 16 entries per thread.
template <typename R>
__global__ __launch_bounds__(256) void k_assemble(int64_t N, int64_t nT, int64_t nTz, const int4 *__restrict__ rwg4,
                                                  const R *__restrict__ LB, double2 *__restrict__ Z64,
                                                  float2 *__restrict__ Z32)
{
    int64_t I, J;
    tile_decode(blockIdx.x, nTz, I, J);
    const int64_t base = int64_t(blockIdx.x) * TB * TB;
#pragma unroll 4
    for (int q = 0; q < TB * TB / 256; ++q) {
        const int e = threadIdx.x + 256 * q;
        const int64_t m = I * TB + e / TB, n = J * TB + e % TB;
        R zr = 0, zi = 0;
        if (m < N && n < N) {
            const int4 em = rwg4[m], en = rwg4[n];
            R r1, i1, r2, i2, r3, i3, r4, i4;
            read_local(LB, nT, em.x, em.z, en.x, en.z, r1, i1);   // (+,+)
            read_local(LB, nT, em.y, em.w, en.y, en.w, r2, i2);   // (-,-)
            read_local(LB, nT, em.x, em.z, en.y, en.w, r3, i3);   // (+,-)
            read_local(LB, nT, em.y, em.w, en.x, en.z, r4, i4);   // (-,+)
            zr = (r1 + r2) + (r3 + r4);
            zi = (i1 + i2) + (i3 + i4);
        }
        if (Z64) Z64[base + e] = make_double2(double(zr), double(zi));
        if (Z32) Z32[base + e] = make_float2(float(zr), float(zi));
    }
}

// V' into packed F x F tiles (TB x TB, I <= J) from the per-pair values of the
// triangle tiles (p <= q; the other half by symmetry).
template <typename R>
__global__ __launch_bounds__(256) void k_assemble_v(int64_t F, int64_t nT, int64_t nTv, const R *__restrict__ VS,
                                                    double2 *__restrict__ V64, float2 *__restrict__ V32)
{
    int64_t I, J;
    tile_decode(blockIdx.x, nTv, I, J);
    const int64_t base = int64_t(blockIdx.x) * TB * TB;
#pragma unroll 4
    for (int q = 0; q < TB * TB / 256; ++q) {
        const int e = threadIdx.x + 256 * q;
        int64_t a = I * TB + e / TB, b = J * TB + e % TB;
        R vr = 0, vi = 0;
        if (a < F && b < F) {
            if (a > b) { const int64_t t = a; a = b; b = t; }
            const R *src = VS + (tile_index(a / TT, b / TT, nT) * 256 + (a % TT) * TT + (b % TT)) * 2;
            vr = src[0];
            vi = src[1];
        }
        if (V64) V64[base + e] = make_double2(double(vr), double(vi));
        if (V32) V32[base + e] = make_float2(float(vr), float(vi));
    }
}

// ---------------------------------------------------------------------------
// Plane-wave excitation:  e_m = sum_{p in m} (s_p/2) sum_i w_i (x_i - v_p).pol exp(-jk d.x_i)
__global__ __launch_bounds__(256) void k_rhs(int64_t N, int64_t R, const int4 *__restrict__ rwg4,
                                             const int8_t *__restrict__ sgn, const double *__restrict__ cent,
                                             const double *__restrict__ loc, const double *__restrict__ vfree,
                                             const double *__restrict__ dirs, const double *__restrict__ pols,
                                             double k, double2 *__restrict__ B)
{
    const int64_t m = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t r = blockIdx.y;
    if (m >= N || r >= R) return;
    const int4 e = rwg4[m];
    const double d[3] = { dirs[3 * r], dirs[3 * r + 1], dirs[3 * r + 2] };
    const double pl[3] = { pols[3 * r], pols[3 * r + 1], pols[3 * r + 2] };
    double br = 0.0, bi = 0.0;
    for (int side = 0; side < 2; ++side) {
        const int64_t t = side ? e.y : e.x;
        const int a = side ? e.w : e.z;
        const double s = 0.5 * double(sgn[t * 3 + a]);
        double tr = 0.0, ti = 0.0;
        for (int i = 0; i < NQ; ++i) {
            double x[3], dv = 0.0, ph = 0.0;
            for (int c = 0; c < 3; ++c) {
                x[c] = cent[t * 3 + c] + loc[(t * NQ + i) * 3 + c];
                dv += (loc[(t * NQ + i) * 3 + c] - vfree[t * 9 + a * 3 + c]) * pl[c];
                ph += d[c] * x[c];
            }
            double sn, cs;
            sincos(k * ph, &sn, &cs);
            tr += c_w[i] * dv * cs;
            ti -= c_w[i] * dv * sn;
        }
        br += s * tr;
        bi += s * ti;
    }
    B[r * N + m] = make_double2(br, bi);
}

// Radiation vector F(o) = int j(y) exp(jk o.y) dS = sum_t sum_i w_i J_t(y_i) exp(jk o.y_i),
// J_t(y) = sum_a x_{m(t,a)} s_a (y - v_a)/2.  One block per (vector, direction).
// RCS: write the bistatic RCS (k^2 / (4 pi)) |r x F|^2 of direction r (unit)
// instead of F: the part of F transverse to r, squared.
template <bool RCS>
__global__ __launch_bounds__(256) void k_farfield(int64_t F, int64_t N, int64_t M,
                                                  const int32_t *__restrict__ slot_m,
                                                  const int8_t *__restrict__ sgn, const double *__restrict__ cent,
                                                  const double *__restrict__ loc, const double *__restrict__ vfree,
                                                  const double *__restrict__ obs, double k,
                                                  const double2 *__restrict__ X, void *__restrict__ outv)
{
    const int64_t mo = blockIdx.x, r = blockIdx.y;
    const double o[3] = { obs[3 * mo], obs[3 * mo + 1], obs[3 * mo + 2] };
    const double2 *x = X + r * N;
    double acc[6] = { 0, 0, 0, 0, 0, 0 };
    for (int64_t t = threadIdx.x; t < F; t += blockDim.x) {
        double2 xa[3];
        double sa[3];
        for (int a = 0; a < 3; ++a) {
            xa[a] = x[slot_m[t * 3 + a]];
            sa[a] = 0.5 * double(sgn[t * 3 + a]);
        }
        for (int i = 0; i < NQ; ++i) {
            double ph = 0.0;
            for (int c = 0; c < 3; ++c) ph += o[c] * (cent[t * 3 + c] + loc[(t * NQ + i) * 3 + c]);
            double sn, cs;
            sincos(k * ph, &sn, &cs);
            for (int c = 0; c < 3; ++c) {
                double jr = 0.0, ji = 0.0;
                for (int a = 0; a < 3; ++a) {
                    const double dv = sa[a] * (loc[(t * NQ + i) * 3 + c] - vfree[t * 9 + a * 3 + c]);
                    jr += xa[a].x * dv;
                    ji += xa[a].y * dv;
                }
                acc[2 * c] += c_w[i] * (jr * cs - ji * sn);
                acc[2 * c + 1] += c_w[i] * (jr * sn + ji * cs);
            }
        }
    }
    __shared__ double red[6][256];
    for (int c = 0; c < 6; ++c) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (int(threadIdx.x) < s)
            for (int c = 0; c < 6; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
        __syncthreads();
    }
    if (RCS) {
        if (threadIdx.x == 0) {
            // r . F, then |F - (r . F) r|^2
            double dr = 0.0, di = 0.0;
            for (int c = 0; c < 3; ++c) {
                dr += o[c] * red[2 * c][0];
                di += o[c] * red[2 * c + 1][0];
            }
            double t2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                const double tr = red[2 * c][0] - dr * o[c], ti = red[2 * c + 1][0] - di * o[c];
                t2 += tr * tr + ti * ti;
            }
            static_cast<double *>(outv)[r * M + mo] = k * k / (4.0 * M_PI) * t2;
        }
    } else if (threadIdx.x < 3) {
        static_cast<double2 *>(outv)[(r * M + mo) * 3 + threadIdx.x] =
            make_double2(red[2 * threadIdx.x][0], red[2 * threadIdx.x + 1][0]);
    }
}

template <typename T>
T *dev_alloc(size_t n)
{
    void *p = nullptr;
    BIE_HIP(hipMalloc(&p, n * sizeof(T)));
    return static_cast<T *>(p);
}

}  // namespace

// Weights of the triangle rule (relative to the area), for other kernels that
// integrate over the same quadrature points.
// The local 3 x 3 blocks L(p, a, q, b) of the flagged pairs (p <= q) of the
// mesh's list, pair after pair (18 doubles each: re, im of (a, b) row-major),
// with the fill's singular treatment.
void singular_blocks(const bie_op *op, const int32_t *pairs, int64_t npairs, double *out, hipStream_t s)
{
    if (npairs == 0) return;
    const TriDev &D = op->tri;
    hipLaunchKernelGGL((k_pairs_singular<double, false>), dim3(unsigned((npairs + 127) / 128)), dim3(128), 0, s, npairs,
                       int64_t(0), pairs, D.cent, D.loc, D.vfree, D.verts, D.area, D.sgn, op->k, (double *)nullptr,
                       (double *)nullptr, out);
    BIE_HIP(hipGetLastError());
}

void quad_weights(double *w)
{
    const Rule rule = make_rule();
    for (int i = 0; i < NQ; ++i) w[i] = rule.w[i];
}

// Per-triangle tables on the device.  Quadrature points and free vertices
// relative to the triangle centroid (keeps FP32 local arithmetic accurate).
void upload_triangles(bie_op *op, hipStream_t s)
{
    const Mesh &M = op->mesh;
    const int64_t F = M.F;
    const Rule rule = make_rule();
    BIE_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_w), rule.w, sizeof(rule.w)));
    std::vector<double> loc(F * NQ * 3), vf(F * 9), vt(F * 9);
    for (int64_t t = 0; t < F; ++t) {
        const double *v[3] = { &M.V[3 * M.T[3 * t]], &M.V[3 * M.T[3 * t + 1]], &M.V[3 * M.T[3 * t + 2]] };
        const double *c = &M.cent[3 * t];
        for (int i = 0; i < NQ; ++i)
            for (int d = 0; d < 3; ++d) {
                const double x = rule.bary[i][0] * v[0][d] + rule.bary[i][1] * v[1][d] + rule.bary[i][2] * v[2][d];
                loc[(t * NQ + i) * 3 + d] = x - c[d];
            }
        for (int a = 0; a < 3; ++a)
            for (int d = 0; d < 3; ++d) {
                vf[t * 9 + a * 3 + d] = v[a][d] - c[d];
                vt[t * 9 + a * 3 + d] = v[a][d];
            }
    }
    TriDev &D = op->tri;
    D.cent = dev_alloc<double>(F * 3);
    D.loc = dev_alloc<double>(F * NQ * 3);
    D.vfree = dev_alloc<double>(F * 9);
    D.verts = dev_alloc<double>(F * 9);
    D.area = dev_alloc<double>(F);
    D.sgn = dev_alloc<int8_t>(F * 3);
    D.slot_m = dev_alloc<int32_t>(F * 3);
    D.edges = dev_alloc<int32_t>(M.N * 4);
    BIE_HIP(hipMemcpy(D.cent, M.cent.data(), F * 3 * sizeof(double), hipMemcpyHostToDevice));
    BIE_HIP(hipMemcpy(D.loc, loc.data(), loc.size() * sizeof(double), hipMemcpyHostToDevice));
    BIE_HIP(hipMemcpy(D.vfree, vf.data(), vf.size() * sizeof(double), hipMemcpyHostToDevice));
    BIE_HIP(hipMemcpy(D.verts, vt.data(), vt.size() * sizeof(double), hipMemcpyHostToDevice));
    BIE_HIP(hipMemcpy(D.area, M.area.data(), F * sizeof(double), hipMemcpyHostToDevice));
    BIE_HIP(hipMemcpy(D.sgn, M.slot_s.data(), F * 3, hipMemcpyHostToDevice));
    BIE_HIP(hipMemcpy(D.slot_m, M.slot_m.data(), F * 3 * sizeof(int32_t), hipMemcpyHostToDevice));
    // rwg4: (c+, c-, slot of m in c+, slot of m in c-)
    std::vector<int32_t> r4(M.N * 4);
    for (int64_t m = 0; m < M.N; ++m) {
        const int32_t tp = M.edges[4 * m + 2], tm = M.edges[4 * m + 3];
        int sp = -1, sm = -1;
        for (int a = 0; a < 3; ++a) {
            if (M.slot_m[3 * tp + a] == m) sp = a;
            if (M.slot_m[3 * tm + a] == m) sm = a;
        }
        r4[4 * m + 0] = tp; r4[4 * m + 1] = tm; r4[4 * m + 2] = sp; r4[4 * m + 3] = sm;
    }
    BIE_HIP(hipMemcpy(D.edges, r4.data(), r4.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    (void)s;
}

template <typename R, bool SPLIT>
static void fill_launch(bie_op *op, int64_t nT, int64_t ntiles, const int32_t *pairs, int64_t npairs, void *LB,
                        void *VS, bool want64, bool want32, hipStream_t s)
{
    const Mesh &M = op->mesh;
    const TriDev &D = op->tri;
    // measurement records: 6 regular pairs (columns = triangle pairs p <= q), 7
    // flagged pairs, 8 assembly (columns = unknowns)
    const int rec_reg = sizeof(R) == 8 ? 6 : 9;
    prof_begin(rec_reg, s, M.F * (M.F + 1) / 2);
    hipLaunchKernelGGL((k_pairs_regular<R, SPLIT>), dim3(unsigned(ntiles)), dim3(256), 0, s, M.F, nT, ntiles, D.cent,
                       D.loc, D.vfree, D.sgn, op->k, (R *)LB, (R *)VS);
    prof_end(rec_reg, s);
    prof_begin(7, s, npairs);
    if (npairs)
        hipLaunchKernelGGL((k_pairs_singular<R, SPLIT>), dim3(unsigned((npairs + 127) / 128)), dim3(128), 0, s, npairs,
                           nT, pairs, D.cent, D.loc, D.vfree, D.verts, D.area, D.sgn, op->k, (R *)LB, (R *)VS);
    prof_end(7, s);
    prof_begin(8, s, M.N);
    hipLaunchKernelGGL(k_assemble<R>, dim3(unsigned(op->pk.ntiles)), dim3(256), 0, s, M.N, nT, op->pk.nT,
                       (const int4 *)D.edges, (const R *)LB, want64 ? (double2 *)op->Z64 : nullptr,
                       want32 ? (float2 *)op->Z32 : nullptr);
    prof_end(8, s);
    if (SPLIT)
        hipLaunchKernelGGL(k_assemble_v<R>, dim3(unsigned(op->pkv.ntiles)), dim3(256), 0, s, M.F, nT, op->pkv.nT,
                           (const R *)VS, want64 ? (double2 *)op->V64 : nullptr, want32 ? (float2 *)op->V32 : nullptr);
}

// The matrix (or, for a star-split operator, T_A' and V') into the packed
// arrays the operator holds.
void fill_matrix(bie_op *op, bool fp64_regular, bool want64, bool want32, hipStream_t s)
{
    const Mesh &M = op->mesh;
    const int64_t F = M.F;
    const int64_t nT = (F + TT - 1) / TT;
    const int64_t ntiles = nT * (nT + 1) / 2;
    const size_t elem = fp64_regular ? sizeof(double) : sizeof(float);
    void *LB = nullptr, *VS = nullptr;
    int32_t *pairs = nullptr;
    const int64_t npairs = int64_t(M.near.size() / 2);
    const bool pooled = setup_pool_active();   // inside a preconditioner setup: kept scratch
    try {
        const size_t lb_bytes = size_t(ntiles) * 9 * 256 * 2 * elem;
        if (pooled) LB = setup_pool_get(0, lb_bytes);
        else BIE_HIP(hipMalloc(&LB, lb_bytes));
        if (op->star) BIE_HIP(hipMalloc(&VS, size_t(ntiles) * 256 * 2 * elem));
        if (npairs) {
            BIE_HIP(hipMalloc(&pairs, M.near.size() * sizeof(int32_t)));
            BIE_HIP(hipMemcpyAsync(pairs, M.near.data(), M.near.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        }
        if (fp64_regular) {
            if (op->star) fill_launch<double, true>(op, nT, ntiles, pairs, npairs, LB, VS, want64, want32, s);
            else fill_launch<double, false>(op, nT, ntiles, pairs, npairs, LB, VS, want64, want32, s);
        } else {
            if (op->star) fill_launch<float, true>(op, nT, ntiles, pairs, npairs, LB, VS, want64, want32, s);
            else fill_launch<float, false>(op, nT, ntiles, pairs, npairs, LB, VS, want64, want32, s);
        }
        BIE_HIP(hipGetLastError());
        BIE_HIP(hipStreamSynchronize(s));
    } catch (...) {
        if (LB && !pooled) hipFree(LB);
        if (VS) hipFree(VS);
        if (pairs) hipFree(pairs);
        throw;
    }
    if (!pooled) hipFree(LB);
    if (VS) hipFree(VS);
    if (pairs) hipFree(pairs);
}

void rhs_planewave(const bie_op *op, const double *dirs, const double *pols, int64_t R, void *B, hipStream_t s)
{
    const int64_t N = op->mesh.N;
    double *dd = nullptr;
    BIE_HIP(hipMalloc(&dd, 6 * R * sizeof(double)));
    BIE_HIP(hipMemcpy(dd, dirs, 3 * R * sizeof(double), hipMemcpyHostToDevice));
    BIE_HIP(hipMemcpy(dd + 3 * R, pols, 3 * R * sizeof(double), hipMemcpyHostToDevice));
    const TriDev &D = op->tri;
    hipLaunchKernelGGL(k_rhs, dim3(unsigned((N + 255) / 256), unsigned(R)), dim3(256), 0, s, N, R,
                       (const int4 *)D.edges, D.sgn, D.cent, D.loc, D.vfree, dd, dd + 3 * R, op->k, (double2 *)B);
    BIE_HIP(hipGetLastError());
    BIE_HIP(hipStreamSynchronize(s));
    hipFree(dd);
}

void farfield(const bie_op *op, const void *X, int64_t R, const double *obs, int64_t M, void *out, bool rcs,
              hipStream_t s)
{
    double *dobs = nullptr;
    BIE_HIP(hipMalloc(&dobs, 3 * M * sizeof(double)));
    BIE_HIP(hipMemcpy(dobs, obs, 3 * M * sizeof(double), hipMemcpyHostToDevice));
    const TriDev &D = op->tri;
    if (rcs)
        hipLaunchKernelGGL(k_farfield<true>, dim3(unsigned(M), unsigned(R)), dim3(256), 0, s, op->mesh.F, op->mesh.N,
                           M, D.slot_m, D.sgn, D.cent, D.loc, D.vfree, dobs, op->k, (const double2 *)X, out);
    else
        hipLaunchKernelGGL(k_farfield<false>, dim3(unsigned(M), unsigned(R)), dim3(256), 0, s, op->mesh.F, op->mesh.N,
                           M, D.slot_m, D.sgn, D.cent, D.loc, D.vfree, dobs, op->k, (const double2 *)X, out);
    const hipError_t e = hipGetLastError();
    const hipError_t e2 = hipStreamSynchronize(s);
    (void)hipFree(dobs);
    BIE_HIP(e);
    BIE_HIP(e2);
}

}  // namespace bie
