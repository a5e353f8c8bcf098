/* Plain FP64 C version of the oracle's EFIE fill: TEST INFRASTRUCTURE ONLY.
 *
 * Same definition as oracle/efie.py (Sec. II of the paper: eq:matTA,
 * eq:matTPhi with RWG functions without edge-length normalisation), written
 * as direct loops over triangle pairs and quadrature points so that full
 * matrices of a few thousand unknowns can be built on the host in seconds.
 *
 *   Z_mn += s_p s_q sum_ij w_i w_j [ (jk/4)(x_i - v_p).(y_j - v_q) + 1/(jk) ] g(|x_i - y_j|)
 *
 * Flagged pairs use g = g_r + 1/(4 pi R) with the closed-form inner integral
 * of 1/R and (y - x)/R over the source triangle and the mean of both
 * orderings (see oracle/potentials.py for the formulas).
 *
 * Parallel over triangles of one colour at a time: triangles of one colour
 * share no RWG function, so each row of Z receives at most one contribution
 * per colour and the result does not depend on the thread count.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

typedef double complex cplx;
static const double FOUR_PI = 12.566370614359172953850573533118;

static inline double dot3(const double *a, const double *b) { return a[0]*b[0] + a[1]*b[1] + a[2]*b[2]; }
static inline void sub3(const double *a, const double *b, double *c) { c[0]=a[0]-b[0]; c[1]=a[1]-b[1]; c[2]=a[2]-b[2]; }
static inline void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1]*b[2] - a[2]*b[1]; c[1] = a[2]*b[0] - a[0]*b[2]; c[2] = a[0]*b[1] - a[1]*b[0];
}

/* K0 = int_tri 1/|y-x| dS, K1 = int_tri (y-x)/|y-x| dS for a CCW triangle (A,B,C). */
static void k0k1(const double *x, const double *A, const double *B, const double *C, double *K0, double *K1)
{
    double e1[3], e2[3], n[3];
    sub3(B, A, e1); sub3(C, A, e2); cross3(e1, e2, n);
    double nn = sqrt(dot3(n, n));
    n[0] /= nn; n[1] /= nn; n[2] /= nn;
    double xa[3]; sub3(x, A, xa);
    double h = dot3(xa, n), ah = fabs(h);
    double rho[3] = { x[0] - h*n[0], x[1] - h*n[1], x[2] - h*n[2] };
    const double *P[3] = { A, B, C }, *Q[3] = { B, C, A };
    double k0 = 0.0, kp[3] = { 0, 0, 0 };
    for (int e = 0; e < 3; ++e) {
        double L[3]; sub3(Q[e], P[e], L);
        double ll = sqrt(dot3(L, L));
        double l[3] = { L[0]/ll, L[1]/ll, L[2]/ll };
        double u[3]; cross3(l, n, u);
        double qr[3], pr[3]; sub3(Q[e], rho, qr); sub3(P[e], rho, pr);
        double lp = dot3(qr, l), lm = dot3(pr, l), P0 = dot3(pr, u);
        double R0s = P0*P0 + h*h;
        double Rp = sqrt(R0s + lp*lp), Rm = sqrt(R0s + lm*lm);
        double f = 0.0;
        if (R0s > 0.0) f = (lp + lm < 0.0) ? log((Rm - lm)/(Rp - lp)) : log((Rp + lp)/(Rm + lm));
        double beta = 0.0;
        if (ah > 0.0) beta = atan2(P0*lp, R0s + ah*Rp) - atan2(P0*lm, R0s + ah*Rm);
        k0 += (R0s > 0.0 ? P0*f : 0.0) - ah*beta;
        double c = 0.5*((R0s > 0.0 ? R0s*f : 0.0) + lp*Rp - lm*Rm);
        kp[0] += c*u[0]; kp[1] += c*u[1]; kp[2] += c*u[2];
    }
    *K0 = k0;
    K1[0] = kp[0] - h*n[0]*k0; K1[1] = kp[1] - h*n[1]*k0; K1[2] = kp[2] - h*n[2]*k0;
}

/* J[a][b] = int_p int_q (x - v_a).(y - v_b) g / (A_p A_q), J0 = int int g /(A_p A_q). */
static void pair_block(int nq, const double *w, const double *Xp, const double *Xq,
                       const double *vp, const double *vq, const double *trip, const double *triq,
                       double Ap, double Aq, double k, int singular, cplx J[3][3], cplx *J0)
{
    cplx Jl[3][3] = { { 0 } }, j0 = 0;
    for (int i = 0; i < nq; ++i) {
        for (int j = 0; j < nq; ++j) {
            double d[3]; sub3(Xp + 3*i, Xq + 3*j, d);
            double R = sqrt(dot3(d, d));
            cplx g;
            if (!singular) {
                g = cexp(-I*k*R) / (FOUR_PI*R);
            } else if (R > 0.0) {
                double s = sin(0.5*k*R);
                g = (-2.0*s*s - I*sin(k*R)) / (FOUR_PI*R);
            } else {
                g = -I*k/FOUR_PI;
            }
            g *= w[i]*w[j];
            j0 += g;
            for (int a = 0; a < 3; ++a) {
                double da[3]; sub3(Xp + 3*i, vp + 3*a, da);
                for (int b = 0; b < 3; ++b) {
                    double db[3]; sub3(Xq + 3*j, vq + 3*b, db);
                    Jl[a][b] += g*dot3(da, db);
                }
            }
        }
    }
    if (singular) {
        /* p outer, closed-form inner over q; then q outer, inner over p; mean. */
        cplx Js[3][3] = { { 0 } }; double j0s = 0.0;
        for (int i = 0; i < nq; ++i) {
            double K0, K1[3];
            k0k1(Xp + 3*i, triq, triq + 3, triq + 6, &K0, K1);
            j0s += w[i]*K0/(FOUR_PI*Aq);
            for (int a = 0; a < 3; ++a) {
                double da[3]; sub3(Xp + 3*i, vp + 3*a, da);
                for (int b = 0; b < 3; ++b) {
                    double xv[3]; sub3(Xp + 3*i, vq + 3*b, xv);
                    double Iv[3] = { K1[0] + xv[0]*K0, K1[1] + xv[1]*K0, K1[2] + xv[2]*K0 };
                    Js[a][b] += w[i]*dot3(da, Iv)/(FOUR_PI*Aq);
                }
            }
        }
        for (int j = 0; j < nq; ++j) {
            double K0, K1[3];
            k0k1(Xq + 3*j, trip, trip + 3, trip + 6, &K0, K1);
            j0s += w[j]*K0/(FOUR_PI*Ap);
            for (int b = 0; b < 3; ++b) {
                double db[3]; sub3(Xq + 3*j, vq + 3*b, db);
                for (int a = 0; a < 3; ++a) {
                    double yv[3]; sub3(Xq + 3*j, vp + 3*a, yv);
                    double Iv[3] = { K1[0] + yv[0]*K0, K1[1] + yv[1]*K0, K1[2] + yv[2]*K0 };
                    Js[a][b] += w[j]*dot3(db, Iv)/(FOUR_PI*Ap);
                }
            }
        }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) Jl[a][b] += 0.5*Js[a][b];
        j0 += 0.5*j0s;
    }
    memcpy(J, Jl, sizeof(Jl));
    *J0 = j0;
}

/* Full matrix.  X: (F,nq,3) quadrature points, Vf: (F,3,3) free vertex of slot a,
 * m_of/s_of: (F,3) RWG index and sign of slot a, flags: (F,F) bytes,
 * colour_ptr/colour_tris: CSR of triangles per colour, Z: (N,N) complex128 (zeroed). */
void oracle_fill(int64_t F, int64_t N, int nq, const double *w, const double *X, const double *Vf,
                 const double *tri, const double *area, const int64_t *m_of, const double *s_of,
                 const uint8_t *flags, double k, int64_t ncol, const int64_t *colour_ptr,
                 const int64_t *colour_tris, double *Zri)
{
    cplx *Z = (cplx *)Zri;
    const cplx jk = I*k;
    for (int64_t c = 0; c < ncol; ++c) {
        #pragma omp parallel for schedule(dynamic, 1)
        for (int64_t it = colour_ptr[c]; it < colour_ptr[c + 1]; ++it) {
            int64_t p = colour_tris[it];
            for (int64_t q = 0; q < F; ++q) {
                cplx J[3][3], J0;
                pair_block(nq, w, X + 3*nq*p, X + 3*nq*q, Vf + 9*p, Vf + 9*q, tri + 9*p, tri + 9*q,
                           area[p], area[q], k, flags[p*F + q] != 0, J, &J0);
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b)
                        Z[m_of[3*p + a]*N + m_of[3*q + b]] +=
                            s_of[3*p + a]*s_of[3*q + b]*(jk*0.25*J[a][b] + J0/jk);
            }
        }
    }
}

/* Closed-form K0, K1 at P points (for tests of this file against oracle/potentials.py). */
void oracle_k0k1(int64_t P, const double *x, const double *tri, double *K0, double *K1)
{
    for (int64_t i = 0; i < P; ++i) k0k1(x + 3*i, tri, tri + 3, tri + 6, K0 + i, K1 + 3*i);
}
