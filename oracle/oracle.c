/*
 * oracle.c -- plain, slow, FP64 CPU reference for the tile micromagnetics
 * hot path of Bjork, Poulsen, Nielsen & Insinga, "MagTense: a micromagnetic
 * framework using the analytical demagnetization tensor", JMMM 535 (2021).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; it shares no source, header, table or helper with the HIP
 * path.  Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark use it.
 *
 * Everything is double precision and SI units.  Tiles are axis-aligned
 * rectangular cuboids given by centre c[3] and full edge lengths s[3]
 * (paper Sec. 3: the domain is split into N adjacent, uniformly magnetised
 * tiles; m is a 3N vector).  Tensor components are ordered
 * (xx, xy, xz, yy, yz, zz).
 *
 * OpenMP is used only to split independent outer loops (pairs, rows); the
 * arithmetic inside every loop body is the plain definition.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846
#define ORC_MU0 (4.0e-7 * ORC_PI) /* vacuum permeability [H/m] */

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads the outer loops use from now on (timing runs only). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Analytical demagnetisation tensor of a uniformly magnetised cuboid        */
/* (paper Sec. 3; the cuboid formula itself is only cited there, so it is    */
/* derived here).                                                            */
/*                                                                           */
/* psi(r) = (1/4pi) int_box dV'/|r-r'|,  N(r) = -grad grad psi(r),           */
/* so the field of the tile is H = -N M (trace N = 1 inside, 0 outside).     */
/* With U_i = x - x_i (x_1 = c-h lower face, x_2 = c+h upper face), V_j, W_k */
/* alike in y, z, R = sqrt(U^2+V^2+W^2), s_1 = +1, s_2 = -1:                 */
/*   N_xx =  1/(4pi) sum_ijk s_i s_j s_k atan(V_j W_k / (U_i R))             */
/*   N_xy = -1/(4pi) sum_ij  s_i s_j  ln[(W_1+R_ij1)/(W_2+R_ij2)]            */
/* and cyclically for the other components.  An atan term with U_i == 0 is   */
/* taken as 0: the point lies in the plane of that face but outside it, and  */
/* the four (j,k) terms of that face cancel exactly.                         */
/* ------------------------------------------------------------------------ */

/* sum over the 8 corners of s_i s_j s_k atan(b c /(a R)), where a runs over
 * the axis that appears in the denominator. */
static double diag_sum(const double a[2], const double b[2], const double c[2]) {
    double acc = 0.0;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int k = 0; k < 2; ++k) {
                double sgn = ((i + j + k) & 1) ? -1.0 : 1.0;
                if (a[i] == 0.0) continue;
                double R = sqrt(a[i] * a[i] + b[j] * b[j] + c[k] * c[k]);
                acc += sgn * atan((b[j] * c[k]) / (a[i] * R));
            }
    return acc;
}

/* ln[(w1 + R1)/(w2 + R2)] for rho^2 = p^2 + q^2, w1 = w2 + (edge) > w2,
 * written so that no term cancels:
 *   both w >= 0 : log1p(d), d = (w1-w2)(1 + (w1+w2)/(R1+R2)) / (w2+R2)
 *   both w <= 0 : (w+R) = rho^2/(R-w), so the ratio is (R2-w2)/(R1-w1)
 *                 = 1 + (w1-w2)(1 - (w1+w2)/(R1+R2)) / (R1-w1)
 *   w1 > 0 > w2 : ln[(w1+R1)(R2-w2)/rho^2]  (rho > 0: the point is not on
 *                 an edge of the tile) */
static double log_ratio(double rho2, double w1, double w2) {
    double R1 = sqrt(rho2 + w1 * w1);
    double R2 = sqrt(rho2 + w2 * w2);
    double e = w1 - w2;
    if (w2 >= 0.0) {
        double d = e * (1.0 + (w1 + w2) / (R1 + R2)) / (w2 + R2);
        return log1p(d);
    } else if (w1 <= 0.0) {
        double d = e * (1.0 - (w1 + w2) / (R1 + R2)) / (R1 - w1);
        return log1p(d);
    } else {
        return log((w1 + R1) * (R2 - w2) / rho2);
    }
}

/* sum_ij s_i s_j ln[(w_1 + R_ij1)/(w_2 + R_ij2)] */
static double offdiag_sum(const double p[2], const double q[2], const double w[2]) {
    double acc = 0.0;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            double sgn = ((i + j) & 1) ? -1.0 : 1.0;
            acc += sgn * log_ratio(p[i] * p[i] + q[j] * q[j], w[0], w[1]);
        }
    return acc;
}

/* Tensor of the cuboid (centre c, full edges s) evaluated at point r.
 * out = (xx, xy, xz, yy, yz, zz). */
void orc_prism_tensor(const double r[3], const double c[3], const double s[3], double out[6]) {
    double U[2], V[2], W[2];
    double dx = r[0] - c[0], dy = r[1] - c[1], dz = r[2] - c[2];
    double hx = 0.5 * s[0], hy = 0.5 * s[1], hz = 0.5 * s[2];
    U[0] = dx + hx; U[1] = dx - hx; /* x - (c-h), x - (c+h) */
    V[0] = dy + hy; V[1] = dy - hy;
    W[0] = dz + hz; W[1] = dz - hz;
    const double k = 1.0 / (4.0 * ORC_PI);
    out[0] = k * diag_sum(U, V, W);      /* xx */
    out[3] = k * diag_sum(V, W, U);      /* yy */
    out[5] = k * diag_sum(W, U, V);      /* zz */
    out[1] = -k * offdiag_sum(U, V, W);  /* xy: ln(W+R) */
    out[2] = -k * offdiag_sum(U, W, V);  /* xz: ln(V+R) */
    out[4] = -k * offdiag_sum(V, W, U);  /* yz: ln(U+R) */
}

/* Dense demag operator (paper Sec. 3 and Sec. 3.1): block (a,b) is the
 * tensor of tile b evaluated at the centre of tile a; T is [3n][3n]
 * row-major, T[3a+i][3b+j]. */
void orc_assemble(int64_t n, const double* centers, const double* sizes, double* T) {
    int64_t ld = 3 * n;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t a = 0; a < n; ++a) {
        for (int64_t b = 0; b < n; ++b) {
            double t6[6];
            orc_prism_tensor(centers + 3 * a, centers + 3 * b, sizes + 3 * b, t6);
            double* blk = T + (3 * a) * ld + 3 * b;
            blk[0] = t6[0]; blk[1] = t6[1]; blk[2] = t6[2];
            blk[ld + 0] = t6[1]; blk[ld + 1] = t6[3]; blk[ld + 2] = t6[4];
            blk[2 * ld + 0] = t6[2]; blk[2 * ld + 1] = t6[4]; blk[2 * ld + 2] = t6[5];
        }
    }
}

/* Demag field H_d,a = -sum_b N^{ab} Ms_b m_b  [A/m]  (paper Sec. 2.3 and the
 * affine operator of Sec. 3.1), from a stored dense operator. */
void orc_demag(int64_t n, const double* T, const double* Ms, const double* m, double* Hd) {
    int64_t ld = 3 * n;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < 3 * n; ++r) {
        double acc = 0.0;
        const double* row = T + r * ld;
        for (int64_t col = 0; col < 3 * n; ++col) acc += row[col] * Ms[col / 3] * m[col];
        Hd[r] = -acc;
    }
}

/* Thresholded operator (paper Sec. 4.3.1): of the nonzero entries of the
 * dense operator, the fraction `frac` with the smallest magnitude is set to
 * zero, and what is left is kept as a sparse matrix.  Readings of that
 * passage: the ranking is over the magnitudes that float storage holds (each
 * FP64 entry rounded to float32) and counts all 9 entries of every 3x3 block,
 * self blocks included; an entry counts as nonzero when its magnitude exceeds
 * ORC_ZERO_FLOOR, the absolute accuracy of the float64 assembly (entries that
 * vanish by symmetry come out as rounding noise of ~1e-17 or as exact zeros
 * depending on the evaluation order; physical entries on meshes below 100 um
 * are far larger); with K nonzero entries the cut is the r-th smallest
 * magnitude, r = ceil(frac K); every entry whose magnitude is at most the cut
 * is removed (ties at the cut go too); entries of self blocks (a == b) are
 * never removed.  frac = 0 removes nothing.  Works in place on T [3n][3n] and
 * returns the cut (-1 when nothing is removed). */
#define ORC_ZERO_FLOOR 1e-14
static int orc_cmp_double(const void* x, const void* y) {
    double a = *(const double*)x, b = *(const double*)y;
    return (a > b) - (a < b);
}

double orc_threshold(int64_t n, double* T, double frac) {
    int64_t ld = 3 * n, K = 0;
    double* v = (double*)malloc(sizeof(double) * (size_t)(ld * ld));
    const double floor32 = (double)(float)ORC_ZERO_FLOOR;
    for (int64_t i = 0; i < ld * ld; ++i) {
        double mag = fabs((double)(float)T[i]);
        if (mag > floor32) v[K++] = mag;
    }
    int64_t r = (int64_t)ceil(frac * (double)K);
    if (r > K) r = K;
    double cut = -1.0;
    if (r > 0) {
        qsort(v, (size_t)K, sizeof(double), orc_cmp_double);
        cut = v[r - 1];
        for (int64_t row = 0; row < ld; ++row)
            for (int64_t col = 0; col < ld; ++col) {
                if (row / 3 == col / 3) continue;
                double* e = T + row * ld + col;
                if (fabs((double)(float)*e) <= cut) *e = 0.0;
            }
    }
    free(v);
    return cut;
}

/* Same field at selected target tiles only, evaluating the tensor on the fly
 * (for meshes whose dense operator does not fit in host memory). */
void orc_demag_rows(int64_t n, const double* centers, const double* sizes, const double* Ms,
                    const double* m, int64_t nrows, const int64_t* rows, double* Hd) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nrows; ++q) {
        int64_t a = rows[q];
        double h[3] = {0.0, 0.0, 0.0};
        for (int64_t b = 0; b < n; ++b) {
            double t6[6];
            orc_prism_tensor(centers + 3 * a, centers + 3 * b, sizes + 3 * b, t6);
            double mx = Ms[b] * m[3 * b], my = Ms[b] * m[3 * b + 1], mz = Ms[b] * m[3 * b + 2];
            h[0] += t6[0] * mx + t6[1] * my + t6[2] * mz;
            h[1] += t6[1] * mx + t6[3] * my + t6[4] * mz;
            h[2] += t6[2] * mx + t6[4] * my + t6[5] * mz;
        }
        Hd[3 * q] = -h[0]; Hd[3 * q + 1] = -h[1]; Hd[3 * q + 2] = -h[2];
    }
}

/* ------------------------------------------------------------------------ */
/* Exchange (paper Sec. 2.3 exchange field and Sec. 3 finite differences;    */
/* Neumann boundary from Brown's second equation, Sec. 2.1).                  */
/* A face pair (a,b) is two tiles that touch along one axis with a shared    */
/* face patch of positive area.  The two-point flux form                      */
/*   H_ex,a = 2A/(mu0 Ms_a V_a) sum_b S_ab (m_b - m_a)/d_ab                   */
/* equals the 3-point Laplacian stencil on a uniform grid; a missing         */
/* neighbour contributes nothing (zero normal derivative).                    */
/* ------------------------------------------------------------------------ */

/* Brute force over all ordered pairs.  Returns the number of ordered face
 * pairs; fills at most cap of them. */
int64_t orc_faces(int64_t n, const double* centers, const double* sizes, int64_t cap,
                  int64_t* fa, int64_t* fb, double* area, double* dist) {
    int64_t cnt = 0;
    for (int64_t a = 0; a < n; ++a) {
        for (int64_t b = 0; b < n; ++b) {
            if (a == b) continue;
            for (int d = 0; d < 3; ++d) {
                int e1 = (d + 1) % 3, e2 = (d + 2) % 3;
                double gap = fabs(centers[3 * a + d] - centers[3 * b + d]) -
                             0.5 * (sizes[3 * a + d] + sizes[3 * b + d]);
                double smin = fmin(sizes[3 * a + d], sizes[3 * b + d]);
                if (fabs(gap) > 1e-9 * smin) continue;
                double o1 = fmin(centers[3 * a + e1] + 0.5 * sizes[3 * a + e1],
                                 centers[3 * b + e1] + 0.5 * sizes[3 * b + e1]) -
                            fmax(centers[3 * a + e1] - 0.5 * sizes[3 * a + e1],
                                 centers[3 * b + e1] - 0.5 * sizes[3 * b + e1]);
                double o2 = fmin(centers[3 * a + e2] + 0.5 * sizes[3 * a + e2],
                                 centers[3 * b + e2] + 0.5 * sizes[3 * b + e2]) -
                            fmax(centers[3 * a + e2] - 0.5 * sizes[3 * a + e2],
                                 centers[3 * b + e2] - 0.5 * sizes[3 * b + e2]);
                double tol1 = 1e-9 * fmin(sizes[3 * a + e1], sizes[3 * b + e1]);
                double tol2 = 1e-9 * fmin(sizes[3 * a + e2], sizes[3 * b + e2]);
                if (o1 <= tol1 || o2 <= tol2) continue;
                if (cnt < cap) {
                    fa[cnt] = a; fb[cnt] = b;
                    area[cnt] = o1 * o2;
                    dist[cnt] = fabs(centers[3 * a + d] - centers[3 * b + d]);
                }
                ++cnt;
            }
        }
    }
    return cnt;
}

/* Everything the effective field needs besides m and the applied field. */
typedef struct {
    int64_t n;
    const double* T;       /* [3n][3n] demag operator */
    const double* vol;     /* [n] tile volumes */
    const double* Ms;      /* [n] saturation magnetisation [A/m] */
    double A;              /* exchange constant [J/m] */
    const double* Ku;      /* [n] uniaxial anisotropy constant [J/m^3] */
    const double* easy;    /* [n][3] unit easy axes */
    int64_t nfaces;        /* ordered face pairs */
    const int64_t* fa;
    const int64_t* fb;
    const double* area;
    const double* dist;
    double c1, c2;         /* LL coefficients: precession, damping */
} orc_problem;

/* H_eff = H_d + H_ex + H_anis + H_a (paper Sec. 2.3; Sec. 3.1 affine form). */
void orc_heff(const orc_problem* P, const double* m, const double Ha[3], double* H) {
    int64_t n = P->n;
    orc_demag(n, P->T, P->Ms, m, H);
    /* exchange */
    for (int64_t f = 0; f < P->nfaces; ++f) {
        int64_t a = P->fa[f], b = P->fb[f];
        double coef = 2.0 * P->A / (ORC_MU0 * P->Ms[a] * P->vol[a]) * P->area[f] / P->dist[f];
        for (int i = 0; i < 3; ++i) H[3 * a + i] += coef * (m[3 * b + i] - m[3 * a + i]);
    }
    for (int64_t a = 0; a < n; ++a) {
        /* uniaxial anisotropy: (2K/(mu0 Ms)) (m.e) e */
        const double* e = P->easy + 3 * a;
        double me = m[3 * a] * e[0] + m[3 * a + 1] * e[1] + m[3 * a + 2] * e[2];
        double ka = 2.0 * P->Ku[a] / (ORC_MU0 * P->Ms[a]);
        for (int i = 0; i < 3; ++i) H[3 * a + i] += ka * me * e[i] + Ha[i];
    }
}

/* Landau-Lifshitz right-hand side (paper Sec. 2.1):
 * dm/dt = -c1 m x H - c2 m x (m x H). */
void orc_ll_rhs(const orc_problem* P, const double* m, const double Ha[3], double* dmdt, double* Hbuf) {
    int64_t n = P->n;
    orc_heff(P, m, Ha, Hbuf);
    for (int64_t a = 0; a < n; ++a) {
        const double* v = m + 3 * a;
        const double* h = Hbuf + 3 * a;
        double p0 = v[1] * h[2] - v[2] * h[1];
        double p1 = v[2] * h[0] - v[0] * h[2];
        double p2 = v[0] * h[1] - v[1] * h[0];
        double q0 = v[1] * p2 - v[2] * p1;
        double q1 = v[2] * p0 - v[0] * p2;
        double q2 = v[0] * p1 - v[1] * p0;
        dmdt[3 * a + 0] = -P->c1 * p0 - P->c2 * q0;
        dmdt[3 * a + 1] = -P->c1 * p1 - P->c2 * q1;
        dmdt[3 * a + 2] = -P->c1 * p2 - P->c2 * q2;
    }
}

static void renormalise(int64_t n, double* m) {
    for (int64_t a = 0; a < n; ++a) {
        double r = sqrt(m[3 * a] * m[3 * a] + m[3 * a + 1] * m[3 * a + 1] + m[3 * a + 2] * m[3 * a + 2]);
        m[3 * a] /= r; m[3 * a + 1] /= r; m[3 * a + 2] /= r;
    }
}

/* One classical fourth-order Runge-Kutta step of fixed size dt, then
 * |m| = 1 restored per tile when renorm != 0 (the LL flow preserves the
 * norm, Sec. 2.1; the discrete step does not exactly). */
void orc_rk4_step(const orc_problem* P, double* m, const double Ha[3], double dt, int renorm) {
    int64_t N3 = 3 * P->n;
    double* k1 = malloc(sizeof(double) * N3);
    double* k2 = malloc(sizeof(double) * N3);
    double* k3 = malloc(sizeof(double) * N3);
    double* k4 = malloc(sizeof(double) * N3);
    double* y = malloc(sizeof(double) * N3);
    double* hb = malloc(sizeof(double) * N3);
    orc_ll_rhs(P, m, Ha, k1, hb);
    for (int64_t i = 0; i < N3; ++i) y[i] = m[i] + 0.5 * dt * k1[i];
    orc_ll_rhs(P, y, Ha, k2, hb);
    for (int64_t i = 0; i < N3; ++i) y[i] = m[i] + 0.5 * dt * k2[i];
    orc_ll_rhs(P, y, Ha, k3, hb);
    for (int64_t i = 0; i < N3; ++i) y[i] = m[i] + dt * k3[i];
    orc_ll_rhs(P, y, Ha, k4, hb);
    for (int64_t i = 0; i < N3; ++i) m[i] += dt / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    if (renorm) renormalise(P->n, m);
    free(k1); free(k2); free(k3); free(k4); free(y); free(hb);
}

/* Dormand-Prince 5(4) coefficients (the embedded explicit Runge-Kutta (4,5)
 * pair the paper integrates with, Sec. 3.1). */
static const double DP_A[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
/* fifth-order weights are the last row of A (first-same-as-last); the
 * embedded fourth-order weights are: */
static const double DP_BSTAR[7] = {5179.0 / 57600, 0, 7571.0 / 16695, 393.0 / 640,
                                   -92097.0 / 339200, 187.0 / 2100, 1.0 / 40};

/* One attempted adaptive Dormand-Prince step.
 *   m      : in/out state (changed only on acceptance)
 *   k1     : in/out f(m) (first-same-as-last: on acceptance it becomes k7)
 *   dt     : in/out step size; on return the proposal for the next attempt
 *   t      : in/out time (advanced on acceptance)
 *   err_out: scaled max-norm error of this attempt
 *   dmdt_max_out: max over tiles of |k7_a| (Euclidean), i.e. of dm/dt at the
 *            proposed new state
 * Error: e = dt sum_s (b_s - b*_s) k_s,
 *        err = max_i |e_i| / (atol + rtol max(|y_i|, |y5_i|)),
 * accept iff err <= 1, dt_next = dt * min(5, max(0.2, 0.9 err^(-1/5)))
 * (factor 5 when err == 0); t_end > 0 caps the next step at t_end - t.
 * Returns 1 when accepted. */
int orc_dp45_attempt(const orc_problem* P, double* m, double* k1, const double Ha[3], double* dt,
                     double* t, double atol, double rtol, int renorm, double t_end,
                     double* err_out, double* dmdt_max_out) {
    int64_t n = P->n, N3 = 3 * n;
    double* k[7];
    k[0] = k1;
    for (int s = 1; s < 7; ++s) k[s] = malloc(sizeof(double) * N3);
    double* y = malloc(sizeof(double) * N3);
    double* hb = malloc(sizeof(double) * N3);
    double h = *dt;
    for (int s = 1; s < 7; ++s) {
        for (int64_t i = 0; i < N3; ++i) {
            double acc = 0.0;
            for (int j = 0; j < s; ++j) acc += DP_A[s][j] * k[j][i];
            y[i] = m[i] + h * acc;
        }
        orc_ll_rhs(P, y, Ha, k[s], hb);
    }
    /* y now holds the fifth-order solution (stage-7 input) and k[6] = f(y). */
    double err = 0.0;
    for (int64_t i = 0; i < N3; ++i) {
        double e = 0.0;
        for (int s = 0; s < 7; ++s) {
            double b5 = (s < 6) ? DP_A[6][s] : 0.0; /* fifth-order weight */
            e += (b5 - DP_BSTAR[s]) * k[s][i];
        }
        e *= h;
        double sc = atol + rtol * fmax(fabs(m[i]), fabs(y[i]));
        double r = fabs(e) / sc;
        if (r > err) err = r;
    }
    double dmax = 0.0;
    for (int64_t a = 0; a < n; ++a) {
        const double* v = k[6] + 3 * a;
        double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        if (r > dmax) dmax = r;
    }
    int accept = err <= 1.0;
    if (accept) {
        memcpy(m, y, sizeof(double) * N3);
        if (renorm) renormalise(n, m);
        memcpy(k1, k[6], sizeof(double) * N3);
        *t += h;
    }
    double fac = (err == 0.0) ? 5.0 : fmin(5.0, fmax(0.2, 0.9 * pow(err, -0.2)));
    double hn = h * fac;
    if (t_end > 0.0 && *t + hn > t_end) hn = t_end - *t;
    *dt = hn;
    *err_out = err;
    *dmdt_max_out = dmax;
    for (int s = 1; s < 7; ++s) free(k[s]);
    free(y); free(hb);
    return accept;
}

/* Free energy, split in its four terms [J] (paper Sec. 2.2 and 2.3):
 *   E[0] demag    = (mu0/2) sum_a V_a Ms_a m_a . (N (Ms m))_a
 *   E[1] exchange = A sum_{faces, each once} S_ab |m_b - m_a|^2 / d_ab
 *   E[2] anis     = - sum_a V_a K_a (m_a . e_a)^2
 *   E[3] Zeeman   = - mu0 sum_a V_a Ms_a m_a . H_a */
void orc_energy(const orc_problem* P, const double* m, const double Ha[3], double E[4]) {
    int64_t n = P->n;
    double* hd = malloc(sizeof(double) * 3 * n);
    orc_demag(n, P->T, P->Ms, m, hd);
    double ed = 0.0, ex = 0.0, ea = 0.0, ez = 0.0;
    for (int64_t a = 0; a < n; ++a) {
        const double* v = m + 3 * a;
        double w = P->vol[a] * P->Ms[a];
        ed += -0.5 * ORC_MU0 * w * (v[0] * hd[3 * a] + v[1] * hd[3 * a + 1] + v[2] * hd[3 * a + 2]);
        ez += -ORC_MU0 * w * (v[0] * Ha[0] + v[1] * Ha[1] + v[2] * Ha[2]);
        const double* e = P->easy + 3 * a;
        double me = v[0] * e[0] + v[1] * e[1] + v[2] * e[2];
        ea += -P->vol[a] * P->Ku[a] * me * me;
    }
    for (int64_t f = 0; f < P->nfaces; ++f) {
        int64_t a = P->fa[f], b = P->fb[f];
        if (b < a) continue; /* each face once */
        double d2 = 0.0;
        for (int i = 0; i < 3; ++i) {
            double d = m[3 * b + i] - m[3 * a + i];
            d2 += d * d;
        }
        ex += P->A * P->area[f] * d2 / P->dist[f];
    }
    E[0] = ed; E[1] = ex; E[2] = ea; E[3] = ez;
    free(hd);
}
