/* Driver for the sanitizer test of the oracle: exercises every entry point of
 * oracle.c on a small mesh of unlike cuboids (ASan + UBSan build, host only).
 * The struct below mirrors the oracle's problem record field for field. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int64_t n;
    const double* T;
    const double* vol;
    const double* Ms;
    double A;
    const double* Ku;
    const double* easy;
    int64_t nfaces;
    const int64_t* fa;
    const int64_t* fb;
    const double* area;
    const double* dist;
    double c1, c2;
} orc_problem;

void orc_assemble(int64_t n, const double* centers, const double* sizes, double* T);
void orc_demag(int64_t n, const double* T, const double* Ms, const double* m, double* Hd);
double orc_threshold(int64_t n, double* T, double frac);
void orc_demag_rows(int64_t n, const double* centers, const double* sizes, const double* Ms, const double* m,
                    int64_t nrows, const int64_t* rows, double* Hd);
int64_t orc_faces(int64_t n, const double* centers, const double* sizes, int64_t cap, int64_t* fa, int64_t* fb,
                  double* area, double* dist);
void orc_heff(const orc_problem* P, const double* m, const double Ha[3], double* H);
void orc_ll_rhs(const orc_problem* P, const double* m, const double Ha[3], double* dmdt, double* Hbuf);
void orc_rk4_step(const orc_problem* P, double* m, const double Ha[3], double dt, int renorm);
int orc_dp45_attempt(const orc_problem* P, double* m, double* k1, const double Ha[3], double* dt, double* t,
                     double atol, double rtol, int renorm, double t_end, double* err, double* dmdt_max);
void orc_energy(const orc_problem* P, const double* m, const double Ha[3], double E[4]);

int main(void) {
    /* a 4 x 3 x 2 grid of 4 x 3 x 2 nm cuboids, one of them split in two along x */
    enum { NX = 4, NY = 3, NZ = 2 };
    const int n = NX * NY * NZ + 1;
    double* c = calloc(3 * n, sizeof(double));
    double* s = calloc(3 * n, sizeof(double));
    int a = 0;
    for (int k = 0; k < NZ; ++k)
        for (int j = 0; j < NY; ++j)
            for (int i = 0; i < NX; ++i) {
                double dx = 4e-9, x0 = i * 4e-9;
                if (i == 1 && j == 1 && k == 0) {
                    for (int h = 0; h < 2; ++h, ++a) {
                        c[3 * a] = x0 + (h + 0.5) * 2e-9; c[3 * a + 1] = (j + 0.5) * 3e-9; c[3 * a + 2] = (k + 0.5) * 2e-9;
                        s[3 * a] = 2e-9; s[3 * a + 1] = 3e-9; s[3 * a + 2] = 2e-9;
                    }
                    continue;
                }
                c[3 * a] = x0 + 0.5 * dx; c[3 * a + 1] = (j + 0.5) * 3e-9; c[3 * a + 2] = (k + 0.5) * 2e-9;
                s[3 * a] = dx; s[3 * a + 1] = 3e-9; s[3 * a + 2] = 2e-9;
                ++a;
            }
    double* T = malloc(sizeof(double) * 9 * n * n);
    orc_assemble(n, c, s, T);
    double* Ms = malloc(sizeof(double) * n);
    double* vol = malloc(sizeof(double) * n);
    double* Ku = malloc(sizeof(double) * n);
    double* easy = malloc(sizeof(double) * 3 * n);
    double* m = malloc(sizeof(double) * 3 * n);
    double* H = malloc(sizeof(double) * 3 * n);
    double* k1 = malloc(sizeof(double) * 3 * n);
    for (int b = 0; b < n; ++b) {
        Ms[b] = 8e5 - 1e4 * b;
        vol[b] = s[3 * b] * s[3 * b + 1] * s[3 * b + 2];
        Ku[b] = 1e4;
        easy[3 * b] = 0.0; easy[3 * b + 1] = 0.6; easy[3 * b + 2] = 0.8;
        double th = 0.3 * b, ph = 0.17 * b;
        m[3 * b] = cos(th) * sin(ph + 0.4); m[3 * b + 1] = sin(th) * sin(ph + 0.4); m[3 * b + 2] = cos(ph + 0.4);
    }
    orc_demag(n, T, Ms, m, H);
    int64_t rows[3] = {0, n / 2, n - 1};
    double Hr[9];
    orc_demag_rows(n, c, s, Ms, m, 3, rows, Hr);
    int64_t cap = 12 * n;
    int64_t* fa = malloc(sizeof(int64_t) * cap);
    int64_t* fb = malloc(sizeof(int64_t) * cap);
    double* area = malloc(sizeof(double) * cap);
    double* dist = malloc(sizeof(double) * cap);
    int64_t nf = orc_faces(n, c, s, cap, fa, fb, area, dist);
    orc_problem P = {n, T, vol, Ms, 1.3e-11, Ku, easy, nf, fa, fb, area, dist, 2.2e5, 4.4e4};
    const double Ha[3] = {1e4, -2e4, 5e3};
    orc_heff(&P, m, Ha, H);
    orc_ll_rhs(&P, m, Ha, k1, H);
    double E[4];
    orc_energy(&P, m, Ha, E);
    orc_rk4_step(&P, m, Ha, 1e-14, 1);
    double dt = 1e-14, t = 0.0, err = 0.0, dmx = 0.0;
    orc_ll_rhs(&P, m, Ha, k1, H);
    for (int it = 0; it < 20; ++it) orc_dp45_attempt(&P, m, k1, Ha, &dt, &t, 1e-6, 1e-6, 1, 0.0, &err, &dmx);
    double* T2 = malloc(sizeof(double) * 9 * n * n);
    for (int64_t i = 0; i < 9 * (int64_t)n * n; ++i) T2[i] = T[i];
    double cut = orc_threshold(n, T2, 0.4);
    int finite = isfinite(E[0]) && isfinite(E[1]) && isfinite(cut) && isfinite(t) && nf > 0;
    printf("n=%d faces=%lld t=%g cut=%g E=%g %g %g %g finite=%d\n", n, (long long)nf, t, cut, E[0], E[1], E[2],
           E[3], finite);
    free(c); free(s); free(T); free(T2); free(Ms); free(vol); free(Ku); free(easy); free(m); free(H); free(k1);
    free(fa); free(fb); free(area); free(dist);
    return finite ? 0 : 1;
}
