/* Drives every entry point of the oracle's C stepper on tiny and ragged lattices, for a build
 * with the address and undefined-behaviour sanitizers: any out-of-bounds access, use of freed
 * memory or undefined arithmetic aborts the run.  Exit status 0 when every call returned what
 * it should. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int nx, ny;
    double a, b, R, T, K, G, A, sigma, tau;
    int scheme, collision;
    double s[9];
    int psi_kind;
    double psi_eps;
} orc_params;

int orc_step(const orc_params *p, double *f, int nsteps);
int orc_collide(const orc_params *p, const double *f, double *fpost);
int orc_fields(const orc_params *p, const double *f, double *rho, double *psi, double *Fx,
               double *Fy, double *ux, double *uy, double *vx, double *vy);
void orc_init_feq(int n, const double *rho, const double *ux, const double *uy, double *f);
void orc_feq(double rho, double ux, double uy, double *out);
double orc_pressure(const orc_params *p, double rho);
double orc_psi(const orc_params *p, double rho);
int orc_mrt_matrix(double *M_out, double *Minv_out);
void orc_guo_bracket(double Fx, double Fy, double Vx, double Vy, double *out);
int orc_threads(void);
void orc_set_threads(int n);

static int failures = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                   \
        }                                                                 \
    } while (0)

int main(void)
{
    const int sizes[][2] = {{1, 1}, {3, 3}, {4, 3}, {1, 7}, {7, 5}, {16, 9}};
    const int kinds[][2] = {{0, 0}, {1, 0}, {2, 0}, {3, 0}, {1, 1}, {2, 1}};
    for (size_t si = 0; si < sizeof sizes / sizeof sizes[0]; ++si)
        for (size_t ki = 0; ki < sizeof kinds / sizeof kinds[0]; ++ki)
            for (int pk = 0; pk < 2; ++pk) {
                const int nx = sizes[si][0], ny = sizes[si][1], n = nx * ny;
                orc_params p = {nx, ny, 1.0, 4.0, 1.0, 0.0660301, 0.3, pk ? -3.0 : -1.0, -0.3,
                                0.11, 0.8, kinds[ki][0], kinds[ki][1],
                                {1.0, 1.1, 1.2, 1.0, 1.3, 1.0, 1.3, 1.25, 1.25}, pk, 1.0};
                double *rho = malloc(sizeof(double) * n), *f = malloc(sizeof(double) * 9 * n);
                double *g = malloc(sizeof(double) * 9 * n), *w[8];
                for (int k = 0; k < 8; ++k) w[k] = malloc(sizeof(double) * n);
                for (int i = 0; i < n; ++i) rho[i] = 0.05 + 0.3 * (double)((i * 7919) % 97) / 97.0;
                orc_init_feq(n, rho, NULL, NULL, f);
                CHECK(orc_fields(&p, f, w[0], w[1], w[2], w[3], w[4], w[5], w[6], w[7]) == 0);
                CHECK(orc_collide(&p, f, g) == 0);
                CHECK(orc_step(&p, f, 3) == 0);
                for (int i = 0; i < 9 * n; ++i) CHECK(isfinite(f[i]));
                free(rho);
                free(f);
                free(g);
                for (int k = 0; k < 8; ++k) free(w[k]);
            }
    /* invalid parameters and unstable states are reported, not stepped */
    orc_params bad = {3, 3, 1.0, 4.0, 1.0, 0.06, 1.0, -1.0, 0.0, 0.0, 0.5, 1, 0,
                      {1, 1, 1, 1, 1, 1, 1, 1, 1}, 0, 1.0};
    double f[81], rho[9];
    for (int i = 0; i < 9; ++i) rho[i] = 0.2;
    orc_init_feq(9, rho, NULL, NULL, f);
    CHECK(orc_step(&bad, f, 1) == -1);                 /* tau = 1/2 */
    bad.tau = 1.0;
    bad.scheme = 0;
    bad.collision = 1;
    CHECK(orc_step(&bad, f, 1) == -1);                 /* MRT with EDM */
    bad.collision = 0;
    for (int i = 0; i < 9; ++i) rho[i] = 1.5;          /* beyond the packing limit 4/b */
    orc_init_feq(9, rho, NULL, NULL, f);
    CHECK(orc_step(&bad, f, 1) == -2);
    CHECK(isnan(orc_psi(&bad, 1.5)) && isnan(orc_psi(&bad, -0.1)));
    CHECK(isfinite(orc_pressure(&bad, 0.2)));
    double M[81], Mi[81], B[9], fe[9];
    CHECK(orc_mrt_matrix(M, Mi) == 0);
    orc_guo_bracket(1e-3, -2e-3, 0.05, 0.01, B);
    orc_feq(0.3, 0.01, -0.02, fe);
    orc_set_threads(1);
    CHECK(orc_threads() == 1);
    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    puts("oracle driver: ok");
    return 0;
}
