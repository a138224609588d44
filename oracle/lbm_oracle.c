/*
 * Oracle: one time step of the pseudo-potential D2Q9 lattice Boltzmann method of
 * Hu, Li & Uddin, "Force Method in a Pseudo-potential Lattice Boltzmann Model"
 * (arXiv:1412.5170), in plain IEEE FP64 on the CPU.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this file.  It shares no code, table or
 * header with the HIP library: the velocity set, weights, moment matrix and every
 * formula are written out here again from the paper.
 *
 * The code is deliberately slow and literal: whole-lattice arrays for rho, psi and
 * F are built first (Sec. 2, Eq. 3, Eq. 7, Eq. 6), then every node is collided
 * (Eq. 1 with the forcing scheme of Sec. 3.2 / Sec. 4.3, or the MRT collision of
 * Sec. 4.4.2) and streamed into a fresh array (Eq. 36).  Periodic boundaries.
 *
 * Readings of the paper taken here (all listed with their reasons in the design
 * notes of the repository):
 *   - the force of Eq. 4/Eq. 5 is a vector: each neighbour term carries e_alpha,
 *     as Eq. 6 and Eq. 8 show;
 *   - omega_alpha of Eq. 6 are the interaction weights w(1)=1/3, w(2)=1/12 given
 *     under Eq. 4, not the D2Q9 weights of Eq. 2;
 *   - c in Eq. 7 is the lattice speed 1, so p0 = rho/3 + G psi^2/2;
 *   - the tensor (F_i v_j + v_j F_i) of Eq. 23 / Eq. 31 is the symmetric
 *     (F_i v_j + v_i F_j);
 *   - upsilon in Li's shifted velocity v' = v + sigma F/(upsilon psi^2) (Eq. 31)
 *     is (tau - 1/2) delta_t, which is what makes Eq. 32 give eps = 1.68 for
 *     sigma = 0.105 (Sec. 4.3.1); f^eq keeps v, only the force bracket takes v';
 *   - the MRT moment basis is Lallemand & Luo's, rows ordered as Lambda in Eq. 35;
 *     m_eq = M f^eq(rho, v) as Eq. 34 defines it; the Guo source in moment space is
 *     S = M B(v) with B the Guo bracket;
 *   - MRT with Li's term (not in the paper): Li's extra stress 2 sigma F F / psi^2
 *     is added per moment with the factor 1/(1/s_k - 1/2) so that, when every
 *     rate equals 1/tau, the collision reduces exactly to BGK with Eq. 31;
 *   - unstable states (psi^2 <= 0, b rho/4 >= 1, non-finite values) are reported,
 *     never clamped.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define Q 9

/* D2Q9 velocities (Sec. 2, under Eq. 2): rest, four axis links, four diagonals. */
static const int EX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
/* D2Q9 weights of Eq. 2: 4/9, 1/9 (axis), 1/36 (diagonal). */
static const double WEQ[Q] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                              1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2 = 1.0 / 3.0; /* c_s^2 = c^2/3 with c = 1 (Sec. 2) */

enum { ORC_EDM = 0, ORC_GUO = 1, ORC_GUO_LI = 2, ORC_SC = 3 };
enum { ORC_BGK = 0, ORC_MRT = 1 };
enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_EUNSTABLE = -2, ORC_ENOMEM = -3 };

typedef struct {
    int nx, ny;
    double a, b, R; /* Carnahan-Starling constants (Eq. 29) */
    double T;       /* absolute temperature */
    double K;       /* EOS rescale (Eq. 30) */
    double G;       /* interaction strength (Eq. 4-7) */
    double A;       /* hybrid weight (Eq. 6) */
    double sigma;   /* Li's constant (Eq. 31) */
    double tau;     /* relaxation time (Eq. 1) */
    int scheme;     /* ORC_EDM / ORC_GUO / ORC_GUO_LI / ORC_SC */
    int collision;  /* ORC_BGK / ORC_MRT */
    double s[Q];    /* MRT rates, Eq. 35 order (rho, e, eps, jx, qx, jy, qy, pxx, pxy) */
    int psi_kind;   /* 0: psi from the EOS through Eq. 7; 1: the effective density of Eq. 33 */
    double psi_eps; /* Eq. 33 exponent eps (psi_kind 1); eps = 0 selects exp(-1/rho) */
} orc_params;

/* Interaction weight w(|e|^2) given under Eq. 4: w(1) = 1/3, w(2) = 1/12. */
static double w_int(int a)
{
    int e2 = EX[a] * EX[a] + EY[a] * EY[a];
    if (e2 == 1) return 1.0 / 3.0;
    if (e2 == 2) return 1.0 / 12.0;
    return 0.0;
}

/* Rescaled Carnahan-Starling pressure, Eq. 29 and Eq. 30. */
double orc_pressure(const orc_params *p, double rho)
{
    double eta = p->b * rho / 4.0;
    double num = 1.0 + eta + eta * eta - eta * eta * eta;
    double den = (1.0 - eta) * (1.0 - eta) * (1.0 - eta);
    return p->K * (rho * p->R * p->T * num / den - p->a * rho * rho);
}

/* Effective density from Eq. 7: p0 = c_s^2 rho + G psi^2 / 2  =>  psi = sqrt(2 (p0 - c_s^2 rho) / G).
 * Returns NaN when the state is outside the EOS (eta >= 1) or the radicand is not positive. */
double orc_psi(const orc_params *p, double rho)
{
    if (p->psi_kind == 1) {
        /* Eq. 33 (Sbragaglia and Shan): psi = exp(-1/rho) for eps = 0, else
         * (rho / (1 + rho))^(1/eps); the pressure is then whatever Eq. 7 implies. */
        if (!(rho > 0.0)) return NAN;
        if (p->psi_eps == 0.0) return exp(-1.0 / rho);
        return pow(rho / (1.0 + rho), 1.0 / p->psi_eps);
    }
    double eta = p->b * rho / 4.0;
    if (!(eta < 1.0) || !(rho > 0.0)) return NAN;
    double U = orc_pressure(p, rho) - CS2 * rho;
    double r = 2.0 * U / p->G;
    if (!(r > 0.0)) return NAN;
    return sqrt(r);
}

/* Equilibrium distribution, Eq. 2. */
void orc_feq(double rho, double ux, double uy, double *out)
{
    for (int a = 0; a < Q; a++) {
        double eu = EX[a] * ux + EY[a] * uy;
        double uu = ux * ux + uy * uy;
        out[a] = WEQ[a] * rho * (1.0 + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
    }
}

/* f^eq(rho, u) for every node; f is laid out [9][n]. */
void orc_init_feq(int n, const double *rho, const double *ux, const double *uy, double *f)
{
    double fe[Q];
    for (int i = 0; i < n; i++) {
        orc_feq(rho[i], ux ? ux[i] : 0.0, uy ? uy[i] : 0.0, fe);
        for (int a = 0; a < Q; a++) f[(size_t)a * n + i] = fe[a];
    }
}

/* The bracket of Guo's forcing term, Eq. 23, without the (1 - 1/(2 tau)) factor:
 *   w_a [ F_i e_ai / c_s^2 + (F_i V_j + V_i F_j)(e_ai e_aj - c_s^2 delta_ij) / (2 c_s^4) ],
 * written with explicit sums over the Cartesian indices i, j. */
static void guo_bracket(double Fx, double Fy, double Vx, double Vy, double *out)
{
    double F[2] = {Fx, Fy}, V[2] = {Vx, Vy};
    for (int a = 0; a < Q; a++) {
        double e[2] = {(double)EX[a], (double)EY[a]};
        double lin = 0.0, quad = 0.0;
        for (int i = 0; i < 2; i++) lin += F[i] * e[i] / CS2;
        for (int i = 0; i < 2; i++)
            for (int j = 0; j < 2; j++)
                quad += (F[i] * V[j] + V[i] * F[j]) * (e[i] * e[j] - CS2 * (i == j ? 1.0 : 0.0)) /
                        (2.0 * CS2 * CS2);
        out[a] = WEQ[a] * (lin + quad);
    }
}

/* MRT transformation matrix (Lallemand & Luo basis), each row written from its
 * polynomial definition, rows in the order of Lambda in Eq. 35. */
static void mrt_matrix(double M[Q][Q])
{
    for (int a = 0; a < Q; a++) {
        double ex = EX[a], ey = EY[a], e2 = ex * ex + ey * ey;
        M[0][a] = 1.0;                               /* density rho          */
        M[1][a] = -4.0 + 3.0 * e2;                   /* energy e             */
        M[2][a] = 4.0 - 10.5 * e2 + 4.5 * e2 * e2;   /* energy square eps    */
        M[3][a] = ex;                                /* momentum j_x         */
        M[4][a] = (-5.0 + 3.0 * e2) * ex;            /* energy flux q_x      */
        M[5][a] = ey;                                /* momentum j_y         */
        M[6][a] = (-5.0 + 3.0 * e2) * ey;            /* energy flux q_y      */
        M[7][a] = ex * ex - ey * ey;                 /* normal stress p_xx   */
        M[8][a] = ex * ey;                           /* shear stress p_xy    */
    }
}

/* Plain Gauss-Jordan inversion with partial pivoting. */
static int invert9(double M[Q][Q], double Minv[Q][Q])
{
    double A[Q][2 * Q];
    for (int i = 0; i < Q; i++)
        for (int j = 0; j < 2 * Q; j++) A[i][j] = j < Q ? M[i][j] : (j - Q == i ? 1.0 : 0.0);
    for (int c = 0; c < Q; c++) {
        int piv = c;
        for (int r = c + 1; r < Q; r++)
            if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
        if (A[piv][c] == 0.0) return -1;
        if (piv != c)
            for (int j = 0; j < 2 * Q; j++) {
                double t = A[c][j];
                A[c][j] = A[piv][j];
                A[piv][j] = t;
            }
        double d = A[c][c];
        for (int j = 0; j < 2 * Q; j++) A[c][j] /= d;
        for (int r = 0; r < Q; r++) {
            if (r == c) continue;
            double m = A[r][c];
            if (m != 0.0)
                for (int j = 0; j < 2 * Q; j++) A[r][j] -= m * A[c][j];
        }
    }
    for (int i = 0; i < Q; i++)
        for (int j = 0; j < Q; j++) Minv[i][j] = A[i][j + Q];
    return 0;
}

static int check_params(const orc_params *p)
{
    if (!p || p->nx < 1 || p->ny < 1) return ORC_EINVAL;
    if (!(p->tau > 0.5)) return ORC_EINVAL;
    if (!(p->G < 0.0)) return ORC_EINVAL;
    if (p->psi_kind == 0 && (!(p->b > 0.0) || !(p->K > 0.0) || !(p->T > 0.0))) return ORC_EINVAL;
    if (p->psi_kind != 0 && (p->psi_kind != 1 || !(p->psi_eps >= 0.0))) return ORC_EINVAL;
    if (p->scheme < ORC_EDM || p->scheme > ORC_SC) return ORC_EINVAL;
    if (p->collision != ORC_BGK && p->collision != ORC_MRT) return ORC_EINVAL;
    if (p->collision == ORC_MRT) {
        if (p->scheme != ORC_GUO && p->scheme != ORC_GUO_LI) return ORC_EINVAL;
        for (int k = 0; k < Q; k++)
            if (!(p->s[k] > 0.0 && p->s[k] < 2.0)) return ORC_EINVAL;
    }
    return ORC_OK;
}

static size_t idx(const orc_params *p, int x, int y) { return (size_t)y * p->nx + x; }

/* Steps 1-4 of one time step on the current populations f ([9][ny][nx]):
 * rho (Eq. 3), psi (Eq. 7 with Eq. 29-30), F (Eq. 6), u and v = u + F/(2 rho)
 * (Sec. 3.2).  Any output pointer may be NULL except those needed internally. */
int orc_fields(const orc_params *p, const double *f, double *rho, double *psi, double *Fx,
               double *Fy, double *ux, double *uy, double *vx, double *vy)
{
    int rc = check_params(p);
    if (rc) return rc;
    const int nx = p->nx, ny = p->ny;
    const size_t n = (size_t)nx * ny;
    int unstable = 0;

    /* Eq. 3: density is the zeroth moment. */
#pragma omp parallel for schedule(static)
    for (size_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int a = 0; a < Q; a++) s += f[a * n + i];
        rho[i] = s;
    }
    /* Eq. 7: effective density of every node, before any force is formed. */
#pragma omp parallel for schedule(static) reduction(| : unstable)
    for (size_t i = 0; i < n; i++) {
        psi[i] = orc_psi(p, rho[i]);
        if (!isfinite(psi[i])) unstable = 1;
    }
    /* Eq. 6: F = -A sum w U(x+e) e - (1-A) G psi(x) sum w psi(x+e) e, U = G psi^2 / 2. */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
            double sUx = 0.0, sUy = 0.0, sPx = 0.0, sPy = 0.0;
            for (int a = 1; a < Q; a++) {
                int xn = ((x + EX[a]) % nx + nx) % nx;
                int yn = ((y + EY[a]) % ny + ny) % ny;
                double pn = psi[idx(p, xn, yn)];
                double Un = p->G * pn * pn / 2.0;
                sUx += w_int(a) * Un * EX[a];
                sUy += w_int(a) * Un * EY[a];
                sPx += w_int(a) * pn * EX[a];
                sPy += w_int(a) * pn * EY[a];
            }
            double ps = psi[idx(p, x, y)];
            Fx[idx(p, x, y)] = -p->A * sUx - (1.0 - p->A) * p->G * ps * sPx;
            Fy[idx(p, x, y)] = -p->A * sUy - (1.0 - p->A) * p->G * ps * sPy;
        }
    /* u = sum f e / rho (Eq. 21/22) and the actual fluid velocity v = u + F/(2 rho). */
#pragma omp parallel for schedule(static) reduction(| : unstable)
    for (size_t i = 0; i < n; i++) {
        double jx = 0.0, jy = 0.0;
        for (int a = 0; a < Q; a++) {
            jx += f[a * n + i] * EX[a];
            jy += f[a * n + i] * EY[a];
        }
        double u_x = jx / rho[i], u_y = jy / rho[i];
        if (ux) ux[i] = u_x;
        if (uy) uy[i] = u_y;
        if (vx) vx[i] = u_x + Fx[i] / (2.0 * rho[i]);
        if (vy) vy[i] = u_y + Fy[i] / (2.0 * rho[i]);
        if (!isfinite(u_x) || !isfinite(u_y)) unstable = 1;
    }
    return unstable ? ORC_EUNSTABLE : ORC_OK;
}

/* Step 5: post-collision populations of one node. */
static void collide_node(const orc_params *p, const double fin[Q], double rho, double psi,
                         double Fx, double Fy, double M[Q][Q], double Minv[Q][Q], double fout[Q])
{
    double jx = 0.0, jy = 0.0;
    for (int a = 0; a < Q; a++) {
        jx += fin[a] * EX[a];
        jy += fin[a] * EY[a];
    }
    const double ux = jx / rho, uy = jy / rho;
    const double vx = ux + Fx / (2.0 * rho), vy = uy + Fy / (2.0 * rho);
    const double tau = p->tau;
    double fe[Q], fe2[Q], B[Q];

    if (p->collision == ORC_BGK) {
        switch (p->scheme) {
        case ORC_SC: /* Eq. 20-21: velocity shift u_eq = u + tau F / rho, no source term */
            orc_feq(rho, ux + tau * Fx / rho, uy + tau * Fy / rho, fe);
            for (int a = 0; a < Q; a++) fout[a] = fin[a] - (fin[a] - fe[a]) / tau;
            break;
        case ORC_EDM: /* Eq. 22: F_a = f^eq(rho, u + du) - f^eq(rho, u), du = F / rho */
            orc_feq(rho, ux, uy, fe);
            orc_feq(rho, ux + Fx / rho, uy + Fy / rho, fe2);
            for (int a = 0; a < Q; a++) fout[a] = fin[a] - (fin[a] - fe[a]) / tau + (fe2[a] - fe[a]);
            break;
        case ORC_GUO: /* Eq. 23, equilibrium at the actual velocity v */
        case ORC_GUO_LI: { /* Eq. 31: bracket at v' = v + sigma F / ((tau - 1/2) psi^2) */
            double bx = vx, by = vy;
            if (p->scheme == ORC_GUO_LI) {
                bx = vx + p->sigma * Fx / ((tau - 0.5) * psi * psi);
                by = vy + p->sigma * Fy / ((tau - 0.5) * psi * psi);
            }
            orc_feq(rho, vx, vy, fe);
            guo_bracket(Fx, Fy, bx, by, B);
            for (int a = 0; a < Q; a++)
                fout[a] = fin[a] - (fin[a] - fe[a]) / tau + (1.0 - 1.0 / (2.0 * tau)) * B[a];
            break;
        }
        }
        return;
    }

    /* MRT, Eq. 34-36: m* = m - Lambda (m - m_eq) + (I - Lambda/2) S,  f* = M^-1 m*. */
    double m[Q], meq[Q], S[Q], mstar[Q];
    orc_feq(rho, vx, vy, fe);
    guo_bracket(Fx, Fy, vx, vy, B);
    for (int k = 0; k < Q; k++) {
        m[k] = meq[k] = S[k] = 0.0;
        for (int a = 0; a < Q; a++) {
            m[k] += M[k][a] * fin[a];
            meq[k] += M[k][a] * fe[a];
            S[k] += M[k][a] * B[a];
        }
    }
    if (p->scheme == ORC_GUO_LI) {
        /* Li's extra stress X = 2 sigma F F / psi^2, one factor 1/(1/s_k - 1/2) per moment. */
        double c = 2.0 * p->sigma / (psi * psi);
        double Xxx = c * Fx * Fx, Xyy = c * Fy * Fy, Xxy = c * Fx * Fy;
        double tr = Xxx + Xyy;
        S[1] += 3.0 * tr / (1.0 / p->s[1] - 0.5);
        S[2] += -3.0 * tr / (1.0 / p->s[2] - 0.5);
        S[7] += (Xxx - Xyy) / (1.0 / p->s[7] - 0.5);
        S[8] += Xxy / (1.0 / p->s[8] - 0.5);
    }
    for (int k = 0; k < Q; k++)
        mstar[k] = m[k] - p->s[k] * (m[k] - meq[k]) + (1.0 - p->s[k] / 2.0) * S[k];
    for (int a = 0; a < Q; a++) {
        double s = 0.0;
        for (int k = 0; k < Q; k++) s += Minv[a][k] * mstar[k];
        fout[a] = s;
    }
}

typedef struct {
    double *rho, *psi, *Fx, *Fy;
} work_t;

static int work_alloc(work_t *w, size_t n)
{
    w->rho = malloc(n * sizeof(double));
    w->psi = malloc(n * sizeof(double));
    w->Fx = malloc(n * sizeof(double));
    w->Fy = malloc(n * sizeof(double));
    if (!w->rho || !w->psi || !w->Fx || !w->Fy) return ORC_ENOMEM;
    return ORC_OK;
}

static void work_free(work_t *w)
{
    free(w->rho);
    free(w->psi);
    free(w->Fx);
    free(w->Fy);
}

/* Post-collision populations f* of every node, before streaming ([9][ny][nx]). */
int orc_collide(const orc_params *p, const double *f, double *fpost)
{
    int rc = check_params(p);
    if (rc) return rc;
    const size_t n = (size_t)p->nx * p->ny;
    double M[Q][Q], Minv[Q][Q];
    mrt_matrix(M);
    if (invert9(M, Minv)) return ORC_EINVAL;
    work_t w;
    if (work_alloc(&w, n)) {
        work_free(&w);
        return ORC_ENOMEM;
    }
    rc = orc_fields(p, f, w.rho, w.psi, w.Fx, w.Fy, NULL, NULL, NULL, NULL);
    if (rc == ORC_OK) {
        for (size_t i = 0; i < n; i++) {
            double fin[Q], fout[Q];
            for (int a = 0; a < Q; a++) fin[a] = f[a * n + i];
            collide_node(p, fin, w.rho[i], w.psi[i], w.Fx[i], w.Fy[i], M, Minv, fout);
            for (int a = 0; a < Q; a++) fpost[a * n + i] = fout[a];
        }
    }
    work_free(&w);
    return rc;
}

/* nsteps full time steps in place on f ([9][ny][nx], post-stream populations):
 * fields (steps 1-4), collision (step 5), periodic streaming (Eq. 36). */
int orc_step(const orc_params *p, double *f, int nsteps)
{
    int rc = check_params(p);
    if (rc) return rc;
    if (nsteps < 0) return ORC_EINVAL;
    const int nx = p->nx, ny = p->ny;
    const size_t n = (size_t)nx * ny;
    double M[Q][Q], Minv[Q][Q];
    mrt_matrix(M);
    if (invert9(M, Minv)) return ORC_EINVAL;
    work_t w;
    double *fnew = malloc(Q * n * sizeof(double));
    if (work_alloc(&w, n) || !fnew) {
        work_free(&w);
        free(fnew);
        return ORC_ENOMEM;
    }
    for (int t = 0; t < nsteps && rc == ORC_OK; t++) {
        rc = orc_fields(p, f, w.rho, w.psi, w.Fx, w.Fy, NULL, NULL, NULL, NULL);
        if (rc != ORC_OK) break;
#pragma omp parallel for schedule(static)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                size_t i = idx(p, x, y);
                double fin[Q], fout[Q];
                for (int a = 0; a < Q; a++) fin[a] = f[a * n + i];
                collide_node(p, fin, w.rho[i], w.psi[i], w.Fx[i], w.Fy[i], M, Minv, fout);
                /* Eq. 36: f_a(x + e_a, t + 1) = f*_a(x, t), periodic wrap. */
                for (int a = 0; a < Q; a++) {
                    int xd = ((x + EX[a]) % nx + nx) % nx;
                    int yd = ((y + EY[a]) % ny + ny) % ny;
                    fnew[a * n + idx(p, xd, yd)] = fout[a];
                }
            }
        memcpy(f, fnew, Q * n * sizeof(double));
    }
    work_free(&w);
    free(fnew);
    return rc;
}

/* The moment matrix as built above and its numerical inverse (for tests). */
int orc_mrt_matrix(double *M_out, double *Minv_out)
{
    double M[Q][Q], Minv[Q][Q];
    mrt_matrix(M);
    if (invert9(M, Minv)) return ORC_EINVAL;
    for (int i = 0; i < Q; i++)
        for (int j = 0; j < Q; j++) {
            if (M_out) M_out[i * Q + j] = M[i][j];
            if (Minv_out) Minv_out[i * Q + j] = Minv[i][j];
        }
    return ORC_OK;
}

/* Guo's bracket of Eq. 23 at one (F, V), without the (1 - 1/(2 tau)) factor (for tests). */
void orc_guo_bracket(double Fx, double Fy, double Vx, double Vy, double *out)
{
    guo_bracket(Fx, Fy, Vx, Vy, out);
}

/* Number of OpenMP threads the stepper's parallel loops use (1 without OpenMP). */
#ifdef _OPENMP
#include <omp.h>
int orc_threads(void) { return omp_get_max_threads(); }
/* Threads of the later parallel loops (for timing the stepper on one core). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
#else
int orc_threads(void) { return 1; }
void orc_set_threads(int n) { (void)n; }
#endif
