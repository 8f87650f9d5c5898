/*
 * Plain FP64 CPU oracle of the 3f model ("three fluids") of Zhan, Chai & Shi
 * (arXiv 2311.05091) on the D2Q9 lattice: the three-component Cahn-Hilliard
 * model of Sec. 2.1 solved for p = 0 and p = 1 by two CH lattices (f0 for
 * phi0, f1 for phi1; phi2 = 1 - phi0 - phi1), coupled to the NS lattice g of
 * Sec. 3, all with the Hermite-moment collision of Sec. 4 (Sec. 3 names the
 * 3f model as the equations with p = 0 and 1; Sec. 4 gives its degenerate
 * mobility f = (1 - phi0)(1 - phi1)(1 - phi2); Sec. 4.1 runs it with
 * sigma01 = sigma02 = sigma12).
 *
 * TEST INFRASTRUCTURE ONLY, like tpf_oracle.c (built into the same library
 * and using its lattice algebra: weights, M0, N, the equilibrium, source,
 * force and pressure formulas, which are the same for every phase).  Nothing
 * in the product path may link, load or call it.
 *
 * Readings of passages the paper leaves open (numbered after the 2f1s ones):
 *   R23 the NS step of the 3f model has no solid: the effective viscosity is
 *       mu (no 1/(1 - phi0)), there is no fluid-structure force phi0 rho f,
 *       and u = u* (Sec. 4.1 lists the viscosity among the differences of
 *       the two models; phase 0 is a fluid).
 *   R24 both CH lattices use the same scale factor d0, the same rates s0,
 *       s1 = 1/tau_phi, s2, s3, s4, and eta_p from (M_cst + M_deg)/gamma_p =
 *       (1/s1 - 1/2) eta_p c_s^2 (Sec. 3, per phase).
 *   R25 the spreading coefficients gamma_p follow from the three pairwise
 *       tensions (Sec. 2.1); the extra mass flux is S = sum_p rho_p M
 *       grad(mubar_p)/gamma_p with all three phases, written with
 *       grad(mubar_2)/gamma_2 = -(grad(mubar_0)/gamma_0 + grad(mubar_1)/gamma_1)
 *       (the sum of mubar_p/gamma_p vanishes by construction of L).
 * Readings R2, R3 (stencils and wall mirrors, now also on phi0 and mubar0),
 * R5-R9 (lagged F_c, explicit Euler from zero, uF + Fu, gauge, initial
 * state) and R11 (the s2a term of H) carry over unchanged.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* grids below this many nodes run each pass on one thread (the per-pass
 * thread start-up would cost more than the pass) */
#define ORC_PAR_MIN 8192

/* lattice algebra of tpf_oracle.c (same library) */
void orc_velocities(int32_t cx[9], int32_t cy[9]);
void orc_weights(double d0, double w[9]);
void orc_M0(double M0[81]);
void orc_N(double cs2, double N[81]);
int orc_inverse9(const double A[81], double Ainv[81]);
void orc_relaxation_matrix(double cs2, const double Kdiag[9], double S[81]);
void orc_collide_with(const double M0[81], const double M0inv[81], const double S[81], const double f[9],
                      const double feq[9], const double R[9], double fout[9]);
void orc_chemical_potentials(const double gamma[3], double D, double phi0, double phi1, double lap0,
                             double lap1, double mu_out[3], double mubar_out[3]);
void orc_feq(double d0, double phi, double eta_mub, double Ax, double Ay, double feq[9]);
void orc_Rpop(double d0, double dAx, double dAy, double a, double eta_gx, double eta_gy, double R[9]);
void orc_geq(double d0, double rho_gauge, double P, double rho, double ux, double uy, double Sx, double Sy,
             double geq[9]);
void orc_Fpop(double d0, double Q, double Gx, double Gy, double Mxx, double Myy, double Mxy, double F[9]);
double orc_pressure(double d0, double s0, double s2a, const double g[9], double u_grad_rho, double B,
                    double B_prev);
double orc_visc_rate(double mu_v, double rho, double phi0, double cfac);

typedef struct {
    int32_t nx, ny;
    int32_t periodic_x, periodic_y;
    double d0, D;
    double sigma01, sigma02, sigma12;  /* pairwise surface tensions            */
    double rho[3], mu[3];              /* densities, viscosities of phases 0-2 */
    double M_cst, M_deg;
    double tau_phi;                    /* 1/s1 of both CH lattices             */
    double s_phi[4];                   /* s0, s2, s3, s4 of both CH lattices   */
    double s_g[4];                     /* s0, s1, s3, s4 of the NS lattice     */
    double Fb[2];
    double rho_gauge;
} orc3f_params;

enum { L_A0X, L_A0Y, L_A1X, L_A1Y, L_B, L_CXX, L_CYY, L_CXY, L_PSI, NLAG3F };
enum { G_PHI0, G_PHI1, G_GX0, G_GY0, G_LAP0, G_GX1, G_GY1, G_LAP1, G_MU0, G_MU1, G_MU2, G_MUB0, G_MUB1,
       G_GM0X, G_GM0Y, G_GM1X, G_GM1Y, G_UX, G_UY, G_P, NG };

typedef struct {
    orc3f_params P;
    double gamma[3], gammaT, eta[2], cs2;
    int nx, ny;
    size_t n;
    double* fpost[2];  /* [9][n] post-collision CH populations of phi0, phi1 */
    double* gpost;     /* [9][n] */
    double* lag;       /* [NLAG3F][n] */
    double* f[2];      /* streamed */
    double* g;
    double* fld;       /* [NG][n] */
    double* lag_new;
    double M0[81], M0inv[81], N[81], Ninv[81], Sphi[81];
    int cx[9], cy[9], opp[9];
    int64_t step;
} orc3f_sim;

#define FL(s, k) ((s)->fld + (size_t)(k) * (s)->n)

/* gamma_p from the pairwise tensions (Sec. 2.1); eta_p (reading R24). */
int orc3f_derive(const orc3f_params* P, double gamma[3], double* gammaT, double eta[2])
{
    gamma[0] = P->sigma01 + P->sigma02 - P->sigma12;
    gamma[1] = P->sigma01 + P->sigma12 - P->sigma02;
    gamma[2] = P->sigma02 + P->sigma12 - P->sigma01;
    if (!(gamma[0] > 0 && gamma[1] > 0 && gamma[2] > 0)) return -1;
    *gammaT = 3.0 / (1.0 / gamma[0] + 1.0 / gamma[1] + 1.0 / gamma[2]);
    for (int p = 0; p < 2; ++p) eta[p] = (P->M_cst + P->M_deg) / (gamma[p] * (P->tau_phi - 0.5) * P->d0);
    return 0;
}

static int wrap_or_mirror3f(int j, int n, int periodic)
{
    if (periodic) { j %= n; if (j < 0) j += n; return j; }
    if (j < 0) return -1 - j;
    if (j >= n) return 2 * n - 1 - j;
    return j;
}

static void stencil3f(const orc3f_sim* s, const double* a, int x, int y, double* gx, double* gy, double* lap)
{
    double v[3][3];
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            int xx = wrap_or_mirror3f(x + dx, s->nx, s->P.periodic_x);
            int yy = wrap_or_mirror3f(y + dy, s->ny, s->P.periodic_y);
            v[dy + 1][dx + 1] = a[(size_t)yy * s->nx + xx];
        }
    double E = v[1][2], W = v[1][0], N = v[2][1], S = v[0][1];
    double NE = v[2][2], NW = v[2][0], SE = v[0][2], SW = v[0][0], C = v[1][1];
    if (gx) *gx = (4.0 * (E - W) + (NE - NW + SE - SW)) / 12.0;
    if (gy) *gy = (4.0 * (N - S) + (NE - SE + NW - SW)) / 12.0;
    if (lap) *lap = (4.0 * (E + W + N + S) + (NE + NW + SE + SW) - 20.0 * C) / 6.0;
}

static void stream3f(orc3f_sim* s)
{
    int nx = s->nx, ny = s->ny;
    size_t n = s->n;
#pragma omp parallel for if ((size_t)nx * ny >= ORC_PAR_MIN)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t id = (size_t)y * nx + x;
            for (int i = 0; i < 9; ++i) {
                int xs = x - s->cx[i], ys = y - s->cy[i], out = 0;
                if (s->P.periodic_x) xs = (xs % nx + nx) % nx; else if (xs < 0 || xs >= nx) out = 1;
                if (s->P.periodic_y) ys = (ys % ny + ny) % ny; else if (ys < 0 || ys >= ny) out = 1;
                size_t src = out ? (size_t)s->opp[i] * n + id : (size_t)i * n + (size_t)ys * nx + xs;
                for (int p = 0; p < 2; ++p) s->f[p][(size_t)i * n + id] = s->fpost[p][src];
                s->g[(size_t)i * n + id] = s->gpost[src];
            }
        }
}

static void matmul3f(const double A[81], const double B[81], double C[81])
{
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 9; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 9; ++k) acc += A[r * 9 + k] * B[k * 9 + c];
            C[r * 9 + c] = acc;
        }
}

static void macro_and_collide3f(orc3f_sim* s, int collide)
{
    const orc3f_params* P = &s->P;
    int nx = s->nx, ny = s->ny;
    size_t n = s->n;
    double cs2 = s->cs2;

    /* phase fields phi0 = sum f0, phi1 = sum f1 */
#pragma omp parallel for if ((size_t)nx * ny >= ORC_PAR_MIN)
    for (size_t id = 0; id < n; ++id) {
        double a = 0.0, b = 0.0;
        for (int i = 0; i < 9; ++i) {
            a += s->f[0][(size_t)i * n + id];
            b += s->f[1][(size_t)i * n + id];
        }
        FL(s, G_PHI0)[id] = a;
        FL(s, G_PHI1)[id] = b;
    }
#pragma omp parallel for if ((size_t)nx * ny >= ORC_PAR_MIN)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t id = (size_t)y * nx + x;
            stencil3f(s, FL(s, G_PHI0), x, y, &FL(s, G_GX0)[id], &FL(s, G_GY0)[id], &FL(s, G_LAP0)[id]);
            stencil3f(s, FL(s, G_PHI1), x, y, &FL(s, G_GX1)[id], &FL(s, G_GY1)[id], &FL(s, G_LAP1)[id]);
        }
    /* chemical potentials mu_p and the corrected mubar_0, mubar_1 */
#pragma omp parallel for if ((size_t)nx * ny >= ORC_PAR_MIN)
    for (size_t id = 0; id < n; ++id) {
        double mu[3], mub[3];
        orc_chemical_potentials(s->gamma, P->D, FL(s, G_PHI0)[id], FL(s, G_PHI1)[id], FL(s, G_LAP0)[id],
                                FL(s, G_LAP1)[id], mu, mub);
        FL(s, G_MU0)[id] = mu[0];
        FL(s, G_MU1)[id] = mu[1];
        FL(s, G_MU2)[id] = mu[2];
        FL(s, G_MUB0)[id] = mub[0];
        FL(s, G_MUB1)[id] = mub[1];
    }
#pragma omp parallel for if ((size_t)nx * ny >= ORC_PAR_MIN)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t id = (size_t)y * nx + x;
            stencil3f(s, FL(s, G_MUB0), x, y, &FL(s, G_GM0X)[id], &FL(s, G_GM0Y)[id], NULL);
            stencil3f(s, FL(s, G_MUB1), x, y, &FL(s, G_GM1X)[id], &FL(s, G_GM1Y)[id], NULL);
        }

    const double* lag = s->lag;
    double* lag_new = s->lag_new;
    const double r0 = P->rho[0], r1 = P->rho[1], r2 = P->rho[2];
#pragma omp parallel for if ((size_t)nx * ny >= ORC_PAR_MIN)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t id = (size_t)y * nx + x;
            double phi0 = FL(s, G_PHI0)[id], phi1 = FL(s, G_PHI1)[id], phi2 = 1.0 - phi0 - phi1;
            double gx0 = FL(s, G_GX0)[id], gy0 = FL(s, G_GY0)[id], gx1 = FL(s, G_GX1)[id], gy1 = FL(s, G_GY1)[id];
            double mu0 = FL(s, G_MU0)[id], mu1 = FL(s, G_MU1)[id], mu2 = FL(s, G_MU2)[id];
            double gm0x = FL(s, G_GM0X)[id], gm0y = FL(s, G_GM0Y)[id];
            double gm1x = FL(s, G_GM1X)[id], gm1y = FL(s, G_GM1Y)[id];

            /* degenerate mobility of the 3f model (Sec. 4) */
            double fdeg = (1.0 - phi0) * (1.0 - phi1) * (1.0 - phi2);
            double Mob = P->M_cst + P->M_deg * fdeg;
            double a = P->M_deg * (1.0 - fdeg) / (P->M_cst + P->M_deg);

            double rho = r0 * phi0 + r1 * phi1 + r2 * phi2;
            double mu_v = P->mu[0] * phi0 + P->mu[1] * phi1 + P->mu[2] * phi2;
            double drx = (r0 - r2) * gx0 + (r1 - r2) * gx1;
            double dry = (r0 - r2) * gy0 + (r1 - r2) * gy1;

            /* S = sum_p rho_p M grad(mubar_p)/gamma_p (reading R25) */
            double Sx = Mob * ((r0 - r2) * gm0x / s->gamma[0] + (r1 - r2) * gm1x / s->gamma[1]);
            double Sy = Mob * ((r0 - r2) * gm0y / s->gamma[0] + (r1 - r2) * gm1y / s->gamma[1]);

            double Fsx = mu0 * gx0 + mu1 * gx1 - mu2 * (gx0 + gx1);
            double Fsy = mu0 * gy0 + mu1 * gy1 - mu2 * (gy0 + gy1);
            double dpx, dpy;
            stencil3f(s, lag + (size_t)L_PSI * n, x, y, &dpx, &dpy, NULL);
            double Fx = Fsx + P->Fb[0] - 0.5 * dpy;
            double Fy = Fsy + P->Fb[1] + 0.5 * dpx;

            /* velocity without a solid (reading R23) */
            double gl[9], jx = 0.0, jy = 0.0;
            for (int i = 0; i < 9; ++i) {
                gl[i] = s->g[(size_t)i * n + id];
                jx += s->cx[i] * gl[i];
                jy += s->cy[i] * gl[i];
            }
            double ux = (jx + 0.5 * Fx) / rho, uy = (jy + 0.5 * Fy) / rho;

            double s2a = orc_visc_rate(mu_v, rho, 0.0, 0.5 * (1.0 - cs2));
            double s2b = orc_visc_rate(mu_v, rho, 0.0, cs2);
            double Q = ux * drx + uy * dry;
            double B = (rho * ux - Sx) * ux + (rho * uy - Sy) * uy;
            double p = orc_pressure(P->d0, P->s_g[0], s2a, gl, Q, B, lag[(size_t)L_B * n + id]);
            FL(s, G_UX)[id] = ux;
            FL(s, G_UY)[id] = uy;
            FL(s, G_P)[id] = p;
            if (!collide) continue;

            /* ---- the two CH collisions ---- */
            const double phis[2] = {phi0, phi1};
            const double mubs[2] = {FL(s, G_MUB0)[id], FL(s, G_MUB1)[id]};
            const double gmx[2] = {gm0x, gm1x}, gmy[2] = {gm0y, gm1y};
            for (int q = 0; q < 2; ++q) {
                double Ax = phis[q] * ux, Ay = phis[q] * uy;
                double fl[9], feq[9], R[9], fo[9];
                for (int i = 0; i < 9; ++i) fl[i] = s->f[q][(size_t)i * n + id];
                orc_feq(P->d0, phis[q], s->eta[q] * mubs[q], Ax, Ay, feq);
                orc_Rpop(P->d0, Ax - lag[(size_t)(L_A0X + 2 * q) * n + id], Ay - lag[(size_t)(L_A0Y + 2 * q) * n + id],
                         a, s->eta[q] * gmx[q], s->eta[q] * gmy[q], R);
                orc_collide_with(s->M0, s->M0inv, s->Sphi, fl, feq, R, fo);
                for (int i = 0; i < 9; ++i) s->fpost[q][(size_t)i * n + id] = fo[i];
                lag_new[(size_t)(L_A0X + 2 * q) * n + id] = Ax;
                lag_new[(size_t)(L_A0Y + 2 * q) * n + id] = Ay;
            }

            /* ---- NS collision (G = F: no fluid-structure force) ---- */
            double Cxx = Sx * ux, Cyy = Sy * uy, Cxy = 0.5 * (Sx * uy + Sy * ux);
            double Mxx = 2.0 * ux * Fx - (Cxx - lag[(size_t)L_CXX * n + id]) + 2.0 * cs2 * ux * drx + (1.0 - 3.0 * cs2) * Q;
            double Myy = 2.0 * uy * Fy - (Cyy - lag[(size_t)L_CYY * n + id]) + 2.0 * cs2 * uy * dry + (1.0 - 3.0 * cs2) * Q;
            double Mxy = ux * Fy + Fx * uy - (Cxy - lag[(size_t)L_CXY * n + id]) + cs2 * (ux * dry + drx * uy);
            double geq[9], Fp[9], go[9];
            orc_geq(P->d0, P->rho_gauge, p, rho, ux, uy, Sx, Sy, geq);
            orc_Fpop(P->d0, Q, Fx, Fy, Mxx, Myy, Mxy, Fp);
            double Kg[9] = {P->s_g[0], P->s_g[1], P->s_g[1], s2a, s2a, s2b, P->s_g[2], P->s_g[2], P->s_g[3]};
            double KN[81], Sg[81];
            for (int r = 0; r < 9; ++r)
                for (int c = 0; c < 9; ++c) KN[r * 9 + c] = Kg[r] * s->N[r * 9 + c];
            matmul3f(s->Ninv, KN, Sg);
            orc_collide_with(s->M0, s->M0inv, Sg, gl, geq, Fp, go);
            for (int i = 0; i < 9; ++i) s->gpost[(size_t)i * n + id] = go[i];
            lag_new[(size_t)L_B * n + id] = B;
            lag_new[(size_t)L_CXX * n + id] = Cxx;
            lag_new[(size_t)L_CYY * n + id] = Cyy;
            lag_new[(size_t)L_CXY * n + id] = Cxy;
            lag_new[(size_t)L_PSI * n + id] = Sx * uy - Sy * ux;
        }
    if (collide) memcpy(s->lag, s->lag_new, (size_t)NLAG3F * n * sizeof(double));
}

orc3f_sim* orc3f_create(const orc3f_params* P, const double* phi0, const double* phi1)
{
    orc3f_sim* s = (orc3f_sim*)calloc(1, sizeof(orc3f_sim));
    s->P = *P;
    if (orc3f_derive(P, s->gamma, &s->gammaT, s->eta) != 0) { free(s); return NULL; }
    s->cs2 = P->d0;
    s->nx = P->nx; s->ny = P->ny; s->n = (size_t)P->nx * P->ny;
    size_t n = s->n;
    for (int p = 0; p < 2; ++p) {
        s->fpost[p] = (double*)malloc(9 * n * sizeof(double));
        s->f[p] = (double*)malloc(9 * n * sizeof(double));
    }
    s->gpost = (double*)malloc(9 * n * sizeof(double));
    s->g = (double*)malloc(9 * n * sizeof(double));
    s->lag = (double*)calloc((size_t)NLAG3F * n, sizeof(double));
    s->lag_new = (double*)calloc((size_t)NLAG3F * n, sizeof(double));
    s->fld = (double*)calloc((size_t)NG * n, sizeof(double));
    int32_t cx[9], cy[9];
    orc_velocities(cx, cy);
    for (int i = 0; i < 9; ++i) { s->cx[i] = cx[i]; s->cy[i] = cy[i]; }
    for (int i = 0; i < 9; ++i)
        for (int j = 0; j < 9; ++j)
            if (cx[j] == -cx[i] && cy[j] == -cy[i]) s->opp[i] = j;
    orc_M0(s->M0);
    orc_inverse9(s->M0, s->M0inv);
    orc_N(s->cs2, s->N);
    orc_inverse9(s->N, s->Ninv);
    double s1 = 1.0 / P->tau_phi;
    double Kphi[9] = {P->s_phi[0], s1, s1, P->s_phi[1], P->s_phi[1], P->s_phi[1], P->s_phi[2], P->s_phi[2],
                      P->s_phi[3]};
    orc_relaxation_matrix(s->cs2, Kphi, s->Sphi);
    memcpy(FL(s, G_PHI0), phi0, n * sizeof(double));
    memcpy(FL(s, G_PHI1), phi1, n * sizeof(double));
    /* initial state (reading R9, per CH lattice) */
    for (int y = 0; y < s->ny; ++y)
        for (int x = 0; x < s->nx; ++x) {
            size_t id = (size_t)y * s->nx + x;
            stencil3f(s, FL(s, G_PHI0), x, y, NULL, NULL, &FL(s, G_LAP0)[id]);
            stencil3f(s, FL(s, G_PHI1), x, y, NULL, NULL, &FL(s, G_LAP1)[id]);
        }
    for (size_t id = 0; id < n; ++id) {
        double mu[3], mub[3], feq[9], geq[9];
        orc_chemical_potentials(s->gamma, P->D, phi0[id], phi1[id], FL(s, G_LAP0)[id], FL(s, G_LAP1)[id], mu, mub);
        for (int p = 0; p < 2; ++p) {
            orc_feq(P->d0, p == 0 ? phi0[id] : phi1[id], s->eta[p] * mub[p], 0.0, 0.0, feq);
            for (int i = 0; i < 9; ++i) s->fpost[p][(size_t)i * n + id] = feq[i];
        }
        orc_geq(P->d0, P->rho_gauge, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0, geq);
        for (int i = 0; i < 9; ++i) s->gpost[(size_t)i * n + id] = geq[i];
    }
    s->step = 0;
    return s;
}

void orc3f_free(orc3f_sim* s)
{
    if (!s) return;
    for (int p = 0; p < 2; ++p) { free(s->fpost[p]); free(s->f[p]); }
    free(s->gpost); free(s->g); free(s->lag); free(s->lag_new); free(s->fld); free(s);
}

void orc3f_step(orc3f_sim* s, int64_t nsteps)
{
    for (int64_t k = 0; k < nsteps; ++k) {
        stream3f(s);
        macro_and_collide3f(s, 1);
        s->step++;
    }
}

/* phi0, phi1, u, p at the current time level (without advancing). */
void orc3f_moments(orc3f_sim* s, double* phi0, double* phi1, double* ux, double* uy, double* p)
{
    stream3f(s);
    macro_and_collide3f(s, 0);
    size_t n = s->n;
    if (phi0) memcpy(phi0, FL(s, G_PHI0), n * sizeof(double));
    if (phi1) memcpy(phi1, FL(s, G_PHI1), n * sizeof(double));
    if (ux) memcpy(ux, FL(s, G_UX), n * sizeof(double));
    if (uy) memcpy(uy, FL(s, G_UY), n * sizeof(double));
    if (p) memcpy(p, FL(s, G_P), n * sizeof(double));
}

/* Phase masses sum phi0 and sum phi1 (streaming only permutes populations). */
void orc3f_mass(const orc3f_sim* s, double m[2])
{
    for (int p = 0; p < 2; ++p) {
        long double acc = 0.0L;
        for (size_t k = 0; k < 9 * s->n; ++k) acc += s->fpost[p][k];
        m[p] = (double)acc;
    }
}

void orc3f_get_state(const orc3f_sim* s, double* f0, double* f1, double* g, double* lag)
{
    size_t n = s->n;
    if (f0) memcpy(f0, s->fpost[0], 9 * n * sizeof(double));
    if (f1) memcpy(f1, s->fpost[1], 9 * n * sizeof(double));
    if (g) memcpy(g, s->gpost, 9 * n * sizeof(double));
    if (lag) memcpy(lag, s->lag, (size_t)NLAG3F * n * sizeof(double));
}

int64_t orc3f_step_count(const orc3f_sim* s) { return s->step; }
