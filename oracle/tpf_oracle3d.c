/*
 * Plain FP64 CPU oracle of the three-dimensional coupled step of Zhan, Chai &
 * Shi, "A ternary phase-field model for two-phase flows in complex
 * geometries" (arXiv 2311.05091): the 2f1s model on the D3Q15 lattice with
 * the Hermite-moment collision, Appendix A (D3Q15 weights, M0 and N_H) and
 * the 3D pressure constants of Sec. 3 (K = 1 - 2 d0, H = K[(1 - d0)/s0 -
 * (3 - 7 d0)/s2a + (1 - 3 d0)]).
 *
 * TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the CPU leg of
 * the benchmark use it.  It shares no source with the GPU library, nor with
 * the two-dimensional oracle (tpf_oracle.c) beyond being compiled into the
 * same shared object.
 *
 * Written to be read against the paper:
 *   - collision with the dense 15x15 matrices M0 and N_H of Appendix A,
 *     S = N_H^-1 K N_H (C_d = I since c = 1), inverses by Gauss-Jordan;
 *   - equilibria and sources per direction as printed in Sec. 3 with the
 *     sums over alpha and alpha < alpha-bar running over x, y, z;
 *   - one pass per field over the grid, in the order of the paper.
 * The readings R1-R11 of the two-dimensional oracle apply unchanged, with:
 *   R2' gradients and Laplacians use the isotropic central stencils built on
 *       the D3Q15 weights at d0 = 1/3 (2/9, 1/9, 1/72; c_s^2 = 1/3), as the
 *       2D stencils are built on the D2Q9 weights at d0 = 1/3;
 *   R5' the correction force F_c = div(Su - uS)/2 is evaluated from the
 *       previous step's psi = S x u: F_c = -curl(psi)/2 (the 2D psi is its
 *       z component);
 *   R11' in H the s2a term is zero where its coefficient K (3 - 7 d0) is zero
 *       (K = 0 at d0 = 1/2, where H vanishes altogether) and, as in 2D, where
 *       s2a = 0 (saturated solid node, phi0 = 1).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* grids below this many nodes run each pass on one thread (the per-pass
 * thread start-up would cost more than the pass) */
#define ORC_PAR_MIN 8192

#define Q15 15

typedef struct {
    int32_t nx, ny, nz;
    int32_t periodic[3];
    double d0, D, sigma12, theta, kappa;
    double rho[3], mu[3];
    double M_cst, M_deg, tau_phi;
    double s_phi[4];    /* s0, s2, s3, s4 of the CH lattice */
    double s_g[4];      /* s0, s1, s3, s4 of the NS lattice */
    double Fb[3];
    double u_wall[3];   /* translation velocity of the solid points */
    double rho_gauge;
} orc3_params;

/* D3Q15 velocities in the order of the columns of M0 (App. A). */
static const int C3[Q15][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                               {0, 0, 1},  {0, 0, -1}, {1, 1, 1},  {-1, 1, 1}, {1, -1, 1},
                               {-1, -1, 1}, {1, 1, -1}, {-1, 1, -1}, {1, -1, -1}, {-1, -1, -1}};

static int opposite(int i)
{
    for (int j = 0; j < Q15; ++j)
        if (C3[j][0] == -C3[i][0] && C3[j][1] == -C3[i][1] && C3[j][2] == -C3[i][2]) return j;
    return -1;
}

void orc3_velocities(int32_t c[45])
{
    for (int i = 0; i < Q15; ++i)
        for (int a = 0; a < 3; ++a) c[3 * i + a] = C3[i][a];
}

/* weights (App. A): w0 = 1 - 3 d0 + 2 d0^2, w1-6 = (d0 - d0^2)/2, w7-14 = d0^2/8 */
void orc3_weights(double d0, double w[Q15])
{
    w[0] = 1.0 - 3.0 * d0 + 2.0 * d0 * d0;
    for (int i = 1; i <= 6; ++i) w[i] = (d0 - d0 * d0) / 2.0;
    for (int i = 7; i < Q15; ++i) w[i] = d0 * d0 / 8.0;
}

/* M0 rows: 1, cx, cy, cz, cx^2, cy^2, cz^2, cx cy, cy cz, cx cz, cx cy^2,
 * cy cz^2, cz cx^2, cx cy cz, cx^2 cy^2 cz^2 (each row takes the values of
 * the printed matrix on the velocities above). */
void orc3_M0(double M0[Q15 * Q15])
{
    for (int i = 0; i < Q15; ++i) {
        double x = C3[i][0], y = C3[i][1], z = C3[i][2];
        double r[Q15] = {1.0, x, y, z, x * x, y * y, z * z, x * y, y * z, x * z,
                         x * y * y, y * z * z, z * x * x, x * y * z, x * x * y * y * z * z};
        for (int k = 0; k < Q15; ++k) M0[k * Q15 + i] = r[k];
    }
}

/* N_H of App. A (D3Q15). */
void orc3_N(double cs2, double N[Q15 * Q15])
{
    memset(N, 0, Q15 * Q15 * sizeof(double));
    for (int i = 0; i < Q15; ++i) N[i * Q15 + i] = 1.0;
    N[4 * Q15 + 0] = -cs2;
    N[5 * Q15 + 0] = -cs2;
    N[6 * Q15 + 0] = -cs2;
    N[10 * Q15 + 1] = -cs2;
    N[11 * Q15 + 2] = -cs2;
    N[12 * Q15 + 3] = -cs2;
    N[14 * Q15 + 0] = 2.0 * cs2 * cs2;
    N[14 * Q15 + 4] = -cs2;
    N[14 * Q15 + 5] = -cs2;
    N[14 * Q15 + 6] = -cs2;
}

/* Gauss-Jordan inverse of an n x n matrix with partial pivoting. */
int orc3_inverse(int n, const double* A, double* Ainv)
{
    double a[Q15][2 * Q15];
    if (n > Q15) return -1;
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < 2 * n; ++c) a[r][c] = c < n ? A[r * n + c] : (c - n == r ? 1.0 : 0.0);
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
        if (fabs(a[piv][col]) < 1e-300) return -1;
        if (piv != col)
            for (int c = 0; c < 2 * n; ++c) { double t = a[col][c]; a[col][c] = a[piv][c]; a[piv][c] = t; }
        double p = a[col][col];
        for (int c = 0; c < 2 * n; ++c) a[col][c] /= p;
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            double m = a[r][col];
            if (m == 0.0) continue;
            for (int c = 0; c < 2 * n; ++c) a[r][c] -= m * a[col][c];
        }
    }
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) Ainv[r * n + c] = a[r][c + n];
    return 0;
}

static void matmul15(const double* A, const double* B, double* C)
{
    for (int r = 0; r < Q15; ++r)
        for (int c = 0; c < Q15; ++c) {
            double s = 0.0;
            for (int k = 0; k < Q15; ++k) s += A[r * Q15 + k] * B[k * Q15 + c];
            C[r * Q15 + c] = s;
        }
}

static void matvec15(const double* A, const double* x, double* y)
{
    for (int r = 0; r < Q15; ++r) {
        double s = 0.0;
        for (int k = 0; k < Q15; ++k) s += A[r * Q15 + k] * x[k];
        y[r] = s;
    }
}

/* S = N_H^-1 K N_H (Sec. 4), K = diag(Kdiag). */
void orc3_relaxation_matrix(double cs2, const double Kdiag[Q15], double S[Q15 * Q15])
{
    double N[Q15 * Q15], Ninv[Q15 * Q15], KN[Q15 * Q15];
    orc3_N(cs2, N);
    orc3_inverse(Q15, N, Ninv);
    for (int r = 0; r < Q15; ++r)
        for (int c = 0; c < Q15; ++c) KN[r * Q15 + c] = Kdiag[r] * N[r * Q15 + c];
    matmul15(Ninv, KN, S);
}

/* m = M0 f,  m* = m - S (m - m_eq) + (I - S/2) M0 R,  f* = M0^-1 m*  (Sec. 4) */
static void collide_with(const double* M0, const double* M0inv, const double* S, const double* f,
                         const double* feq, const double* R, double* fout)
{
    double m[Q15], meq[Q15], mR[Q15], d[Q15], Sd[Q15], SR[Q15], ms[Q15];
    matvec15(M0, f, m);
    matvec15(M0, feq, meq);
    matvec15(M0, R, mR);
    for (int k = 0; k < Q15; ++k) d[k] = m[k] - meq[k];
    matvec15(S, d, Sd);
    matvec15(S, mR, SR);
    for (int k = 0; k < Q15; ++k) ms[k] = m[k] - Sd[k] + mR[k] - 0.5 * SR[k];
    matvec15(M0inv, ms, fout);
}

void orc3_collide(double cs2, const double Kdiag[Q15], const double f[Q15], const double feq[Q15],
                  const double R[Q15], double fout[Q15])
{
    double M0[Q15 * Q15], M0inv[Q15 * Q15], S[Q15 * Q15];
    orc3_M0(M0);
    orc3_inverse(Q15, M0, M0inv);
    orc3_relaxation_matrix(cs2, Kdiag, S);
    collide_with(M0, M0inv, S, f, feq, R, fout);
}

/* ---------------------------------------------------------------------- */
/* Equilibria and sources (Sec. 3), sums over alpha = x, y, z             */
/* ---------------------------------------------------------------------- */
static double cdot(int i, const double v[3]) { return C3[i][0] * v[0] + C3[i][1] * v[1] + C3[i][2] * v[2]; }

void orc3_feq(double d0, double phi, double eta_mub, const double A[3], double feq[Q15])
{
    double w[Q15];
    orc3_weights(d0, w);
    feq[0] = phi + (w[0] - 1.0) * eta_mub;
    for (int i = 1; i < Q15; ++i) feq[i] = w[i] * eta_mub + w[i] * cdot(i, A) / d0;
}

void orc3_Rpop(double d0, const double dA[3], double a, const double eta_g[3], double R[Q15])
{
    double w[Q15];
    orc3_weights(d0, w);
    for (int i = 0; i < Q15; ++i) R[i] = w[i] * (cdot(i, dA) / d0 + a * cdot(i, eta_g));
}

/* symmetric tensor T as (xx, yy, zz, xy, yz, xz) */
static double tensor_term(int i, double cs2, const double T[6])
{
    const int pa[3][2] = {{0, 1}, {1, 2}, {0, 2}};
    double diag = 0.0, off = 0.0;
    for (int a = 0; a < 3; ++a) diag += (C3[i][a] * C3[i][a] - cs2) * T[a];
    for (int k = 0; k < 3; ++k) off += C3[i][pa[k][0]] * C3[i][pa[k][1]] * T[3 + k];
    return diag / (cs2 - cs2 * cs2) + off / (cs2 * cs2);
}

void orc3_geq(double d0, double gauge, double P, double rho, const double u[3], const double S[3],
              double geq[Q15])
{
    double w[Q15], cs2 = d0, j[3], Pi[6];
    orc3_weights(d0, w);
    for (int a = 0; a < 3; ++a) j[a] = rho * u[a];
    for (int a = 0; a < 3; ++a) Pi[a] = rho * u[a] * u[a] - S[a] * u[a];
    Pi[3] = rho * u[0] * u[1] - 0.5 * (S[0] * u[1] + u[0] * S[1]);
    Pi[4] = rho * u[1] * u[2] - 0.5 * (S[1] * u[2] + u[1] * S[2]);
    Pi[5] = rho * u[0] * u[2] - 0.5 * (S[0] * u[2] + u[0] * S[2]);
    for (int i = 0; i < Q15; ++i) {
        double lam = (i == 0) ? (w[0] - 1.0) * P / cs2 + gauge : w[i] * P / cs2;
        geq[i] = lam + w[i] * cdot(i, j) / cs2 + w[i] * tensor_term(i, cs2, Pi);
    }
}

void orc3_Fpop(double d0, double Q, const double G[3], const double M2[6], double F[Q15])
{
    double w[Q15], cs2 = d0;
    orc3_weights(d0, w);
    for (int i = 0; i < Q15; ++i) F[i] = w[i] * (Q + cdot(i, G) / cs2 + tensor_term(i, cs2, M2));
}

/* Pressure (Sec. 3, 3D constants), reading R11'. */
double orc3_pressure(double d0, double s0, double s2a, const double g[Q15], double Q, double B, double B_prev)
{
    double w[Q15], cs2 = d0;
    orc3_weights(d0, w);
    double K = 1.0 - 2.0 * d0;
    double cH = K * (3.0 - 7.0 * d0);
    double H = K * ((1.0 - d0) / s0 + (1.0 - 3.0 * d0)) - ((cH == 0.0 || s2a == 0.0) ? 0.0 : cH / s2a);
    double sum = 0.0;
    for (int i = 1; i < Q15; ++i) sum += g[i];
    return cs2 / (1.0 - w[0]) * (sum + (0.5 + H) * Q - w[0] * B / (1.0 - cs2) + 0.5 * K * (B - B_prev));
}

/* ---------------------------------------------------------------------- */
/* Simulation state                                                        */
/* ---------------------------------------------------------------------- */
enum { L_AX, L_AY, L_AZ, L_B, L_CXX, L_CYY, L_CZZ, L_CXY, L_CYZ, L_CXZ, L_PX, L_PY, L_PZ, NLAG };
enum { F_PHI1, F_LAP0, F_GX0, F_GY0, F_GZ0, F_LAP1, F_GX1, F_GY1, F_GZ1, F_MU0, F_MU1, F_MU2, F_MUB,
       F_GMX, F_GMY, F_GMZ, F_UX, F_UY, F_UZ, F_P, NF };

typedef struct {
    orc3_params P;
    int n[3];
    size_t N;
    double k, gamma[3], eta;
    double* phi0;
    double* fpost;   /* [15][N] */
    double* gpost;
    double* lag;     /* [NLAG][N] */
    double* lag_new;
    double* f;       /* streamed */
    double* g;
    double* fld;     /* [NF][N] */
    double M0[Q15 * Q15], M0inv[Q15 * Q15], N_H[Q15 * Q15], Ninv[Q15 * Q15], Sphi[Q15 * Q15];
    double ws[Q15];  /* stencil weights (D3Q15 at d0 = 1/3), reading R2' */
    int64_t step;
} orc3_sim;

#define FLD3(s, k) ((s)->fld + (size_t)(k) * (s)->N)
#define IDX3(s, x, y, z) (((size_t)(z) * (s)->n[1] + (y)) * (s)->n[0] + (x))

static int wrap_or_mirror3(int j, int n, int periodic)
{
    if (periodic) { j %= n; if (j < 0) j += n; return j; }
    if (j < 0) return -1 - j;
    if (j >= n) return 2 * n - 1 - j;
    return j;
}

/* isotropic central gradient sum_i w_i c_i a(x + c_i)/c_s^2 and Laplacian
 * 2 sum_i w_i (a(x + c_i) - a(x))/c_s^2 with the D3Q15 weights at d0 = 1/3 */
static void stencil3(const orc3_sim* s, const double* a, int x, int y, int z, double g[3], double* lap)
{
    const double cs2 = 1.0 / 3.0;
    double a0 = a[IDX3(s, x, y, z)], gx = 0, gy = 0, gz = 0, l = 0;
    for (int i = 1; i < Q15; ++i) {
        int xx = wrap_or_mirror3(x + C3[i][0], s->n[0], s->P.periodic[0]);
        int yy = wrap_or_mirror3(y + C3[i][1], s->n[1], s->P.periodic[1]);
        int zz = wrap_or_mirror3(z + C3[i][2], s->n[2], s->P.periodic[2]);
        double v = a[IDX3(s, xx, yy, zz)];
        gx += s->ws[i] * C3[i][0] * v;
        gy += s->ws[i] * C3[i][1] * v;
        gz += s->ws[i] * C3[i][2] * v;
        l += s->ws[i] * (v - a0);
    }
    if (g) { g[0] = gx / cs2; g[1] = gy / cs2; g[2] = gz / cs2; }
    if (lap) *lap = 2.0 * l / cs2;
}

static void stream3(orc3_sim* s)
{
    int nx = s->n[0], ny = s->n[1], nz = s->n[2];
    size_t N = s->N;
#pragma omp parallel for collapse(2) if ((size_t)nx * ny * nz >= ORC_PAR_MIN)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t id = IDX3(s, x, y, z);
                for (int i = 0; i < Q15; ++i) {
                    int src[3] = {x - C3[i][0], y - C3[i][1], z - C3[i][2]};
                    int out = 0;
                    for (int a = 0; a < 3; ++a) {
                        if (s->P.periodic[a]) src[a] = (src[a] % s->n[a] + s->n[a]) % s->n[a];
                        else if (src[a] < 0 || src[a] >= s->n[a]) out = 1;
                    }
                    if (out) {
                        int o = opposite(i);
                        s->f[(size_t)i * N + id] = s->fpost[(size_t)o * N + id];
                        s->g[(size_t)i * N + id] = s->gpost[(size_t)o * N + id];
                    } else {
                        size_t sid = IDX3(s, src[0], src[1], src[2]);
                        s->f[(size_t)i * N + id] = s->fpost[(size_t)i * N + sid];
                        s->g[(size_t)i * N + id] = s->gpost[(size_t)i * N + sid];
                    }
                }
            }
}

static void chem3(const double gamma[3], double D, double phi0, double phi1, double lap0, double lap1,
                  double mu[3], double* mub1)
{
    double phi[3] = {phi0, phi1, 1.0 - phi0 - phi1};
    double lap[3] = {lap0, lap1, -lap0 - lap1};
    for (int p = 0; p < 3; ++p)
        mu[p] = 12.0 / D * gamma[p] * phi[p] * (1.0 - phi[p]) * (1.0 - 2.0 * phi[p]) - 0.75 * D * gamma[p] * lap[p];
    double gT = 3.0 / (1.0 / gamma[0] + 1.0 / gamma[1] + 1.0 / gamma[2]);
    *mub1 = gT / 3.0 * ((mu[1] - mu[0]) / gamma[0] + (mu[1] - mu[2]) / gamma[2]);
}

static double visc_rate3(double mu_v, double rho, double phi0, double cfac)
{
    return (1.0 - phi0) / (mu_v / (rho * cfac) + 0.5 * (1.0 - phi0));
}

static void macro_and_collide3(orc3_sim* s, int collide)
{
    const orc3_params* P = &s->P;
    int nx = s->n[0], ny = s->n[1], nz = s->n[2];
    size_t N = s->N;
    double cs2 = P->d0;

#pragma omp parallel for if ((size_t)nx * ny * nz >= ORC_PAR_MIN)
    for (size_t id = 0; id < N; ++id) {
        double sum = 0.0;
        for (int i = 0; i < Q15; ++i) sum += s->f[(size_t)i * N + id];
        FLD3(s, F_PHI1)[id] = sum;
    }
#pragma omp parallel for collapse(2) if ((size_t)nx * ny * nz >= ORC_PAR_MIN)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t id = IDX3(s, x, y, z);
                double g0[3], g1[3];
                stencil3(s, s->phi0, x, y, z, g0, &FLD3(s, F_LAP0)[id]);
                stencil3(s, FLD3(s, F_PHI1), x, y, z, g1, &FLD3(s, F_LAP1)[id]);
                FLD3(s, F_GX0)[id] = g0[0]; FLD3(s, F_GY0)[id] = g0[1]; FLD3(s, F_GZ0)[id] = g0[2];
                FLD3(s, F_GX1)[id] = g1[0]; FLD3(s, F_GY1)[id] = g1[1]; FLD3(s, F_GZ1)[id] = g1[2];
            }
#pragma omp parallel for if ((size_t)nx * ny * nz >= ORC_PAR_MIN)
    for (size_t id = 0; id < N; ++id) {
        double mu[3], mub;
        chem3(s->gamma, P->D, s->phi0[id], FLD3(s, F_PHI1)[id], FLD3(s, F_LAP0)[id], FLD3(s, F_LAP1)[id], mu, &mub);
        FLD3(s, F_MU0)[id] = mu[0];
        FLD3(s, F_MU1)[id] = mu[1];
        FLD3(s, F_MU2)[id] = mu[2];
        FLD3(s, F_MUB)[id] = mub;
    }
#pragma omp parallel for collapse(2) if ((size_t)nx * ny * nz >= ORC_PAR_MIN)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t id = IDX3(s, x, y, z);
                double gm[3];
                stencil3(s, FLD3(s, F_MUB), x, y, z, gm, NULL);
                FLD3(s, F_GMX)[id] = gm[0]; FLD3(s, F_GMY)[id] = gm[1]; FLD3(s, F_GMZ)[id] = gm[2];
            }

    const double* lag = s->lag;
    double* lnew = s->lag_new;
    double rho0 = P->rho[0], rho1 = P->rho[1], rho2 = P->rho[2];
#pragma omp parallel for collapse(2) if ((size_t)nx * ny * nz >= ORC_PAR_MIN)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t id = IDX3(s, x, y, z);
                double phi0 = s->phi0[id], phi1 = FLD3(s, F_PHI1)[id];
                double mu0 = FLD3(s, F_MU0)[id], mu1 = FLD3(s, F_MU1)[id], mu2 = FLD3(s, F_MU2)[id];
                double mub = FLD3(s, F_MUB)[id];
                double g0[3] = {FLD3(s, F_GX0)[id], FLD3(s, F_GY0)[id], FLD3(s, F_GZ0)[id]};
                double g1[3] = {FLD3(s, F_GX1)[id], FLD3(s, F_GY1)[id], FLD3(s, F_GZ1)[id]};
                double gm[3] = {FLD3(s, F_GMX)[id], FLD3(s, F_GMY)[id], FLD3(s, F_GMZ)[id]};

                /* degenerate mobility, 2f1s form (Sec. 4) */
                double fdeg = phi1 * (1.0 - phi1) * (1.0 - phi0);
                double Mob = P->M_cst + P->M_deg * fdeg;
                double a = P->M_deg * (1.0 - fdeg) / (P->M_cst + P->M_deg);
                double phi2 = 1.0 - phi0 - phi1;
                double rho = rho0 * phi0 + rho1 * phi1 + rho2 * phi2;
                double mu_v = P->mu[0] * phi0 + P->mu[1] * phi1 + P->mu[2] * phi2;
                double dr[3], S[3], F[3];
                for (int k = 0; k < 3; ++k) {
                    dr[k] = (rho0 - rho2) * g0[k] + (rho1 - rho2) * g1[k];
                    S[k] = (rho1 - rho2) * Mob / s->gamma[1] * gm[k];
                    /* F_s = sum_p mu_p grad(phi_p), grad(phi2) = -grad(phi0) - grad(phi1) */
                    F[k] = mu0 * g0[k] + mu1 * g1[k] + mu2 * (-g0[k] - g1[k]) + P->Fb[k];
                }
                /* F_c = -curl(psi)/2 from the previous step's psi = S x u (reading R5') */
                double dpx[3], dpy[3], dpz[3];
                stencil3(s, lag + (size_t)L_PX * N, x, y, z, dpx, NULL);
                stencil3(s, lag + (size_t)L_PY * N, x, y, z, dpy, NULL);
                stencil3(s, lag + (size_t)L_PZ * N, x, y, z, dpz, NULL);
                F[0] += -0.5 * (dpz[1] - dpy[2]);
                F[1] += -0.5 * (dpx[2] - dpz[0]);
                F[2] += -0.5 * (dpy[0] - dpx[1]);

                /* velocity with the solid force f = (u_w - u*)/dt (Sec. 3) */
                double gl[Q15];
                for (int i = 0; i < Q15; ++i) gl[i] = s->g[(size_t)i * N + id];
                double j[3] = {0, 0, 0};
                for (int i = 0; i < Q15; ++i)
                    for (int k = 0; k < 3; ++k) j[k] += C3[i][k] * gl[i];
                double us[3], fs[3], u[3], G[3];
                for (int k = 0; k < 3; ++k) {
                    us[k] = (j[k] + 0.5 * F[k]) / rho;
                    fs[k] = P->u_wall[k] - us[k];
                    u[k] = us[k] + 0.5 * phi0 * fs[k];
                    G[k] = F[k] + phi0 * rho * fs[k];
                }
                double s2a = visc_rate3(mu_v, rho, phi0, 0.5 * (1.0 - cs2));
                double s2b = visc_rate3(mu_v, rho, phi0, cs2);
                double Qg = u[0] * dr[0] + u[1] * dr[1] + u[2] * dr[2];
                double B = 0.0;
                for (int k = 0; k < 3; ++k) B += (rho * u[k] - S[k]) * u[k];
                double p = orc3_pressure(P->d0, P->s_g[0], s2a, gl, Qg, B, lag[(size_t)L_B * N + id]);
                FLD3(s, F_UX)[id] = u[0];
                FLD3(s, F_UY)[id] = u[1];
                FLD3(s, F_UZ)[id] = u[2];
                FLD3(s, F_P)[id] = p;
                if (!collide) continue;

                /* CH collision */
                double A[3] = {phi1 * u[0], phi1 * u[1], phi1 * u[2]};
                double dA[3], eg[3];
                for (int k = 0; k < 3; ++k) {
                    dA[k] = A[k] - lag[(size_t)(L_AX + k) * N + id];
                    eg[k] = s->eta * gm[k];
                }
                double fl[Q15], feq[Q15], R[Q15], fo[Q15];
                for (int i = 0; i < Q15; ++i) fl[i] = s->f[(size_t)i * N + id];
                orc3_feq(P->d0, phi1, s->eta * mub, A, feq);
                orc3_Rpop(P->d0, dA, a, eg, R);
                collide_with(s->M0, s->M0inv, s->Sphi, fl, feq, R, fo);
                for (int i = 0; i < Q15; ++i) s->fpost[(size_t)i * N + id] = fo[i];

                /* NS collision: C = sym(S u); M2F = uF + Fu - d_t C
                 *   + c_s^2 (u grad rho + grad rho u) + (c^2 - 3 c_s^2)(u . grad rho) I */
                double Cn[6] = {S[0] * u[0], S[1] * u[1], S[2] * u[2], 0.5 * (S[0] * u[1] + S[1] * u[0]),
                                0.5 * (S[1] * u[2] + S[2] * u[1]), 0.5 * (S[0] * u[2] + S[2] * u[0])};
                const int pa[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {1, 2}, {0, 2}};
                double M2[6];
                for (int k = 0; k < 6; ++k) {
                    int a1 = pa[k][0], a2 = pa[k][1];
                    M2[k] = u[a1] * F[a2] + F[a1] * u[a2] - (Cn[k] - lag[(size_t)(L_CXX + k) * N + id]) +
                            cs2 * (u[a1] * dr[a2] + dr[a1] * u[a2]) + (a1 == a2 ? (1.0 - 3.0 * cs2) * Qg : 0.0);
                }
                double geq[Q15], Fp[Q15], go[Q15];
                orc3_geq(P->d0, P->rho_gauge, p, rho, u, S, geq);
                orc3_Fpop(P->d0, Qg, G, M2, Fp);
                double Kg[Q15] = {P->s_g[0], P->s_g[1], P->s_g[1], P->s_g[1], s2a, s2a, s2a, s2b, s2b, s2b,
                                  P->s_g[2], P->s_g[2], P->s_g[2], P->s_g[2], P->s_g[3]};
                double KN[Q15 * Q15], Sg[Q15 * Q15];
                for (int r = 0; r < Q15; ++r)
                    for (int c = 0; c < Q15; ++c) KN[r * Q15 + c] = Kg[r] * s->N_H[r * Q15 + c];
                matmul15(s->Ninv, KN, Sg);
                collide_with(s->M0, s->M0inv, Sg, gl, geq, Fp, go);
                for (int i = 0; i < Q15; ++i) s->gpost[(size_t)i * N + id] = go[i];

                for (int k = 0; k < 3; ++k) lnew[(size_t)(L_AX + k) * N + id] = A[k];
                lnew[(size_t)L_B * N + id] = B;
                for (int k = 0; k < 6; ++k) lnew[(size_t)(L_CXX + k) * N + id] = Cn[k];
                lnew[(size_t)L_PX * N + id] = S[1] * u[2] - S[2] * u[1];
                lnew[(size_t)L_PY * N + id] = S[2] * u[0] - S[0] * u[2];
                lnew[(size_t)L_PZ * N + id] = S[0] * u[1] - S[1] * u[0];
            }
    if (collide) memcpy(s->lag, s->lag_new, (size_t)NLAG * N * sizeof(double));
}

/* ---------------------------------------------------------------------- */
/* Entry points                                                            */
/* ---------------------------------------------------------------------- */
static double sgn3(double x) { return (x > 0.0) - (x < 0.0); }

orc3_sim* orc3_create(const orc3_params* P, const double* phi0, const double* phi1)
{
    orc3_sim* s = (orc3_sim*)calloc(1, sizeof(orc3_sim));
    s->P = *P;
    s->n[0] = P->nx; s->n[1] = P->ny; s->n[2] = P->nz;
    s->N = (size_t)P->nx * P->ny * P->nz;
    /* spreading factor, Young's law and gamma_p (Sec. 2.1-2.2) */
    double sn = sin(0.25 * M_PI * cos(P->theta));
    s->k = 9.0 / (1.0 + P->kappa) * (1.0 + 2.0 * sgn3(P->theta - 0.5 * M_PI) * sn * sn);
    double s01 = s->k * P->sigma12, s02 = s01 + P->sigma12 * cos(P->theta), s12 = P->sigma12;
    s->gamma[0] = s01 + s02 - s12;
    s->gamma[1] = s01 + s12 - s02;
    s->gamma[2] = s02 + s12 - s01;
    if (!(s->gamma[0] > 0 && s->gamma[1] > 0 && s->gamma[2] > 0)) { free(s); return NULL; }
    /* (M_cst + M_deg)/gamma_1 = (1/s1 - 1/2) eta c_s^2  (reading R1) */
    s->eta = (P->M_cst + P->M_deg) / (s->gamma[1] * (P->tau_phi - 0.5) * P->d0);
    size_t N = s->N;
    s->phi0 = (double*)malloc(N * sizeof(double));
    s->fpost = (double*)malloc(Q15 * N * sizeof(double));
    s->gpost = (double*)malloc(Q15 * N * sizeof(double));
    s->f = (double*)malloc(Q15 * N * sizeof(double));
    s->g = (double*)malloc(Q15 * N * sizeof(double));
    s->lag = (double*)calloc((size_t)NLAG * N, sizeof(double));
    s->lag_new = (double*)calloc((size_t)NLAG * N, sizeof(double));
    s->fld = (double*)calloc((size_t)NF * N, sizeof(double));
    orc3_M0(s->M0);
    orc3_inverse(Q15, s->M0, s->M0inv);
    orc3_N(P->d0, s->N_H);
    orc3_inverse(Q15, s->N_H, s->Ninv);
    orc3_weights(1.0 / 3.0, s->ws);
    {
        double s1 = 1.0 / P->tau_phi;
        double Kphi[Q15] = {P->s_phi[0], s1, s1, s1, P->s_phi[1], P->s_phi[1], P->s_phi[1], P->s_phi[1],
                            P->s_phi[1], P->s_phi[1], P->s_phi[2], P->s_phi[2], P->s_phi[2], P->s_phi[2],
                            P->s_phi[3]};
        orc3_relaxation_matrix(P->d0, Kphi, s->Sphi);
    }
    memcpy(s->phi0, phi0, N * sizeof(double));
    memcpy(FLD3(s, F_PHI1), phi1, N * sizeof(double));
    /* initial state (reading R9): f = f^eq(phi1, mubar1, u = 0), g = g^eq(P = 0, u = 0) */
    for (int z = 0; z < s->n[2]; ++z)
        for (int y = 0; y < s->n[1]; ++y)
            for (int x = 0; x < s->n[0]; ++x) {
                size_t id = IDX3(s, x, y, z);
                stencil3(s, s->phi0, x, y, z, NULL, &FLD3(s, F_LAP0)[id]);
                stencil3(s, FLD3(s, F_PHI1), x, y, z, NULL, &FLD3(s, F_LAP1)[id]);
            }
    for (size_t id = 0; id < N; ++id) {
        double mu[3], mub, feq[Q15], geq[Q15], zero[3] = {0, 0, 0};
        chem3(s->gamma, P->D, phi0[id], phi1[id], FLD3(s, F_LAP0)[id], FLD3(s, F_LAP1)[id], mu, &mub);
        orc3_feq(P->d0, phi1[id], s->eta * mub, zero, feq);
        orc3_geq(P->d0, P->rho_gauge, 0.0, 1.0, zero, zero, geq);
        for (int i = 0; i < Q15; ++i) {
            s->fpost[(size_t)i * N + id] = feq[i];
            s->gpost[(size_t)i * N + id] = geq[i];
        }
    }
    return s;
}

void orc3_free(orc3_sim* s)
{
    if (!s) return;
    free(s->phi0); free(s->fpost); free(s->gpost); free(s->f); free(s->g);
    free(s->lag); free(s->lag_new); free(s->fld); free(s);
}

void orc3_step(orc3_sim* s, int64_t nsteps)
{
    for (int64_t k = 0; k < nsteps; ++k) {
        stream3(s);
        macro_and_collide3(s, 1);
        s->step++;
    }
}

void orc3_moments(orc3_sim* s, double* phi1, double* ux, double* uy, double* uz, double* p)
{
    stream3(s);
    macro_and_collide3(s, 0);
    size_t N = s->N;
    if (phi1) memcpy(phi1, FLD3(s, F_PHI1), N * sizeof(double));
    if (ux) memcpy(ux, FLD3(s, F_UX), N * sizeof(double));
    if (uy) memcpy(uy, FLD3(s, F_UY), N * sizeof(double));
    if (uz) memcpy(uz, FLD3(s, F_UZ), N * sizeof(double));
    if (p) memcpy(p, FLD3(s, F_P), N * sizeof(double));
}

void orc3_aux(orc3_sim* s, double* mub, double* gm)
{
    stream3(s);
    macro_and_collide3(s, 0);
    size_t N = s->N;
    if (mub) memcpy(mub, FLD3(s, F_MUB), N * sizeof(double));
    if (gm) {
        memcpy(gm, FLD3(s, F_GMX), N * sizeof(double));
        memcpy(gm + N, FLD3(s, F_GMY), N * sizeof(double));
        memcpy(gm + 2 * N, FLD3(s, F_GMZ), N * sizeof(double));
    }
}

double orc3_mass(const orc3_sim* s)
{
    long double m = 0.0L;
    for (size_t k = 0; k < Q15 * s->N; ++k) m += s->fpost[k];
    return (double)m;
}

int64_t orc3_step_count(const orc3_sim* s) { return s->step; }

void orc3_get_state(const orc3_sim* s, double* f, double* g, double* lag)
{
    size_t N = s->N;
    if (f) memcpy(f, s->fpost, Q15 * N * sizeof(double));
    if (g) memcpy(g, s->gpost, Q15 * N * sizeof(double));
    if (lag) memcpy(lag, s->lag, (size_t)NLAG * N * sizeof(double));
}

void orc3_set_state(orc3_sim* s, const double* f, const double* g, const double* lag)
{
    size_t N = s->N;
    if (f) memcpy(s->fpost, f, Q15 * N * sizeof(double));
    if (g) memcpy(s->gpost, g, Q15 * N * sizeof(double));
    if (lag) memcpy(s->lag, lag, (size_t)NLAG * N * sizeof(double));
}

void orc3_derived(const orc3_sim* s, double* k, double gamma3[3], double* eta)
{
    if (k) *k = s->k;
    if (gamma3) memcpy(gamma3, s->gamma, 3 * sizeof(double));
    if (eta) *eta = s->eta;
}
