/*
 * Plain FP64 CPU oracle of the coupled ternary phase-field lattice Boltzmann
 * step of Zhan, Chai & Shi, "A ternary phase-field model for two-phase flows
 * in complex geometries" (arXiv 2311.05091), 2f1s model ("two fluids, one
 * solid") on the D2Q9 lattice with the Hermite-moment collision.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no source with the GPU library.
 *
 * It is written to be checked against the paper by eye, not to be fast:
 *   - the collision uses the dense 9x9 matrices M0 and N of Appendix A and
 *     the relaxation matrix S = N^-1 K N of Sec. 4 (C_d = I since c = 1),
 *     with N^-1 and M0^-1 obtained by Gauss-Jordan elimination at start-up;
 *   - every equilibrium and source population is formed per direction
 *     exactly as printed in Sec. 3 and transformed with M0;
 *   - each field is computed over the whole grid in its own pass, in the
 *     order in which the paper defines it.
 * Lattice units throughout: c = dx = dt = 1.
 *
 * Readings of passages the paper leaves open:
 *   R1  eta is derived from the CH relaxation time tau_phi = 1/s1 through
 *       (M_cst+M_deg)/gamma_1 = (1/s1 - 1/2) eta c_s^2 (Sec. 3).
 *   R2  gradients and Laplacians use the standard isotropic 9-point central
 *       stencils (weights 4/9, 1/9, 1/36 and c_s^2 = 1/3), independent of d0.
 *   R3  scalar values across a no-flux wall are even mirrors of the interior
 *       (the wall sits half-way between nodes).
 *   R4  2f1s flux: J0 = 0, J2 = -J1, so S = (rho1 - rho2) M grad(mubar1)/gamma1
 *       with the degenerate mobility M = M_cst + M_deg f(phi).
 *   R5  the correction force F_c = div(Su - uS)/2 is evaluated from the
 *       previous step's psi = S_x u_y - S_y u_x (it is implicit in u otherwise).
 *   R6  explicit-Euler time derivatives start from zero lagged values.
 *   R7  d_t(rho u u) ~ uF + Fu uses F = F_s + F_b + F_c (without phi0 rho f).
 *   R8  the constant in lambda_0 is a gauge rho_gauge (default 0), not the
 *       solid density.
 *   R9  initial populations: f = f^eq(phi1, mubar1, u = 0), g = g^eq(P = 0,
 *       u = 0); they are taken as post-collision values of step -1.
 *   R10 the per-node NS rates are written s = (1-phi0)/(mu/(rho c) + (1-phi0)/2),
 *       identical to the viscosity relation of Sec. 3 for phi0 < 1 and finite
 *       (s -> 0) at phi0 = 1.
 *   R11 in the 2D pressure constant H the term (2 - 4 d0)/s2a is taken as zero
 *       where its coefficient is zero (d0 = 1/2) and where s2a = 0 (a saturated
 *       solid node, phi0 = 1: its second-order NS moments do not relax, and
 *       the relation for p holds no finite value of the term).
 *   R27 open boundaries (Sec. 4 names non-equilibrium extrapolation for
 *       velocity and pressure boundaries): applied after the collision to
 *       the inlet column x = 0 and outlet column x = nx - 1 with the inner
 *       neighbour's non-equilibrium part (see open_boundaries).
 *   R19 the solid-point velocity u_w of f = (u_w - u*)/dt (Sec. 3) is that of a
 *       rigid body: u_w(x) = u_wall + omega_wall e_z x (x - wall_center), with
 *       the solid field phi0 held fixed (a solid whose shape is invariant under
 *       its own motion: a sliding plate, a spinning cylinder).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* grids below this many nodes run each pass on one thread (the per-pass
 * thread start-up would cost more than the pass) */
#define ORC_PAR_MIN 8192

/* ---------------------------------------------------------------------- */
/* Parameters (own definition; the GPU library has its own).               */
/* ---------------------------------------------------------------------- */
typedef struct {
    int32_t nx, ny;
    int32_t periodic_x, periodic_y;
    double d0;          /* scale factor, c_s^2 = d0 (Sec. 3, App. A)      */
    double D;           /* interface thickness                            */
    double sigma12;     /* fluid-fluid surface tension                    */
    double theta;       /* contact angle of fluid 1 on the solid [rad]   */
    double kappa;       /* minimum dimensionless solid curvature          */
    double rho[3];      /* densities of phase 0 (solid), 1, 2             */
    double mu[3];       /* dynamic viscosities of phase 0, 1, 2           */
    double M_cst, M_deg;
    double tau_phi;     /* 1/s1 of the CH lattice                         */
    double s_phi[4];    /* s0, s2, s3, s4 of the CH lattice               */
    double s_g[4];      /* s0, s1, s3, s4 of the NS lattice               */
    double Fb[2];       /* body force                                     */
    double u_wall[2];   /* translation of the solid                       */
    double omega_wall;  /* angular velocity of the solid about wall_center */
    double wall_center[2];
    double rho_gauge;   /* constant in lambda_0                           */
    int32_t open_x;     /* 1: inlet at x = 0, outlet at x = nx - 1 (R27)  */
    int32_t inlet_type; /* 0: pressure p_in, 1: velocity (u_in, 0)        */
    double p_in, u_in, p_out;
    double phi1_in;     /* phase-1 share of the fluid entering (x (1 - phi0)) */
} orc_params;

typedef struct {
    double k;                 /* sigma01 / sigma12, Eq. (eq-kk)          */
    double sigma01, sigma02;  /* Young's law                             */
    double gamma[3];          /* spreading coefficients                  */
    double gammaT;            /* 3/gammaT = sum 1/gamma_p                */
    double eta;               /* CH equilibrium parameter                */
    double cs2;               /* lattice sound speed squared = d0        */
    double w[9];              /* D2Q9 weights                            */
    double Kp;                /* pressure constant K = 1 - d0 (2D)       */
} orc_derived;

/* D2Q9 velocities in the order fixed by the rows of M0 (App. A). */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

/* ---------------------------------------------------------------------- */
/* Lattice algebra (App. A)                                               */
/* ---------------------------------------------------------------------- */
void orc_velocities(int32_t cx[9], int32_t cy[9])
{
    for (int i = 0; i < 9; ++i) { cx[i] = CX[i]; cy[i] = CY[i]; }
}

void orc_weights(double d0, double w[9])
{
    w[0] = 1.0 - 2.0 * d0 + d0 * d0;
    for (int i = 1; i <= 4; ++i) w[i] = (d0 - d0 * d0) / 2.0;
    for (int i = 5; i <= 8; ++i) w[i] = d0 * d0 / 4.0;
}

/* M0: rows 1, cx, cy, cx^2, cy^2, cx cy, cx cy^2, cx^2 cy, cx^2 cy^2. */
void orc_M0(double M0[81])
{
    for (int i = 0; i < 9; ++i) {
        double x = CX[i], y = CY[i];
        M0[0 * 9 + i] = 1.0;
        M0[1 * 9 + i] = x;
        M0[2 * 9 + i] = y;
        M0[3 * 9 + i] = x * x;
        M0[4 * 9 + i] = y * y;
        M0[5 * 9 + i] = x * y;
        M0[6 * 9 + i] = x * y * y;
        M0[7 * 9 + i] = x * x * y;
        M0[8 * 9 + i] = x * x * y * y;
    }
}

/* N: the lower-triangular matrix of App. A (D2Q9). */
void orc_N(double cs2, double N[81])
{
    memset(N, 0, 81 * sizeof(double));
    for (int i = 0; i < 9; ++i) N[i * 9 + i] = 1.0;
    N[3 * 9 + 0] = -cs2;
    N[4 * 9 + 0] = -cs2;
    N[6 * 9 + 1] = -cs2;
    N[7 * 9 + 2] = -cs2;
    N[8 * 9 + 0] = cs2 * cs2;
    N[8 * 9 + 3] = -cs2;
    N[8 * 9 + 4] = -cs2;
}

/* Gauss-Jordan inverse with partial pivoting; returns 0 on success. */
int orc_inverse9(const double A[81], double Ainv[81])
{
    double a[9][18];
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 18; ++c)
            a[r][c] = c < 9 ? A[r * 9 + c] : (c - 9 == r ? 1.0 : 0.0);
    for (int col = 0; col < 9; ++col) {
        int piv = col;
        for (int r = col + 1; r < 9; ++r)
            if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
        if (fabs(a[piv][col]) < 1e-300) return -1;
        if (piv != col)
            for (int c = 0; c < 18; ++c) { double t = a[col][c]; a[col][c] = a[piv][c]; a[piv][c] = t; }
        double p = a[col][col];
        for (int c = 0; c < 18; ++c) a[col][c] /= p;
        for (int r = 0; r < 9; ++r) {
            if (r == col) continue;
            double m = a[r][col];
            if (m == 0.0) continue;
            for (int c = 0; c < 18; ++c) a[r][c] -= m * a[col][c];
        }
    }
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 9; ++c) Ainv[r * 9 + c] = a[r][c + 9];
    return 0;
}

static void matmul9(const double A[81], const double B[81], double C[81])
{
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 9; ++c) {
            double s = 0.0;
            for (int k = 0; k < 9; ++k) s += A[r * 9 + k] * B[k * 9 + c];
            C[r * 9 + c] = s;
        }
}

static void matvec9(const double A[81], const double x[9], double y[9])
{
    for (int r = 0; r < 9; ++r) {
        double s = 0.0;
        for (int k = 0; k < 9; ++k) s += A[r * 9 + k] * x[k];
        y[r] = s;
    }
}

/* S = N^-1 K N (Sec. 4), K = diag(Kdiag). */
void orc_relaxation_matrix(double cs2, const double Kdiag[9], double S[81])
{
    double N[81], Ninv[81], KN[81];
    orc_N(cs2, N);
    orc_inverse9(N, Ninv);
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 9; ++c) KN[r * 9 + c] = Kdiag[r] * N[r * 9 + c];
    matmul9(Ninv, KN, S);
}

/* MRT collision in natural-moment space (Sec. 4) with given M0, M0^-1, S:
 *   m = M0 f,  m* = m - S (m - m_eq) + (I - S/2) M0 R,  f* = M0^-1 m*. */
void orc_collide_with(const double M0[81], const double M0inv[81], const double S[81],
                         const double f[9], const double feq[9], const double R[9], double fout[9])
{
    double m[9], meq[9], mR[9], d[9], Sd[9], SR[9], ms[9];
    matvec9(M0, f, m);
    matvec9(M0, feq, meq);
    matvec9(M0, R, mR);
    for (int k = 0; k < 9; ++k) d[k] = m[k] - meq[k];
    matvec9(S, d, Sd);
    matvec9(S, mR, SR);
    for (int k = 0; k < 9; ++k) ms[k] = m[k] - Sd[k] + mR[k] - 0.5 * SR[k];
    matvec9(M0inv, ms, fout);
}

/* Same collision, building M0, M0^-1 and S = N^-1 K N from scratch. */
void orc_collide(double cs2, const double Kdiag[9], const double f[9],
                 const double feq[9], const double R[9], double fout[9])
{
    double M0[81], M0inv[81], S[81];
    orc_M0(M0);
    orc_inverse9(M0, M0inv);
    orc_relaxation_matrix(cs2, Kdiag, S);
    orc_collide_with(M0, M0inv, S, f, feq, R, fout);
}

/* ---------------------------------------------------------------------- */
/* Model parameters (Sec. 2.1-2.2, Sec. 3)                                 */
/* ---------------------------------------------------------------------- */
static double sgn(double x) { return (x > 0.0) - (x < 0.0); }

/* Spreading factor k(theta, kappa), Eq. (eq-kk). */
double orc_spreading_factor(double theta, double kappa)
{
    double s = sin(0.25 * M_PI * cos(theta));
    return 9.0 / (1.0 + kappa) * (1.0 + 2.0 * sgn(theta - 0.5 * M_PI) * s * s);
}

int orc_derive(const orc_params* P, orc_derived* d)
{
    d->k = orc_spreading_factor(P->theta, P->kappa);
    /* sigma01 = k sigma12; Young's law sigma02 = sigma01 + sigma12 cos(theta) */
    d->sigma01 = d->k * P->sigma12;
    d->sigma02 = d->sigma01 + P->sigma12 * cos(P->theta);
    /* spreading coefficients from the pairwise tensions (Sec. 2.1) */
    d->gamma[0] = d->sigma01 + d->sigma02 - P->sigma12;
    d->gamma[1] = d->sigma01 + P->sigma12 - d->sigma02;
    d->gamma[2] = d->sigma02 + P->sigma12 - d->sigma01;
    d->gammaT = 3.0 / (1.0 / d->gamma[0] + 1.0 / d->gamma[1] + 1.0 / d->gamma[2]);
    d->cs2 = P->d0;
    orc_weights(P->d0, d->w);
    /* (M_cst + M_deg)/gamma_1 = (1/s1 - 1/2) eta c_s^2   (reading R1) */
    d->eta = (P->M_cst + P->M_deg) / (d->gamma[1] * (P->tau_phi - 0.5) * d->cs2);
    d->Kp = 1.0 - P->d0;
    return (d->gamma[0] > 0 && d->gamma[1] > 0 && d->gamma[2] > 0) ? 0 : -1;
}

/* ---------------------------------------------------------------------- */
/* Pointwise physics                                                       */
/* ---------------------------------------------------------------------- */
/* Chemical potentials mu_p (Sec. 2.1) and the Lagrange-corrected mubar_p
 * (Eq. eq-CHmodel) for all three phases; phi2 = 1 - phi0 - phi1. */
void orc_chemical_potentials(const double gamma[3], double D,
                             double phi0, double phi1, double lap0, double lap1,
                             double mu_out[3], double mubar_out[3])
{
    double phi[3] = {phi0, phi1, 1.0 - phi0 - phi1};
    double lap[3] = {lap0, lap1, -lap0 - lap1};
    for (int p = 0; p < 3; ++p) {
        /* d f_b / d phi_p = (12/D) gamma_p phi (1 - phi)(1 - 2 phi) */
        double dfb = 12.0 / D * gamma[p] * phi[p] * (1.0 - phi[p]) * (1.0 - 2.0 * phi[p]);
        mu_out[p] = dfb - 0.75 * D * gamma[p] * lap[p];
    }
    double gT = 3.0 / (1.0 / gamma[0] + 1.0 / gamma[1] + 1.0 / gamma[2]);
    for (int p = 0; p < 3; ++p) {
        double s = 0.0;
        for (int q = 0; q < 3; ++q)
            if (q != p) s += (mu_out[p] - mu_out[q]) / gamma[q];
        mubar_out[p] = gT / 3.0 * s;
    }
}

/* CH equilibrium (Sec. 3): eta_mub = eta * mubar, (Ax, Ay) = phi u. */
void orc_feq(double d0, double phi, double eta_mub, double Ax, double Ay, double feq[9])
{
    double w[9], cs2 = d0;
    orc_weights(d0, w);
    feq[0] = phi + (w[0] - 1.0) * eta_mub;
    for (int i = 1; i < 9; ++i)
        feq[i] = w[i] * eta_mub + w[i] * (CX[i] * Ax + CY[i] * Ay) / cs2;
}

/* CH source (Sec. 3): dAx, dAy = d_t(phi u); a = M_deg (1-f)/(M_cst+M_deg);
 * eta_gx, eta_gy = eta grad(mubar). */
void orc_Rpop(double d0, double dAx, double dAy, double a, double eta_gx, double eta_gy,
              double R[9])
{
    double w[9], cs2 = d0;
    orc_weights(d0, w);
    for (int i = 0; i < 9; ++i)
        R[i] = w[i] * ((CX[i] * dAx + CY[i] * dAy) / cs2 + a * (CX[i] * eta_gx + CY[i] * eta_gy));
}

/* NS equilibrium (Sec. 3) with c = 1. */
void orc_geq(double d0, double rho_gauge, double P, double rho, double ux, double uy,
             double Sx, double Sy, double geq[9])
{
    double w[9], cs2 = d0;
    orc_weights(d0, w);
    double Pixx = rho * ux * ux - Sx * ux;
    double Piyy = rho * uy * uy - Sy * uy;
    double Pixy = rho * ux * uy - 0.5 * (Sx * uy + ux * Sy);
    for (int i = 0; i < 9; ++i) {
        double lam = (i == 0) ? (w[0] - 1.0) * P / cs2 + rho_gauge : w[i] * P / cs2;
        double cu = CX[i] * rho * ux + CY[i] * rho * uy;
        double diag = (CX[i] * CX[i] - cs2) * Pixx + (CY[i] * CY[i] - cs2) * Piyy;
        geq[i] = lam + w[i] * cu / cs2
               + w[i] * (diag / (cs2 - cs2 * cs2) + CX[i] * CY[i] * Pixy / (cs2 * cs2));
    }
}

/* NS force populations (Sec. 3): Q = u.grad(rho), (Gx, Gy) = F + phi0 rho f,
 * M2 = (Mxx, Myy, Mxy). */
void orc_Fpop(double d0, double Q, double Gx, double Gy, double Mxx, double Myy, double Mxy,
              double F[9])
{
    double w[9], cs2 = d0;
    orc_weights(d0, w);
    for (int i = 0; i < 9; ++i) {
        double diag = (CX[i] * CX[i] - cs2) * Mxx + (CY[i] * CY[i] - cs2) * Myy;
        F[i] = w[i] * (Q + (CX[i] * Gx + CY[i] * Gy) / cs2
                       + diag / (cs2 - cs2 * cs2) + CX[i] * CY[i] * Mxy / (cs2 * cs2));
    }
}

/* Pressure (Sec. 3, 2D constants K = 1 - d0 and H). */
double orc_pressure(double d0, double s0, double s2a, const double g[9], double u_grad_rho,
                    double B, double B_prev)
{
    double w[9], cs2 = d0;
    orc_weights(d0, w);
    double K = 1.0 - d0;
    /* the s2a term is zero where its coefficient (2 - 4 d0) is (d0 = 1/2) and
     * at a saturated solid node (phi0 = 1, s2a = 0), reading R11 */
    double cH = 2.0 - 4.0 * d0;
    double H = K * ((1.0 - d0) / s0 - ((cH == 0.0 || s2a == 0.0) ? 0.0 : cH / s2a) + (1.0 - 3.0 * d0) / 2.0);
    double sum = 0.0;
    for (int i = 1; i < 9; ++i) sum += g[i];
    return cs2 / (1.0 - w[0]) *
           (sum + (0.5 + H) * u_grad_rho - w[0] * B / (1.0 - cs2) + 0.5 * K * (B - B_prev));
}

/* Per-node NS relaxation rate for a viscosity relation with factor cfac
 * (cfac = (1 - c_s^2)/2 for s2a, c_s^2 for s2b); reading R10. */
double orc_visc_rate(double mu_v, double rho, double phi0, double cfac)
{
    return (1.0 - phi0) / (mu_v / (rho * cfac) + 0.5 * (1.0 - phi0));
}

/* ---------------------------------------------------------------------- */
/* Simulation state                                                        */
/* ---------------------------------------------------------------------- */
typedef struct {
    orc_params P;
    orc_derived d;
    int nx, ny;
    size_t n;
    double* phi0;
    double* fpost;  /* [9][n] post-collision populations */
    double* gpost;  /* [9][n] */
    double* lag;    /* [7][n]: Ax, Ay, B, Cxx, Cyy, Cxy, psi of the previous step */
    /* pass buffers */
    double* f;      /* [9][n] streamed populations */
    double* g;      /* [9][n] */
    double* fld;    /* [NF][n] intermediate fields */
    double* lag_new; /* [7][n] lagged state being written */
    double M0[81], M0inv[81], N[81], Ninv[81];
    double Sphi[81]; /* constant CH relaxation matrix */
    int64_t step;
} orc_sim;

enum { F_PHI1, F_LAP0, F_GX0, F_GY0, F_LAP1, F_GX1, F_GY1, F_MU0, F_MU1, F_MU2,
       F_MUB, F_GMX, F_GMY, F_UX, F_UY, F_P, F_SX, F_SY, NF };

#define FLD(s, k) ((s)->fld + (size_t)(k) * (s)->n)

static int wrap_or_mirror(int j, int n, int periodic)
{
    if (periodic) { j %= n; if (j < 0) j += n; return j; }
    if (j < 0) return -1 - j;          /* even mirror across the half-way wall */
    if (j >= n) return 2 * n - 1 - j;
    return j;
}

/* Isotropic 9-point central stencils (reading R2). */
static void stencil(const orc_sim* s, const double* a, int x, int y,
                    double* gx, double* gy, double* lap)
{
    double v[3][3];
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            int xx = wrap_or_mirror(x + dx, s->nx, s->P.periodic_x);
            int yy = wrap_or_mirror(y + dy, s->ny, s->P.periodic_y);
            v[dy + 1][dx + 1] = a[(size_t)yy * s->nx + xx];
        }
    double E = v[1][2], W = v[1][0], N = v[2][1], S = v[0][1];
    double NE = v[2][2], NW = v[2][0], SE = v[0][2], SW = v[0][0], C = v[1][1];
    if (gx) *gx = (4.0 * (E - W) + (NE - NW + SE - SW)) / 12.0;
    if (gy) *gy = (4.0 * (N - S) + (NE - SE + NW - SW)) / 12.0;
    if (lap) *lap = (4.0 * (E + W + N + S) + (NE + NW + SE + SW) - 20.0 * C) / 6.0;
}

/* Pull streaming with half-way bounce-back on non-periodic axes (Sec. 4). */
static void stream(orc_sim* s)
{
    int nx = s->nx, ny = s->ny;
#pragma omp parallel for if ((size_t)nx * ny >= ORC_PAR_MIN)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t id = (size_t)y * nx + x;
            for (int i = 0; i < 9; ++i) {
                int xs = x - CX[i], ys = y - CY[i];
                int out = 0;
                if (s->P.periodic_x) xs = (xs % nx + nx) % nx; else if (xs < 0 || xs >= nx) out = 1;
                if (s->P.periodic_y) ys = (ys % ny + ny) % ny; else if (ys < 0 || ys >= ny) out = 1;
                if (out) {
                    s->f[(size_t)i * s->n + id] = s->fpost[(size_t)OPP[i] * s->n + id];
                    s->g[(size_t)i * s->n + id] = s->gpost[(size_t)OPP[i] * s->n + id];
                } else {
                    size_t src = (size_t)ys * nx + xs;
                    s->f[(size_t)i * s->n + id] = s->fpost[(size_t)i * s->n + src];
                    s->g[(size_t)i * s->n + id] = s->gpost[(size_t)i * s->n + src];
                }
            }
        }
}

/* Macroscopic fields and everything up to the collision.  When `collide` is
 * set, the post-collision populations and the lagged state are written. */
static void macro_and_collide(orc_sim* s, int collide)
{
    const orc_params* P = &s->P;
    const orc_derived* d = &s->d;
    int nx = s->nx, ny = s->ny;
    size_t n = s->n;
    double cs2 = d->cs2;

    /* phase field phi1 = sum_i f_i */
#pragma omp parallel for if ((size_t)nx * ny >= ORC_PAR_MIN)
    for (size_t id = 0; id < n; ++id) {
        double sum = 0.0;
        for (int i = 0; i < 9; ++i) sum += s->f[(size_t)i * n + id];
        FLD(s, F_PHI1)[id] = sum;
    }
    /* stencils on phi0 and phi1 */
#pragma omp parallel for if ((size_t)nx * ny >= ORC_PAR_MIN)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t id = (size_t)y * nx + x;
            stencil(s, s->phi0, x, y, &FLD(s, F_GX0)[id], &FLD(s, F_GY0)[id], &FLD(s, F_LAP0)[id]);
            stencil(s, FLD(s, F_PHI1), x, y, &FLD(s, F_GX1)[id], &FLD(s, F_GY1)[id], &FLD(s, F_LAP1)[id]);
        }
    /* chemical potentials and mubar1 */
#pragma omp parallel for if ((size_t)nx * ny >= ORC_PAR_MIN)
    for (size_t id = 0; id < n; ++id) {
        double mu[3], mub[3];
        orc_chemical_potentials(d->gamma, P->D, s->phi0[id], FLD(s, F_PHI1)[id],
                                FLD(s, F_LAP0)[id], FLD(s, F_LAP1)[id], mu, mub);
        FLD(s, F_MU0)[id] = mu[0];
        FLD(s, F_MU1)[id] = mu[1];
        FLD(s, F_MU2)[id] = mu[2];
        FLD(s, F_MUB)[id] = mub[1];
    }
    /* grad(mubar1) */
#pragma omp parallel for if ((size_t)nx * ny >= ORC_PAR_MIN)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t id = (size_t)y * nx + x;
            stencil(s, FLD(s, F_MUB), x, y, &FLD(s, F_GMX)[id], &FLD(s, F_GMY)[id], NULL);
        }

    double* Ax = s->lag + 0 * n; double* Ay = s->lag + 1 * n; double* Bl = s->lag + 2 * n;
    double* Cxx = s->lag + 3 * n; double* Cyy = s->lag + 4 * n; double* Cxy = s->lag + 5 * n;
    double* psi = s->lag + 6 * n;
    double* lag_new = s->lag_new;
    double* psi_new = lag_new + 6 * n;
    double rho0 = P->rho[0], rho1 = P->rho[1], rho2 = P->rho[2];

#pragma omp parallel for if ((size_t)nx * ny >= ORC_PAR_MIN)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t id = (size_t)y * nx + x;
            double phi0 = s->phi0[id], phi1 = FLD(s, F_PHI1)[id];
            double mu0 = FLD(s, F_MU0)[id], mu1 = FLD(s, F_MU1)[id], mu2 = FLD(s, F_MU2)[id];
            double mub = FLD(s, F_MUB)[id];
            double gx0 = FLD(s, F_GX0)[id], gy0 = FLD(s, F_GY0)[id];
            double gx1 = FLD(s, F_GX1)[id], gy1 = FLD(s, F_GY1)[id];
            double gmx = FLD(s, F_GMX)[id], gmy = FLD(s, F_GMY)[id];

            /* degenerate mobility, 2f1s form (Sec. 4) */
            double fdeg = phi1 * (1.0 - phi1) * (1.0 - phi0);
            double Mob = P->M_cst + P->M_deg * fdeg;
            double a = P->M_deg * (1.0 - fdeg) / (P->M_cst + P->M_deg);

            /* density and viscosity: linear in the phase fields, phi2 = 1-phi0-phi1 */
            double phi2 = 1.0 - phi0 - phi1;
            double rho = rho0 * phi0 + rho1 * phi1 + rho2 * phi2;
            double mu_v = P->mu[0] * phi0 + P->mu[1] * phi1 + P->mu[2] * phi2;
            double drx = (rho0 - rho2) * gx0 + (rho1 - rho2) * gx1;
            double dry = (rho0 - rho2) * gy0 + (rho1 - rho2) * gy1;

            /* extra mass flux S (reading R4) */
            double Sx = (rho1 - rho2) * Mob / d->gamma[1] * gmx;
            double Sy = (rho1 - rho2) * Mob / d->gamma[1] * gmy;

            /* surface tension F_s = sum_p mu_p grad(phi_p), grad(phi2) = -grad(phi0)-grad(phi1) */
            double Fsx = mu0 * gx0 + mu1 * gx1 + mu2 * (-gx0 - gx1);
            double Fsy = mu0 * gy0 + mu1 * gy1 + mu2 * (-gy0 - gy1);
            /* correction force from the previous step's psi (reading R5):
             * F_c = div(Su - uS)/2 = (-d_y psi, d_x psi)/2 */
            double dpsix, dpsiy;
            stencil(s, psi, x, y, &dpsix, &dpsiy, NULL);
            double Fcx = -0.5 * dpsiy, Fcy = 0.5 * dpsix;
            double Fx = Fsx + P->Fb[0] + Fcx;
            double Fy = Fsy + P->Fb[1] + Fcy;

            /* velocity: rho u* = sum c g + F/2, f = (u_w - u*), u = u* + phi0 f / 2 */
            double gl[9];
            for (int i = 0; i < 9; ++i) gl[i] = s->g[(size_t)i * n + id];
            double jx = 0.0, jy = 0.0;
            for (int i = 0; i < 9; ++i) { jx += CX[i] * gl[i]; jy += CY[i] * gl[i]; }
            double usx = (jx + 0.5 * Fx) / rho, usy = (jy + 0.5 * Fy) / rho;
            /* rigid-body velocity of the solid point (reading R19) */
            double uwx = P->u_wall[0] - P->omega_wall * (y - P->wall_center[1]);
            double uwy = P->u_wall[1] + P->omega_wall * (x - P->wall_center[0]);
            double fsx = uwx - usx, fsy = uwy - usy;
            double ux = usx + 0.5 * phi0 * fsx, uy = usy + 0.5 * phi0 * fsy;
            double Gx = Fx + phi0 * rho * fsx, Gy = Fy + phi0 * rho * fsy;

            /* per-node NS relaxation rates from the viscosity relation (reading R10) */
            double s2a = orc_visc_rate(mu_v, rho, phi0, 0.5 * (1.0 - cs2));
            double s2b = orc_visc_rate(mu_v, rho, phi0, cs2);

            /* pressure */
            double Q = ux * drx + uy * dry;
            double B = (rho * ux - Sx) * ux + (rho * uy - Sy) * uy;
            double p = orc_pressure(P->d0, P->s_g[0], s2a, gl, Q, B, Bl[id]);

            FLD(s, F_UX)[id] = ux;
            FLD(s, F_UY)[id] = uy;
            FLD(s, F_P)[id] = p;
            FLD(s, F_SX)[id] = Sx;
            FLD(s, F_SY)[id] = Sy;
            if (!collide) continue;

            /* ---- CH collision ---- */
            double Anx = phi1 * ux, Any = phi1 * uy;
            double fl[9], feq[9], R[9], fo[9];
            for (int i = 0; i < 9; ++i) fl[i] = s->f[(size_t)i * n + id];
            orc_feq(P->d0, phi1, d->eta * mub, Anx, Any, feq);
            orc_Rpop(P->d0, Anx - Ax[id], Any - Ay[id], a, d->eta * gmx, d->eta * gmy, R);
            orc_collide_with(s->M0, s->M0inv, s->Sphi, fl, feq, R, fo);
            for (int i = 0; i < 9; ++i) s->fpost[(size_t)i * n + id] = fo[i];

            /* ---- NS collision ---- */
            double Cnxx = Sx * ux, Cnyy = Sy * uy, Cnxy = 0.5 * (Sx * uy + Sy * ux);
            /* M^2F = (uF + Fu) - d_t((Su+uS)/2) + c_s^2 (u grad rho + grad rho u)
             *        + (c^2 - 3 c_s^2)(u . grad rho) I   (reading R7) */
            double Mxx = 2.0 * ux * Fx - (Cnxx - Cxx[id]) + 2.0 * cs2 * ux * drx + (1.0 - 3.0 * cs2) * Q;
            double Myy = 2.0 * uy * Fy - (Cnyy - Cyy[id]) + 2.0 * cs2 * uy * dry + (1.0 - 3.0 * cs2) * Q;
            double Mxy = ux * Fy + Fx * uy - (Cnxy - Cxy[id]) + cs2 * (ux * dry + drx * uy);
            double geq[9], Fp[9], go[9];
            orc_geq(P->d0, P->rho_gauge, p, rho, ux, uy, Sx, Sy, geq);
            orc_Fpop(P->d0, Q, Gx, Gy, Mxx, Myy, Mxy, Fp);
            double Kg[9] = {P->s_g[0], P->s_g[1], P->s_g[1], s2a, s2a, s2b,
                            P->s_g[2], P->s_g[2], P->s_g[3]};
            double KN[81], Sg[81];
            for (int r = 0; r < 9; ++r)
                for (int c = 0; c < 9; ++c) KN[r * 9 + c] = Kg[r] * s->N[r * 9 + c];
            matmul9(s->Ninv, KN, Sg);            /* S = N^-1 K N */
            orc_collide_with(s->M0, s->M0inv, Sg, gl, geq, Fp, go);
            for (int i = 0; i < 9; ++i) s->gpost[(size_t)i * n + id] = go[i];

            lag_new[0 * n + id] = Anx;
            lag_new[1 * n + id] = Any;
            lag_new[2 * n + id] = B;
            lag_new[3 * n + id] = Cnxx;
            lag_new[4 * n + id] = Cnyy;
            lag_new[5 * n + id] = Cnxy;
            psi_new[id] = Sx * uy - Sy * ux;
        }
    if (collide) memcpy(s->lag, lag_new, 7 * n * sizeof(double));
}

/* Open boundaries in x by non-equilibrium extrapolation (Sec. 4, reading
 * R27): after the collision, the populations of a boundary node b (x = 0,
 * the inlet; x = nx - 1, the outlet) are its equilibrium at the boundary
 * values plus the non-equilibrium part of its inner neighbour n (x = 1,
 * x = nx - 2) at this step:  f*_i(b) = f^eq_i(b) + f*_i(n) - f^eq_i(n), and
 * the same for g.  Boundary values: inlet phi1 = phi1_in (1 - phi0), mubar1
 * = 0, S = 0, and either p = p_in with u from n or u = (u_in, 0) with p from
 * n; outlet p = p_out with phi1, mubar1, u, S from n.  The lagged fields of b
 * are set from the same values. */
static void open_boundaries(orc_sim* s)
{
    const orc_params* P = &s->P;
    const int nx = s->nx, ny = s->ny;
    const size_t n = s->n;
    const double r0 = P->rho[0], r1 = P->rho[1], r2 = P->rho[2];
    for (int y = 0; y < ny; ++y)
        for (int side = 0; side < 2; ++side) {
            const size_t ib = (size_t)y * nx + (side ? nx - 1 : 0);
            const size_t in = (size_t)y * nx + (side ? nx - 2 : 1);
            const double p0n = s->phi0[in], p1n = FLD(s, F_PHI1)[in], mbn = FLD(s, F_MUB)[in];
            const double uxn = FLD(s, F_UX)[in], uyn = FLD(s, F_UY)[in], pn = FLD(s, F_P)[in];
            const double Sxn = FLD(s, F_SX)[in], Syn = FLD(s, F_SY)[in];
            const double rhon = r0 * p0n + r1 * p1n + r2 * (1.0 - p0n - p1n);
            const double p0b = s->phi0[ib];
            double p1b, mbb, uxb, uyb, pb, Sxb, Syb;
            if (side == 0) {
                p1b = P->phi1_in * (1.0 - p0b);
                mbb = 0.0;
                Sxb = Syb = 0.0;
                if (P->inlet_type == 0) { pb = P->p_in; uxb = uxn; uyb = uyn; }
                else { pb = pn; uxb = P->u_in; uyb = 0.0; }
            } else {
                p1b = p1n; mbb = mbn; pb = P->p_out; uxb = uxn; uyb = uyn; Sxb = Sxn; Syb = Syn;
            }
            const double rhob = r0 * p0b + r1 * p1b + r2 * (1.0 - p0b - p1b);
            double feb[9], fen[9], geb[9], gen[9];
            orc_feq(P->d0, p1b, s->d.eta * mbb, p1b * uxb, p1b * uyb, feb);
            orc_feq(P->d0, p1n, s->d.eta * mbn, p1n * uxn, p1n * uyn, fen);
            orc_geq(P->d0, P->rho_gauge, pb, rhob, uxb, uyb, Sxb, Syb, geb);
            orc_geq(P->d0, P->rho_gauge, pn, rhon, uxn, uyn, Sxn, Syn, gen);
            for (int i = 0; i < 9; ++i) {
                s->fpost[(size_t)i * n + ib] = feb[i] + s->fpost[(size_t)i * n + in] - fen[i];
                s->gpost[(size_t)i * n + ib] = geb[i] + s->gpost[(size_t)i * n + in] - gen[i];
            }
            s->lag[0 * n + ib] = p1b * uxb;
            s->lag[1 * n + ib] = p1b * uyb;
            s->lag[2 * n + ib] = (rhob * uxb - Sxb) * uxb + (rhob * uyb - Syb) * uyb;
            s->lag[3 * n + ib] = Sxb * uxb;
            s->lag[4 * n + ib] = Syb * uyb;
            s->lag[5 * n + ib] = 0.5 * (Sxb * uyb + Syb * uxb);
            s->lag[6 * n + ib] = Sxb * uyb - Syb * uxb;
        }
}

/* Sums over the pore space (phi0 <= 1/2) of u_x, phi1 u_x and phi2 u_x at
 * the current time level: the integrals of the relative permeability
 * K_p (Sec. 4.6), with u_{x,p} read as phi_p u_x. */
void orc_flow_rates(orc_sim* s, double q[3]);

/* ---------------------------------------------------------------------- */
/* Public entry points (called through ctypes by the tests)                */
/* ---------------------------------------------------------------------- */
orc_sim* orc_create(const orc_params* P, const double* phi0, const double* phi1)
{
    orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
    s->P = *P;
    if (orc_derive(P, &s->d) != 0 || (P->open_x && P->periodic_x)) { free(s); return NULL; }
    s->nx = P->nx; s->ny = P->ny; s->n = (size_t)P->nx * P->ny;
    size_t n = s->n;
    s->phi0 = (double*)malloc(n * sizeof(double));
    s->fpost = (double*)malloc(9 * n * sizeof(double));
    s->gpost = (double*)malloc(9 * n * sizeof(double));
    s->lag = (double*)calloc(7 * n, sizeof(double));          /* reading R6 */
    s->f = (double*)malloc(9 * n * sizeof(double));
    s->g = (double*)malloc(9 * n * sizeof(double));
    s->fld = (double*)calloc((size_t)NF * n, sizeof(double));
    s->lag_new = (double*)calloc(7 * n, sizeof(double));
    orc_M0(s->M0);
    orc_inverse9(s->M0, s->M0inv);
    orc_N(s->d.cs2, s->N);
    orc_inverse9(s->N, s->Ninv);
    {
        double s1 = 1.0 / P->tau_phi;
        double Kphi[9] = {P->s_phi[0], s1, s1, P->s_phi[1], P->s_phi[1], P->s_phi[1],
                          P->s_phi[2], P->s_phi[2], P->s_phi[3]};
        orc_relaxation_matrix(s->d.cs2, Kphi, s->Sphi);
    }
    memcpy(s->phi0, phi0, n * sizeof(double));
    memcpy(FLD(s, F_PHI1), phi1, n * sizeof(double));

    /* initial state (reading R9): mubar1 from the initial phi1 */
    for (int y = 0; y < s->ny; ++y)
        for (int x = 0; x < s->nx; ++x) {
            size_t id = (size_t)y * s->nx + x;
            stencil(s, s->phi0, x, y, NULL, NULL, &FLD(s, F_LAP0)[id]);
            stencil(s, FLD(s, F_PHI1), x, y, NULL, NULL, &FLD(s, F_LAP1)[id]);
        }
    for (size_t id = 0; id < n; ++id) {
        double mu[3], mub[3], feq[9], geq[9];
        orc_chemical_potentials(s->d.gamma, P->D, phi0[id], phi1[id],
                                FLD(s, F_LAP0)[id], FLD(s, F_LAP1)[id], mu, mub);
        orc_feq(P->d0, phi1[id], s->d.eta * mub[1], 0.0, 0.0, feq);
        orc_geq(P->d0, P->rho_gauge, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0, geq);
        for (int i = 0; i < 9; ++i) {
            s->fpost[(size_t)i * n + id] = feq[i];
            s->gpost[(size_t)i * n + id] = geq[i];
        }
    }
    s->step = 0;
    return s;
}

void orc_free(orc_sim* s)
{
    if (!s) return;
    free(s->phi0); free(s->fpost); free(s->gpost); free(s->lag);
    free(s->f); free(s->g); free(s->fld); free(s->lag_new); free(s);
}

void orc_step(orc_sim* s, int64_t nsteps)
{
    for (int64_t k = 0; k < nsteps; ++k) {
        stream(s);
        macro_and_collide(s, 1);
        if (s->P.open_x) open_boundaries(s);
        s->step++;
    }
}

/* Macroscopic fields at the current time level (streamed from the stored
 * post-collision populations), without advancing the state. */
void orc_moments(orc_sim* s, double* phi1, double* ux, double* uy, double* p)
{
    stream(s);
    macro_and_collide(s, 0);
    size_t n = s->n;
    if (phi1) memcpy(phi1, FLD(s, F_PHI1), n * sizeof(double));
    if (ux) memcpy(ux, FLD(s, F_UX), n * sizeof(double));
    if (uy) memcpy(uy, FLD(s, F_UY), n * sizeof(double));
    if (p) memcpy(p, FLD(s, F_P), n * sizeof(double));
}

/* Auxiliary fields at the current time level: mubar1, grad(mubar1). */
void orc_aux(orc_sim* s, double* mub, double* gmx, double* gmy)
{
    stream(s);
    macro_and_collide(s, 0);
    size_t n = s->n;
    if (mub) memcpy(mub, FLD(s, F_MUB), n * sizeof(double));
    if (gmx) memcpy(gmx, FLD(s, F_GMX), n * sizeof(double));
    if (gmy) memcpy(gmy, FLD(s, F_GMY), n * sizeof(double));
}

/* Phase mass sum_x phi1(x) = sum_x sum_i f*_i(x) (streaming only permutes). */
double orc_mass(const orc_sim* s)
{
    long double m = 0.0L;
    for (size_t k = 0; k < 9 * s->n; ++k) m += s->fpost[k];
    return (double)m;
}

int64_t orc_step_count(const orc_sim* s) { return s->step; }

void orc_get_state(const orc_sim* s, double* fpost, double* gpost, double* lag)
{
    size_t n = s->n;
    if (fpost) memcpy(fpost, s->fpost, 9 * n * sizeof(double));
    if (gpost) memcpy(gpost, s->gpost, 9 * n * sizeof(double));
    if (lag) memcpy(lag, s->lag, 7 * n * sizeof(double));
}

void orc_set_state(orc_sim* s, const double* fpost, const double* gpost, const double* lag)
{
    size_t n = s->n;
    if (fpost) memcpy(s->fpost, fpost, 9 * n * sizeof(double));
    if (gpost) memcpy(s->gpost, gpost, 9 * n * sizeof(double));
    if (lag) memcpy(s->lag, lag, 7 * n * sizeof(double));
}

void orc_get_derived(const orc_sim* s, orc_derived* d) { *d = s->d; }

int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_flow_rates(orc_sim* s, double q[3])
{
    stream(s);
    macro_and_collide(s, 0);
    long double a = 0.0L, b = 0.0L, c = 0.0L;
    for (size_t id = 0; id < s->n; ++id) {
        if (s->phi0[id] > 0.5) continue;
        const double ux = FLD(s, F_UX)[id], p1 = FLD(s, F_PHI1)[id];
        a += ux;
        b += p1 * ux;
        c += (1.0 - s->phi0[id] - p1) * ux;
    }
    q[0] = (double)a;
    q[1] = (double)b;
    q[2] = (double)c;
}
