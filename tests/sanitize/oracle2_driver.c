/* Host-sanitizer driver of the 2D oracle (test infrastructure): compiled
 * together with oracle/tpf_oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer, it runs every public entry point on small
 * domains that reach the wall, solid, S-flux and moving-solid branches, so
 * an out-of-bounds access or undefined operation in the oracle aborts. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/tpf_oracle.c"

static orc_params base(int nx, int ny) {
    orc_params p = {0};
    p.nx = nx;
    p.ny = ny;
    p.periodic_x = 1;
    p.periodic_y = 0;
    p.d0 = 0.5;
    p.D = 4.0;
    p.sigma12 = 0.01;
    p.theta = M_PI / 3.0;
    p.rho[0] = p.rho[1] = p.rho[2] = 1.0;
    p.mu[0] = p.mu[1] = p.mu[2] = 0.15;
    p.M_deg = 0.01;
    p.tau_phi = 0.8;
    for (int i = 0; i < 4; ++i) p.s_phi[i] = p.s_g[i] = 1.0;
    return p;
}

static int run(const orc_params* p, int steps) {
    const int nx = p->nx, ny = p->ny, N = nx * ny;
    double* phi0 = malloc(sizeof(double) * N);
    double* phi1 = malloc(sizeof(double) * N);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const double rs = hypot(x - 0.3 * nx, y - 0.4 * ny), rd = hypot(x - 0.65 * nx, y - 0.55 * ny);
            phi0[y * nx + x] = 0.5 + 0.5 * tanh(2.0 * (0.2 * nx - rs) / p->D);
            phi1[y * nx + x] = (1.0 - phi0[y * nx + x]) * (0.5 + 0.5 * tanh(2.0 * (0.2 * nx - rd) / p->D));
        }
    if (nx * ny > 16) phi0[0] = 1.0;  /* one saturated node (s2a = 0) */
    orc_sim* s = orc_create(p, phi0, phi1);
    if (!s) return 1;
    orc_step(s, steps);
    double *a = malloc(sizeof(double) * N), *b = malloc(sizeof(double) * N), *c = malloc(sizeof(double) * N),
           *d = malloc(sizeof(double) * N);
    orc_moments(s, a, b, c, d);
    orc_aux(s, a, b, c);
    double* f = malloc(sizeof(double) * 9 * N);
    double* g = malloc(sizeof(double) * 9 * N);
    double* lag = malloc(sizeof(double) * 8 * N);
    orc_get_state(s, f, g, lag);
    orc_set_state(s, f, g, lag);
    orc_step(s, 2);
    orc_derived dv;
    orc_get_derived(s, &dv);
    const double m = orc_mass(s);
    const int bad = !isfinite(m) || orc_step_count(s) != steps + 2;
    orc_free(s);
    free(phi0); free(phi1); free(a); free(b); free(c); free(d); free(f); free(g); free(lag);
    return bad;
}

int main(void) {
    int bad = 0;
    orc_params p = base(24, 18);
    bad |= run(&p, 20);
    p.rho[2] = 0.1;                       /* S flux, F_c, C terms */
    p.mu[2] = 0.015;
    p.d0 = 0.4;                           /* H with its s2a term */
    p.u_wall[0] = 1e-3;                   /* moving solid */
    p.omega_wall = 1e-4;
    p.wall_center[0] = 7.0;
    p.wall_center[1] = 7.0;
    p.Fb[0] = 1e-5;
    bad |= run(&p, 20);
    p.periodic_x = 0;                     /* closed box */
    bad |= run(&p, 10);
    orc_params q = base(3, 3);            /* smallest domain */
    q.periodic_y = 1;
    bad |= run(&q, 5);
    double w[9], M0[81], Mi[81], Nm[81], S[81], K[9] = {1, 1.25, 1.25, 0.9, 0.9, 0.8, 1, 1, 1};
    orc_weights(0.4, w);
    orc_M0(M0);
    bad |= orc_inverse9(M0, Mi) != 0;
    orc_N(0.4, Nm);
    orc_relaxation_matrix(0.4, K, S);
    for (int t = 1; t < 180; t += 7) bad |= !isfinite(orc_spreading_factor(t * M_PI / 180.0, 0.8));
    printf("oracle2 sanitized run %s\n", bad ? "FAILED" : "ok");
    return bad;
}
