/* Host-sanitizer driver of the 3D oracle (test infrastructure), compiled with
 * oracle/tpf_oracle3d.c under AddressSanitizer and UndefinedBehaviorSanitizer:
 * small boxes with walls, a solid sphere, the S flux and a translating solid. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/tpf_oracle3d.c"

static int run(const orc3_params* p, int steps) {
    const int nx = p->nx, ny = p->ny, nz = p->nz, N = nx * ny * nz;
    double* phi0 = malloc(sizeof(double) * N);
    double* phi1 = malloc(sizeof(double) * N);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int i = (z * ny + y) * nx + x;
                const double rs = sqrt((x - 0.3 * nx) * (x - 0.3 * nx) + (y - 0.5 * ny) * (y - 0.5 * ny) +
                                       (z - 0.5 * nz) * (z - 0.5 * nz));
                const double rd = sqrt((x - 0.7 * nx) * (x - 0.7 * nx) + (y - 0.5 * ny) * (y - 0.5 * ny) +
                                       (z - 0.5 * nz) * (z - 0.5 * nz));
                phi0[i] = 0.5 + 0.5 * tanh(2.0 * (0.2 * nx - rs) / p->D);
                phi1[i] = (1.0 - phi0[i]) * (0.5 + 0.5 * tanh(2.0 * (0.2 * nx - rd) / p->D));
            }
    phi0[0] = 1.0;
    orc3_sim* s = orc3_create(p, phi0, phi1);
    if (!s) return 1;
    orc3_step(s, steps);
    double* m = malloc(sizeof(double) * 5 * N);
    orc3_moments(s, m, m + N, m + 2 * N, m + 3 * N, m + 4 * N);
    orc3_aux(s, m, m + N);
    double* f = malloc(sizeof(double) * 15 * N);
    double* g = malloc(sizeof(double) * 15 * N);
    double* lag = malloc(sizeof(double) * 13 * N);
    orc3_get_state(s, f, g, lag);
    orc3_set_state(s, f, g, lag);
    orc3_step(s, 1);
    const int bad = !isfinite(orc3_mass(s)) || orc3_step_count(s) != steps + 1;
    orc3_free(s);
    free(phi0); free(phi1); free(m); free(f); free(g); free(lag);
    return bad;
}

int main(void) {
    orc3_params p = {0};
    p.nx = 12; p.ny = 9; p.nz = 10;
    p.periodic[0] = 1; p.periodic[1] = 1; p.periodic[2] = 0;
    p.d0 = 0.4; p.D = 3.0; p.sigma12 = 0.01; p.theta = M_PI / 3.0;
    p.rho[0] = 1.0; p.rho[1] = 1.0; p.rho[2] = 0.1;
    p.mu[0] = 0.15; p.mu[1] = 0.15; p.mu[2] = 0.015;
    p.M_deg = 0.004; p.tau_phi = 0.8;
    for (int i = 0; i < 4; ++i) p.s_phi[i] = p.s_g[i] = 1.0;
    p.s_g[2] = p.s_g[3] = 0.5;
    p.u_wall[0] = 1e-3; p.Fb[2] = 1e-5;
    int bad = run(&p, 8);
    p.periodic[0] = p.periodic[1] = 0;
    p.nx = p.ny = p.nz = 3;
    bad |= run(&p, 3);
    printf("oracle3 sanitized run %s\n", bad ? "FAILED" : "ok");
    return bad;
}
