/*
 * tpf3.h -- C ABI of the three-dimensional coupled step of Zhan, Chai & Shi,
 * "A ternary phase-field model for two-phase flows in complex geometries"
 * (arXiv 2311.05091), 2f1s model on the D3Q15 lattice: Cahn-Hilliard lattice
 * f for the fluid phase field phi1 (solid field phi0 fixed, phi2 = 1 - phi0 -
 * phi1) and the modified Navier-Stokes lattice g, both with the
 * Hermite-moment collision (Sec. 4) and the D3Q15 weights and matrices of
 * Appendix A, the 3D pressure constants K = 1 - 2 d0 and H of Sec. 3.
 *
 * Conventions as in tpf.h: int status codes (TPF_OK = 0, TPF_EINVAL = -1,
 * TPF_EDEVICE = -2, TPF_ESTATE = -5; tpf_strerror() names them); host arrays
 * float64, row-major [nz][ny][nx] with x fastest, copied in and out (the
 * caller keeps ownership); one device arena, caller-provided (>=
 * tpf3_arena_bytes()) or allocated by the library (NULL); work enqueued on
 * the stream given to tpf3_create; read calls synchronise it; one context per
 * host thread.  Lattice units (c = dx = dt = 1).
 */
#ifndef TPF3_H
#define TPF3_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Parameters of one 3D domain.  Defaults (tpf3_default_params): periodic in
 * x and y, walls in z, d0 = 0.4, D = 4, sigma12 = 0.01, theta = pi/3,
 * kappa = 0, rho = 1, mu = 0.15, M_cst = 0, M_deg = 0.004, tau_phi = 0.8,
 * NS rates s3 = s4 = 1/2, all other rates 1, no forces.  (d0 = 1/2 leaves the
 * D3Q15 rest velocity without weight and makes the step diverge next to a
 * diffuse solid; NS s3 = s4 = 1 diverge next to a solid whose interior
 * saturates (phi0 -> 1); M_cst + M_deg above about 0.005 makes the explicit
 * 15-point scheme unstable.  All are accepted, none is recommended.) */
typedef struct {
    int32_t nx, ny, nz;           /* nodes (>= 3 each)                                    */
    int32_t periodic[3];          /* per axis: 1 periodic, 0 half-way bounce-back walls   */
    double d0;                    /* c_s^2 = d0, in (0, 1)                                */
    double D, sigma12, theta, kappa;
    double rho[3], mu[3];         /* phases 0 (solid), 1, 2                               */
    double M_cst, M_deg, tau_phi;
    double s_phi[4];              /* CH rates s0, s2, s3, s4                              */
    double s_g[4];                /* NS rates s0, s1, s3, s4 (s2a, s2b per node, Sec. 3)  */
    double Fb[3];                 /* body force                                           */
    double u_wall[3];             /* velocity of the solid points (a translation)         */
    double rho_gauge;             /* constant in lambda_0; 0 = offset storage             */
} tpf3_domain_params;

typedef struct tpf3_ctx tpf3_ctx;

void tpf3_default_params(tpf3_domain_params* p, int32_t nx, int32_t ny, int32_t nz);

/* precision 32 (FP32 storage and arithmetic, FP64 mass sums) or 64.  Touches
 * no device (tpf3_finalize returns TPF_EDEVICE when there is none). */
int tpf3_create(tpf3_ctx** out, int32_t precision, void* hip_stream);

/* phi0, phi1_init: nx*ny*nz float64 each.  TPF_EINVAL for sizes < 3 or more
 * than 2^31 / 15 nodes, theta outside (0, pi), a non-positive gamma_p,
 * tau_phi <= 1/2, d0 outside (0, 1), non-positive densities or viscosities,
 * M_cst + M_deg <= 0, rates outside (0, 2).  Only before tpf3_finalize(). */
int tpf3_add_domain(tpf3_ctx* ctx, const tpf3_domain_params* p, const double* phi0, const double* phi1_init,
                    int32_t* domain_id);

int tpf3_arena_bytes(tpf3_ctx* ctx, uint64_t* bytes);

/* Derives the constants and initialises every domain: f = f^eq(phi1, mubar1,
 * u = 0), g = g^eq(P = 0, u = 0), lagged fields zero (readings R6, R9). */
int tpf3_finalize(tpf3_ctx* ctx, void* arena, uint64_t arena_bytes);

/* nsteps coupled steps of every domain (Sec. 3): pull streaming with
 * bounce-back, phi1, the 15-point stencils, mubar1, forces, u, p, and the
 * Hermite-moment collisions of both D3Q15 lattices. */
int tpf3_step(tpf3_ctx* ctx, int64_t nsteps);

/* phi1, u (with the solid correction) and p of domain id at the current time
 * level; host arrays of nx*ny*nz float64, any may be NULL. */
int tpf3_read_moments(tpf3_ctx* ctx, int32_t id, double* phi1, double* ux, double* uy, double* uz, double* p);

/* Phase mass sum phi1 of domain id (FP64, compensated). */
int tpf3_read_mass(tpf3_ctx* ctx, int32_t id, double* mass);

/* Post-collision populations f[15][nz][ny][nx], g[...] as float64 (NULL ok). */
int tpf3_get_populations(tpf3_ctx* ctx, int32_t id, double* f, double* g);

/* Tile of the fused kernel: 64 x ty x 32 nodes (ty = 2, 4 or 8; 0 = the
 * largest the precision and the extra flux S allow: FP32 8 without S, 4 with;
 * FP64 4 without, 2 with).  TPF_EINVAL for a ty the LDS cannot hold. */
int tpf3_set_tile(tpf3_ctx* ctx, int32_t ty);
int tpf3_get_tile(tpf3_ctx* ctx, int32_t* tx, int32_t* ty, int32_t* tz);

/* Bytes a step moves by definition per node: 30 population reads and writes,
 * phi0, and the lagged fields read and written (phi1 u, B; with S also
 * sym(Su) and S x u). */
int tpf3_bytes_per_node(tpf3_ctx* ctx, int32_t id, double* bytes);

/* Average time per launch of the fused kernel (HIP events around each
 * tpf3_step call's launches) since the last call with timing enabled. */
int tpf3_kernel_timing(tpf3_ctx* ctx, int32_t enable, double* avg_ms, int64_t* launches);

void tpf3_destroy(tpf3_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* TPF3_H */
