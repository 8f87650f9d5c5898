/*
 * tpf3f.h -- C ABI of the 3f model ("three fluids") of Zhan, Chai & Shi,
 * "A ternary phase-field model for two-phase flows in complex geometries"
 * (arXiv 2311.05091), on the D2Q9 lattice: the three-component
 * Cahn-Hilliard model of Sec. 2.1 for phases 0 and 1, each on its own CH
 * lattice (phi2 = 1 - phi0 - phi1), coupled to the modified NS lattice of
 * Sec. 3 without solid terms, all with the Hermite-moment collision of
 * Sec. 4; the degenerate mobility M = M_cst + M_deg (1 - phi0)(1 - phi1)
 * (1 - phi2) of Sec. 4; the spreading coefficients from three pairwise
 * surface tensions (Sec. 2.1); the extra mass flux S summed over the three
 * phases.  Sec. 4.1 runs this model with sigma01 = sigma02 = sigma12.
 *
 * Conventions as in tpf.h: int status codes (TPF_OK = 0, TPF_EINVAL = -1,
 * TPF_EDEVICE = -2, TPF_ESTATE = -5; tpf_strerror() names them); host arrays
 * float64, row-major [ny][nx] with x fastest, copied in and out (the caller
 * keeps ownership); one device arena, caller-provided (>= tpf3f_arena_bytes())
 * or allocated by the library (NULL); work enqueued on the stream given to
 * tpf3f_create; read calls synchronise it; one context per host thread; no
 * device work before tpf3f_finalize.  Lattice units (c = dx = dt = 1).
 */
#ifndef TPF3F_H
#define TPF3F_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Parameters of one 3f domain.  Defaults (tpf3f_default_params): periodic in
 * x, walls in y, d0 = 1/2, D = 4, sigma01 = sigma02 = sigma12 = 0.01,
 * rho = 1, mu = 0.15, M_cst = 0, M_deg = 0.01, tau_phi = 0.8, all other
 * rates 1, no force. */
typedef struct {
    int32_t nx, ny;
    int32_t periodic_x, periodic_y;  /* 1 periodic, 0 half-way bounce-back walls */
    double d0, D;
    double sigma01, sigma02, sigma12;/* pairwise surface tensions (every gamma_p > 0) */
    double rho[3], mu[3];            /* densities and viscosities of phases 0, 1, 2   */
    double M_cst, M_deg, tau_phi;    /* mobility; 1/s1 of both CH lattices            */
    double s_phi[4];                 /* s0, s2, s3, s4 of both CH lattices            */
    double s_g[4];                   /* s0, s1, s3, s4 of the NS lattice              */
    double Fb[2];                    /* body force                                    */
    double rho_gauge;                /* constant in lambda_0; 0 = offset storage      */
} tpf3f_domain_params;

typedef struct tpf3f_ctx tpf3f_ctx;

void tpf3f_default_params(tpf3f_domain_params* p, int32_t nx, int32_t ny);

/* precision 32 (FP32 storage and arithmetic, FP64 mass sums) or 64. */
int tpf3f_create(tpf3f_ctx** out, int32_t precision, void* hip_stream);

/* phi0_init, phi1_init: nx*ny float64 each.  TPF_EINVAL for sizes < 3 or more
 * than 2^31 / 9 nodes, a gamma_p <= 0, tau_phi <= 1/2, d0 outside (0, 1),
 * non-positive densities, viscosities or D, M_cst + M_deg <= 0, rates outside
 * (0, 2).  Only before tpf3f_finalize(). */
int tpf3f_add_domain(tpf3f_ctx* ctx, const tpf3f_domain_params* p, const double* phi0_init,
                     const double* phi1_init, int32_t* domain_id);

int tpf3f_arena_bytes(tpf3f_ctx* ctx, uint64_t* bytes);

/* Derives the constants (gamma_p, gamma^T, eta_p, the 2D pressure constants)
 * and initialises every domain: f_p = f^eq(phi_p, eta_p mubar_p, u = 0) for
 * p = 0, 1, g = g^eq(P = 0, u = 0), lagged fields zero.  TPF_EDEVICE when no
 * device is present. */
int tpf3f_finalize(tpf3f_ctx* ctx, void* arena, uint64_t arena_bytes);

/* nsteps coupled steps of every domain: pull streaming of the three lattices
 * with bounce-back, phi0 and phi1, the 9-point stencils, mu_p and mubar_0,
 * mubar_1, S, the forces, u, p and the three Hermite-moment collisions. */
int tpf3f_step(tpf3f_ctx* ctx, int64_t nsteps);

/* phi0, phi1, ux, uy, p of domain id at the current time level (host arrays
 * of nx*ny float64; any may be NULL). */
int tpf3f_read_moments(tpf3f_ctx* ctx, int32_t id, double* phi0, double* phi1, double* ux, double* uy,
                       double* p);

/* Phase masses sum phi0 and sum phi1 of domain id (FP64, compensated). */
int tpf3f_read_mass(tpf3f_ctx* ctx, int32_t id, double mass[2]);

/* Post-collision populations f0[9][ny][nx], f1[...], g[...] as float64 (each
 * may be NULL). */
int tpf3f_get_populations(tpf3f_ctx* ctx, int32_t id, double* f0, double* f1, double* g);

/* Bytes a step moves by definition per node: 27 population reads and writes,
 * the lagged phi0 u, phi1 u and B read and written; with S (rho_p not all
 * equal) also sym(Su) and S_x u_y - S_y u_x. */
int tpf3f_bytes_per_node(tpf3f_ctx* ctx, int32_t id, double* bytes);

/* Average time per launch of the fused kernel since the last call with timing
 * enabled (HIP events around each tpf3f_step call's launches). */
int tpf3f_kernel_timing(tpf3f_ctx* ctx, int32_t enable, double* avg_ms, int64_t* launches);

void tpf3f_destroy(tpf3f_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* TPF3F_H */
