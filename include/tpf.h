/*
 * tpf.h -- C ABI of the MI355X (gfx950) library that advances the coupled
 * ternary phase-field lattice Boltzmann step of Zhan, Chai & Shi, "A ternary
 * phase-field model for two-phase flows in complex geometries"
 * (arXiv 2311.05091), 2f1s model: one Cahn-Hilliard lattice f for the fluid
 * phase field phi1 (the solid field phi0 is fixed and phi2 = 1 - phi0 - phi1,
 * Sec. 2.2 Remarks 2-3) and one lattice g for the modified Navier-Stokes
 * equations (Sec. 2.3), both D2Q9 with the Hermite-moment collision of
 * Sec. 4 and the matrices of Appendix A.
 *
 * Conventions
 *   - Every function returns an int status: TPF_OK (0) or a negative
 *     TPF_E* code; nothing throws across the ABI.  tpf_strerror() names it.
 *   - Host arrays are float64, row-major [ny][nx] with x fastest; the library
 *     copies them in and out, the caller keeps ownership.
 *   - Device memory: one arena.  The caller may hand in a device pointer of at
 *     least tpf_arena_bytes() bytes (e.g. from a torch tensor); it must stay
 *     valid until tpf_destroy().  With a NULL arena the library allocates
 *     (hipMalloc) and frees it itself.
 *   - Work is enqueued on the HIP stream given to tpf_create() (NULL = the
 *     default stream).  Read/diagnostic calls synchronise that stream.
 *   - One context per host thread; contexts are independent.
 *   - Units: lattice units, c = dx = dt = 1.
 */
#ifndef TPF_H
#define TPF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    TPF_OK = 0,
    TPF_EINVAL = -1,  /* invalid argument or parameter set                 */
    TPF_EDEVICE = -2, /* HIP runtime error or no gfx950 device             */
    TPF_ENAN = -3,    /* a domain produced NaN/Inf (only that domain stops) */
    TPF_EBUDGET = -4, /* step cap reached before the residual tolerance    */
    TPF_ESTATE = -5,  /* call not valid in the context's current state     */
    TPF_EIO = -6      /* checkpoint file could not be read or written      */
};

/* Physical and numerical parameters of one domain.  Citations are to the
 * paper; the defaults listed are those tpf_default_params() fills in. */
typedef struct {
    int32_t nx, ny;               /* nodes (>= 3 each)                                   */
    int32_t periodic_x;           /* 1 = periodic, 0 = half-way bounce-back walls (Sec. 4) */
    int32_t periodic_y;
    double d0;                    /* scale factor, c_s^2 = d0 c^2, in (0,1); 0.5 (App. A) */
    double D;                     /* interface thickness (Sec. 2.1); 4                   */
    double sigma12;               /* fluid 1 - fluid 2 surface tension; 0.01             */
    double theta;                 /* contact angle of fluid 1 on the solid, radians, in (0, pi) */
    double kappa;                 /* minimum dimensionless solid curvature, Eq. (eq-kk); 0 */
    double rho[3];                /* densities of phases 0 (solid), 1, 2 (Sec. 2.3); > 0  */
    double mu[3];                 /* dynamic viscosities of phases 0, 1, 2; > 0         */
    double M_cst, M_deg;          /* mobility M = M_cst + M_deg f(phi) (Sec. 2.2, Sec. 4) */
    double tau_phi;               /* 1/s1 of the CH lattice (> 1/2); eta follows from
                                     (M_cst + M_deg)/gamma_1 = (1/s1 - 1/2) eta c_s^2 (Sec. 3) */
    double s_phi[4];              /* s0, s2, s3, s4 of the CH lattice; 1                */
    double s_g[4];                /* s0, s1, s3, s4 of the NS lattice; 1 (s2a, s2b follow
                                     per node from the viscosity relation of Sec. 3)   */
    double Fb[2];                 /* body force F_b (Sec. 2.3)                          */
    double u_wall[2];             /* velocity u_w of the solid points in f = (u_w - u*)/dt
                                     (Sec. 3): a rigid motion, u_w(x, y) = u_wall +
                                     omega_wall e_z x ((x, y) - wall_center), node (i, j)
                                     at (x, y) = (i, j); phi0 stays fixed, so the motion
                                     must leave the solid's shape invariant (a sliding
                                     plate, a spinning disk or ring); 0                   */
    double omega_wall;            /* angular velocity of the solid; 0                   */
    double wall_center[2];        /* centre of that rotation; 0                         */
    double rho_gauge;             /* constant in lambda_0 (Sec. 3); 0 = offset storage   */
    int32_t open_x;               /* 1: open ends in x, an inlet at x = 0 and an outlet at
                                     x = nx - 1, imposed after each collision by
                                     non-equilibrium extrapolation from the inner
                                     neighbour (Sec. 4); needs periodic_x = 0; 0      */
    int32_t inlet_type;           /* 0: pressure inlet p_in (u extrapolated), 1: velocity
                                     inlet (u_in, 0) (p extrapolated); 0               */
    double p_in, u_in, p_out;     /* inlet pressure or velocity, outlet pressure; 0      */
    double phi1_in;               /* phase-1 share of the fluid entering: phi1 = phi1_in
                                     (1 - phi0) at the inlet, mubar1 = 0 there; the outlet
                                     takes phi1 and mubar1 from its neighbour; 0       */
} tpf_domain_params;

typedef struct tpf_ctx tpf_ctx;

/* Fills *p with the defaults above for an nx x ny domain (periodic in x,
 * walls in y, theta = pi/3). */
void tpf_default_params(tpf_domain_params* p, int32_t nx, int32_t ny);

/* Creates a context.  precision: 32 (FP32 storage and arithmetic, FP64
 * reductions) or 64 (FP64 throughout).  hip_stream: a hipStream_t or NULL.
 * Touches no device: domains can be added and the arena size, derived
 * constants and bytes per node queried on a host without a GPU;
 * tpf_finalize fails with TPF_EDEVICE when no device is present. */
int tpf_create(tpf_ctx** out, int32_t precision, void* hip_stream);

/* Adds a domain: phi0 (solid field, fixed) and phi1_init, each nx*ny
 * float64.  Validates the parameters (TPF_EINVAL: nx or ny < 3, theta not in
 * (0, pi), any gamma_p <= 0, tau_phi <= 1/2, d0 not in (0, 1), densities or
 * viscosities <= 0, M_cst + M_deg <= 0).  Only before tpf_finalize(). */
int tpf_add_domain(tpf_ctx* ctx, const tpf_domain_params* p, const double* phi0,
                   const double* phi1_init, int32_t* domain_id);

/* Device bytes the context needs after the domains have been added. */
int tpf_arena_bytes(tpf_ctx* ctx, uint64_t* bytes);

/* Allocates (or binds) the device arena, derives the per-domain constants
 * (spreading factor, gamma_p, eta, Sec. 2.2-3) and initialises every domain:
 * f = f^eq(phi1, mubar1, u = 0), g = g^eq(P = 0, u = 0), lagged fields 0.
 * arena: device pointer of >= tpf_arena_bytes() bytes, 256-byte aligned, or NULL.
 * TPF_EDEVICE when no device is present. */
int tpf_finalize(tpf_ctx* ctx, void* arena, uint64_t arena_bytes);

/* Advances every live domain by nsteps coupled time steps (Sec. 3): per step
 * and node, pull-streaming of f and g with half-way bounce-back, phi1, the
 * chemical potentials and mubar1, grad(mubar1), the forces, u, p, and the
 * Hermite-moment collisions of both lattices. */
int tpf_step(tpf_ctx* ctx, int64_t nsteps);

/* Runs every live domain until its residual
 *   r = ||phi1^n - phi1^(n-K)||_2 / (K ||phi1^n||_2),  K = check_every,
 * drops below tol, or max_steps more steps have been taken.  steps_out
 * (n_domains entries, may be NULL) receives each domain's steps in this call.
 * Returns TPF_EBUDGET if some domain reached max_steps, TPF_ENAN if some
 * domain produced NaN (the others still run), else TPF_OK. */
int tpf_run_to_residual(tpf_ctx* ctx, double tol, int32_t check_every, int64_t max_steps,
                        int64_t* steps_out);

/* Macroscopic fields of domain id at the current time level: phi1 = sum f_i,
 * u (with the solid correction u = u* + phi0 f/2) and p (Sec. 3).  Host
 * arrays of nx*ny float64; any may be NULL. */
int tpf_read_moments(tpf_ctx* ctx, int32_t id, double* phi1, double* ux, double* uy, double* p);

/* Flow rates of domain id at the current time level over its pore space
 * (phi0 <= 1/2): q[0] = sum u_x, q[1] = sum phi1 u_x, q[2] = sum phi2 u_x,
 * FP64 compensated.  The relative permeability of fluid p (Sec. 4.6) is
 * q[p] of a two-phase run over q[0] of a single-phase run of fluid p under
 * the same drive. */
int tpf_flow_rates(tpf_ctx* ctx, int32_t id, double* q);

/* Diagnostics of domain id from the last reduction: mass = sum phi1 (FP64,
 * compensated), residual as in tpf_run_to_residual (NaN before two checks),
 * status (TPF_OK, TPF_ENAN, or 1 when retired by the residual test), steps
 * taken so far.  Triggers a fresh mass reduction. */
int tpf_read_diag(tpf_ctx* ctx, int32_t id, double* mass, double* residual, int32_t* status,
                  int64_t* steps);

/* Re-initialises domain id from a new phi1 field (warm start): populations
 * at equilibrium with u = 0, lagged fields zeroed, residual history reset. */
int tpf_set_phi1(tpf_ctx* ctx, int32_t id, const double* phi1);

/* Leaves domain id out of (active = 0) or back in (1) every following
 * tpf_step and tpf_run_to_residual of the batch: its state stays as it is and
 * its step count in steps_per_domain is 0 while inactive.  Domains are active
 * when added; tpf_set_phi1 and tpf_load leave the flag as it is.  TPF_EINVAL
 * for a bad id or value. */
int tpf_set_active(tpf_ctx* ctx, int32_t id, int32_t active);

/* Raw state of domain id (post-collision populations f[9][ny][nx],
 * g[9][ny][nx]) as float64, for checkpoints and tests; either may be NULL. */
int tpf_get_populations(tpf_ctx* ctx, int32_t id, double* f, double* g);

/* Checkpoint / restart of the whole context (same build, same domains).
 * tpf_load checks the whole file before it changes any state: TPF_EINVAL when
 * the file holds another precision, another number of domains or any domain
 * whose parameters differ from the context's in any field; TPF_EIO when the
 * file cannot be opened or is shorter than its header promises.  Only a file
 * that changes while it is being loaded can leave the context part-loaded
 * (TPF_EIO). */
int tpf_save(tpf_ctx* ctx, const char* path);
int tpf_load(tpf_ctx* ctx, const char* path);

/* Tile shape of the fused step kernel: code from tpf_tile_codes(); 0 = let
 * the autotuner choose on the next step.  TPF_EINVAL for unknown codes. */
int tpf_set_tile(tpf_ctx* ctx, int32_t tile_code);
int tpf_get_tile(tpf_ctx* ctx, int32_t* tile_code, int32_t* tile_x, int32_t* tile_y);
/* Number of tile shapes and their codes/extents (arrays of n entries). */
int tpf_tile_codes(int32_t* n, int32_t* codes, int32_t* tx, int32_t* ty);
/* Times every tile shape on the current domains for `steps` steps each and
 * keeps the fastest for all of them (clearing per-domain codes); the state is
 * restored afterwards.  best_ms may be NULL. */
int tpf_autotune(tpf_ctx* ctx, int32_t steps, double* best_ms);

/* Size class of a domain for the per-class autotuner: precision, whether it
 * carries the flux S (rho1 != rho2), and nx, ny rounded up to powers of two,
 * written as "p32_s0_w256_h512" into buf (len bytes, NUL-terminated).  Host
 * only.  TPF_EINVAL for bad arguments or a short buffer. */
int tpf_size_class(int32_t precision, int32_t nx, int32_t ny, int32_t has_s, char* buf, int32_t len);

/* Per-size-class autotuning.  For every class among the domains that take
 * part in the steps, the tile code comes from the cache file cache_path when
 * it holds that class for this device (architecture and compute-unit count),
 * else every tile shape is timed for `steps` steps on the class's domains
 * alone and the fastest kept.  Each domain then runs its class's code:
 * tpf_step launches one kernel per (code, S) group.  The state of every
 * domain is restored.  When classes were timed and cache_path is not NULL,
 * the cache is rewritten (its other entries kept; written to a temporary
 * file and renamed); a file of another format or device is replaced.
 * n_timed (may be NULL) = classes that were timed.  TPF_EINVAL in launch mode
 * 2 (which chooses one code itself) or for steps <= 0; TPF_EIO if the cache
 * cannot be written.  tpf_set_tile and tpf_autotune return to one code for
 * all domains.  Cache format (JSON, one entry per line):
 *   {"format": "tpf-autotune-1", "device": "gfx950:256", "entries": {
 *     "p32_s0_w256_h256": {"code": 21, "ms_per_step": 0.05}, ... }} */
int tpf_autotune_classes(tpf_ctx* ctx, int32_t steps, const char* cache_path, int32_t* n_timed);

/* Tile code domain id runs in the next step. */
int tpf_domain_tile(tpf_ctx* ctx, int32_t id, int32_t* code);

/* Launch mode of tpf_step / tpf_run_to_residual: 0 = one kernel launch per
 * step over all live domains' tiles; 1 = one persistent launch per call that
 * advances all live domains through the steps: a work queue of (step, tile)
 * items with a per-domain barrier between steps (device-scope counters).
 * Under tpf_run_to_residual the residual checks run inside the launch (one
 * check item per live domain every check_every steps and at the last step)
 * and a converged or non-finite domain leaves the queue there, with the same
 * statuses, step counts and residuals as in mode 0.  Mode 1 applies when
 * every live domain runs one of the strip codes 8-10 or strip-group codes
 * 17, 20-24 and no domain has open ends; otherwise the calls fall back to
 * one launch per step.  Both modes give the same state up to the rounding
 * of separately compiled kernels.
 * A barrier wait that exceeds its spin bound (it cannot in a correct run)
 * makes the call return TPF_EDEVICE.  2 = one launch per step with the tile
 * shape re-chosen at every call (and every residual check) from the live
 * domains: the largest of the shapes 17, 9, 8, 2, 1 that still gives one
 * wavefront per resident slot of the device, so that batches whose domains
 * retire keep the device filled; the FP32 state may then differ from mode 0
 * by rounding (the tile kernel contracts multiply-adds differently).
 * TPF_EINVAL for other modes. */
int tpf_set_launch_mode(tpf_ctx* ctx, int32_t mode);

/* Bytes a step moves by definition per node: 18 population reads and writes,
 * phi0 and the lagged fields read and written. */
int tpf_bytes_per_node(tpf_ctx* ctx, int32_t id, double* bytes);

/* Number of domains; nodes of domain id. */
int tpf_num_domains(tpf_ctx* ctx, int32_t* n);
int tpf_domain_size(tpf_ctx* ctx, int32_t id, int32_t* nx, int32_t* ny);

/* Derived per-domain constants for inspection: k, gamma[3], gammaT, eta. */
int tpf_derived(tpf_ctx* ctx, int32_t id, double* k, double* gamma3, double* gammaT, double* eta);

/* Average duration (ms) per launch of the fused step kernel over the steps
 * issued since the last call while timing was enabled, measured with HIP
 * events on the context's stream: one event pair around the launches of each
 * tpf_step call (or each persistent launch), so the average includes the short
 * gaps between back-to-back launches and no event sits between two of them. */
int tpf_kernel_timing(tpf_ctx* ctx, int32_t enable, double* avg_ms, int64_t* launches);

/* Roofline context, not part of the method: device-to-device copy of `bytes`
 * bytes from src to dst (caller-owned device buffers, 16-byte aligned, bytes
 * a positive multiple of 16, not overlapping) with 16-byte vector loads and
 * stores, plain (nontemporal = 0) or with the non-temporal hint (1), as a
 * grid-stride loop over 65536 workgroups of 256 threads; two untimed copies,
 * then `reps` copies timed with HIP events on hip_stream (NULL: the null
 * stream).  *ms_per_copy receives the mean duration of one copy; it moves
 * 2 * bytes of HBM traffic.  TPF_EINVAL for bad arguments, TPF_EDEVICE for a
 * HIP error. */
int tpf_copy_bandwidth(const void* src, void* dst, uint64_t bytes, int32_t nontemporal, int32_t reps,
                       void* hip_stream, double* ms_per_copy);

const char* tpf_strerror(int32_t status);
void tpf_destroy(tpf_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* TPF_H */
