// Host side of the C ABI declared in include/tpf.h: context and domain
// management, per-domain constants (Sec. 2.2-3 of arXiv 2311.05091), arena
// layout, launch of the fused step kernel over all live domains' tiles,
// FP64 reductions, residual-driven retirement, checkpoints and the tile
// autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "tpf.h"
#include "tpf_kernels.h"
#include "tpf_launch.h"

namespace tpf {

struct TileShape {
    int code, tx, ty, threads;
};
// codes are stable across builds.  1, 2: tile kernel (256 threads, whole-tile
// LDS window, 64 x 4 and 64 x 8 nodes: the small tiles of launch mode 2);
// 8-10: strip kernel (one wavefront marching down a 64-column strip of ty
// rows; also the persistent launch); 17, 18, 20: groups of 4 or 2 strip
// wavefronts per workgroup advancing in lockstep (groups of 8 would need more
// than the 64 KB of LDS a workgroup may hold in FP64 with the S flux); 21,
// 22: groups of 4 strips of 32 or 64 rows with the register budget left to
// the compiler; 23, 24: code 22 with non-temporal loads of the pulled
// populations of both lattices (23; each strip's halo cells with plain
// loads) or of the NS lattice only (24).  Codes 3-7
// and 11-16 (other tile sizes, a pipelined strip and a five-waves strip) were
// never the fastest on any workload measured and are no longer built.
static const TileShape kTiles[] = {{1, 64, 4, 256},   {2, 64, 8, 256},   {8, 64, 16, 64},
                                   {9, 64, 32, 64},   {10, 64, 64, 64},  {17, 256, 32, 256},
                                   {18, 128, 32, 128}, {20, 256, 16, 256}, {21, 256, 32, 256},
                                   {22, 256, 64, 256}, {23, 256, 64, 256}, {24, 256, 64, 256}};
static const int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);
static const int kDefaultTile = 9;

struct HostDomain {
    tpf_domain_params p;
    std::vector<double> phi0, phi1;
    DomDev dev;               // host copy of the device descriptor
    int64_t steps = 0;
    int32_t status = TPF_OK;  // TPF_OK, TPF_ENAN, or 1 = retired (residual)
    bool active = true;       // false: left out of every step until set active again
    double mass = NAN, residual = NAN, snap_norm = NAN;
    int64_t snap_step = -1;
    double k = 0, gamma[3] = {0, 0, 0}, gammaT = 0, eta = 0;
    size_t off = 0, bytes = 0;  // arena slice
    int tile = 0;               // tile code of this domain (0: the context's)
};

// A contiguous run of the tile table whose tiles share one kernel instance.
struct TileGroup {
    int code;
    bool s;
    int begin, count;
};

}  // namespace tpf

using namespace tpf;

struct tpf_ctx {
    int precision = 64;
    hipStream_t stream = nullptr;
    std::vector<HostDomain> doms;
    bool finalized = false;
    char* arena = nullptr;
    uint64_t arena_bytes = 0;
    bool own_arena = false;
    // device-side tables inside the arena
    DomDev* d_doms = nullptr;
    int4* d_tiles = nullptr;
    int* d_domlist = nullptr;
    int* d_open = nullptr;       // ids of the domains with open ends in x
    int n_open = 0;
    double* d_partials = nullptr;
    double* d_red = nullptr;   // [ndom][4]
    double* d_scratch = nullptr;  // max(4 N, 18 N) doubles
    size_t max_tiles = 0;
    int tile_code = kDefaultTile;
    bool tile_from_user = false;
    bool tuned = false;
    int launch_mode = 0;
    // persistent launcher state (inside the arena)
    int* d_ctl = nullptr;        // [3]: next item, failure flag, domains still live
    int* d_retired = nullptr;    // [ndom] call-relative step at which a domain left (-1: live)
    int* d_lastchk = nullptr;    // [ndom] call-relative step of its last residual check
    int* d_done = nullptr;       // [ndom]
    int* d_dom_tiles = nullptr;  // [ndom]
    int n_cu = 0;
    std::string device;          // architecture name and compute units (autotune cache key)
    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<int64_t> ev_steps;
    double t_acc_ms = 0;
    int64_t t_launches = 0;
    // current tile table
    std::vector<int4> tiles;
    std::vector<TileGroup> groups;  // one per (tile code, S) among the live domains
    std::vector<int> live_list;
    int tiles_code_built = -1;
    bool tiles_dirty = true;
};

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// A domain takes part in the steps while it is finite, not retired and active.
static bool stepping(const HostDomain& h) { return h.status == TPF_OK && h.active; }

static const TileShape* find_tile(int code) {
    for (int i = 0; i < kNumTiles; ++i)
        if (kTiles[i].code == code) return &kTiles[i];
    return nullptr;
}

// Tile code a domain runs: its own (set by the per-class autotuner) unless
// launch mode 2 chooses one code for all.
static int eff_code(const tpf_ctx* c, const HostDomain& h) {
    return (c->launch_mode != 2 && h.tile) ? h.tile : c->tile_code;
}

#define HIP_OK(expr)                                  \
    do {                                              \
        hipError_t _e = (expr);                       \
        if (_e != hipSuccess) {                       \
            std::fprintf(stderr, "tpf: %s failed: %s\n", #expr, hipGetErrorString(_e)); \
            return TPF_EDEVICE;                       \
        }                                             \
    } while (0)

// ---------------------------------------------------------------------------
// Parameters and derived constants
// ---------------------------------------------------------------------------
extern "C" void tpf_default_params(tpf_domain_params* p, int32_t nx, int32_t ny) {
    std::memset(p, 0, sizeof(*p));
    p->nx = nx;
    p->ny = ny;
    p->periodic_x = 1;
    p->periodic_y = 0;
    p->d0 = 0.5;
    p->D = 4.0;
    p->sigma12 = 0.01;
    p->theta = M_PI / 3.0;
    p->kappa = 0.0;
    for (int i = 0; i < 3; ++i) {
        p->rho[i] = 1.0;
        p->mu[i] = 0.15;
    }
    p->M_cst = 0.0;
    p->M_deg = 0.01;
    p->tau_phi = 0.8;
    for (int i = 0; i < 4; ++i) {
        p->s_phi[i] = 1.0;
        p->s_g[i] = 1.0;
    }
}

// sigma01 = k sigma12 with k(theta, kappa) of Eq. (eq-kk); Young's law gives
// sigma02; the spreading coefficients follow from the pairwise tensions.
static void derive_gamma(const tpf_domain_params& p, double& k, double g[3], double& gT) {
    const double th = p.theta;
    const double sg = (th > 0.5 * M_PI) ? 1.0 : (th < 0.5 * M_PI ? -1.0 : 0.0);
    const double sn = std::sin(0.25 * M_PI * std::cos(th));
    k = 9.0 / (1.0 + p.kappa) * (1.0 + 2.0 * sg * sn * sn);
    const double s12 = p.sigma12;
    const double s01 = k * s12;
    const double s02 = s01 + s12 * std::cos(th);
    g[0] = s01 + s02 - s12;
    g[1] = s01 + s12 - s02;
    g[2] = s02 + s12 - s01;
    gT = 3.0 / (1.0 / g[0] + 1.0 / g[1] + 1.0 / g[2]);
}

// Row stride of a domain's fields in elements: nx rounded up to 64, the
// width of a strip, so that every strip row starts on a cache-line boundary
// (a 64-lane load then touches whole lines, not a partial line at each end).
// The columns past nx are never read.
static int pitch_of(int nx) { return (nx + 63) / 64 * 64; }

static int validate(const tpf_domain_params& p) {
    if (p.nx < 3 || p.ny < 3) return TPF_EINVAL;
    if ((int64_t)pitch_of(p.nx) * p.ny * 9 >= (int64_t)1 << 31) return TPF_EINVAL;
    if (!(p.theta > 0.0 && p.theta < M_PI)) return TPF_EINVAL;
    if (!(p.d0 > 0.0 && p.d0 < 1.0)) return TPF_EINVAL;
    if (!(p.tau_phi > 0.5)) return TPF_EINVAL;
    if (!(p.D > 0.0) || !(p.sigma12 > 0.0)) return TPF_EINVAL;
    for (int i = 0; i < 3; ++i)
        if (!(p.rho[i] > 0.0) || !(p.mu[i] > 0.0)) return TPF_EINVAL;
    if (!(p.M_cst >= 0.0 && p.M_deg >= 0.0 && p.M_cst + p.M_deg > 0.0)) return TPF_EINVAL;
    for (int i = 0; i < 4; ++i)
        if (!(p.s_phi[i] > 0.0 && p.s_phi[i] < 2.0) || !(p.s_g[i] > 0.0 && p.s_g[i] < 2.0))
            return TPF_EINVAL;
    if (!(p.kappa > -1.0)) return TPF_EINVAL;
    if (!std::isfinite(p.omega_wall) || !std::isfinite(p.wall_center[0]) || !std::isfinite(p.wall_center[1]) ||
        !std::isfinite(p.u_wall[0]) || !std::isfinite(p.u_wall[1]))
        return TPF_EINVAL;
    if (p.open_x != 0 && p.open_x != 1) return TPF_EINVAL;
    if (p.open_x && (p.periodic_x || p.nx < 4 || (p.inlet_type != 0 && p.inlet_type != 1))) return TPF_EINVAL;
    if (!std::isfinite(p.p_in) || !std::isfinite(p.u_in) || !std::isfinite(p.p_out) || !std::isfinite(p.phi1_in))
        return TPF_EINVAL;
    double k, g[3], gT;
    derive_gamma(p, k, g, gT);
    if (!(g[0] > 0 && g[1] > 0 && g[2] > 0)) return TPF_EINVAL;
    return TPF_OK;
}

template <typename T>
static void fill_kconst(const tpf_domain_params& p, const HostDomain& h, KConst<T>& K) {
    const double c2 = p.d0;
    const double w0 = (1.0 - c2) * (1.0 - c2);
    K.c2 = (T)c2;
    K.w0 = (T)w0;
    K.gam0 = (T)h.gamma[0];
    K.gam1 = (T)h.gamma[1];
    K.gam2 = (T)h.gamma[2];
    K.gT3 = (T)(h.gammaT / 3.0);
    K.inv_gam0 = (T)(1.0 / h.gamma[0]);
    K.inv_gam2 = (T)(1.0 / h.gamma[2]);
    K.c12D = (T)(12.0 / p.D);
    K.c3D4 = (T)(0.75 * p.D);
    K.eta = (T)h.eta;
    K.Mcst = (T)p.M_cst;
    K.Mdeg = (T)p.M_deg;
    K.Mdeg_frac = (T)(p.M_deg / (p.M_cst + p.M_deg));
    K.s0 = (T)p.s_phi[0];
    K.s1 = (T)(1.0 / p.tau_phi);
    K.s2 = (T)p.s_phi[1];
    K.s3 = (T)p.s_phi[2];
    K.s4 = (T)p.s_phi[3];
    K.rho0 = (T)p.rho[0];
    K.rho1 = (T)p.rho[1];
    K.rho2 = (T)p.rho[2];
    K.muv0 = (T)p.mu[0];
    K.muv1 = (T)p.mu[1];
    K.muv2 = (T)p.mu[2];
    K.drho0 = (T)(p.rho[0] - p.rho[2]);
    K.drho1 = (T)(p.rho[1] - p.rho[2]);
    K.Sfac = (T)((p.rho[1] - p.rho[2]) / h.gamma[1]);
    K.sg0 = (T)p.s_g[0];
    K.sg1 = (T)p.s_g[1];
    K.sg3 = (T)p.s_g[2];
    K.sg4 = (T)p.s_g[3];
    // mu/(rho (1 - phi0)) = (1/s2a - 1/2)(c^2 - c_s^2)/2 = (1/s2b - 1/2) c_s^2  (Sec. 3)
    K.inv_cfa = (T)(2.0 / (1.0 - c2));
    K.inv_cfb = (T)(1.0 / c2);
    K.Fbx = (T)p.Fb[0];
    K.Fby = (T)p.Fb[1];
    K.uwx = (T)p.u_wall[0];
    K.uwy = (T)p.u_wall[1];
    K.om = (T)p.omega_wall;
    K.xc = (T)p.wall_center[0];
    K.yc = (T)p.wall_center[1];
    K.gauge = (T)p.rho_gauge;
    // p = c_s^2/(1 - w0) [ sum_{i != 0} g_i + (1/2 + H) u.grad(rho)
    //      - w0 (rho u - S).u/(c^2 - c_s^2) + (K/c^2)(dt/2) d_t((rho u - S).u) ]
    // 2D: K = 1 - d0, H = K [ (1 - d0)/s0 - (2 - 4 d0)/s2a + (1 - 3 d0)/2 ]
    K.pfac = (T)(c2 / (1.0 - w0));
    K.pw = (T)(w0 / (1.0 - c2));
    K.Kp = (T)(1.0 - c2);
    K.AH = (T)((1.0 - c2) / p.s_g[0] + 0.5 * (1.0 - 3.0 * c2));
    K.BH = (T)(2.0 - 4.0 * c2);
    K.p_in = (T)p.p_in;
    K.u_in = (T)p.u_in;
    K.p_out = (T)p.p_out;
    K.phi1_in = (T)p.phi1_in;
}

static void fill_constants(HostDomain& h) {
    const tpf_domain_params& p = h.p;
    DomDev& d = h.dev;
    derive_gamma(p, h.k, h.gamma, h.gammaT);
    // (M_cst + M_deg)/gamma_1 = (1/s1 - 1/2) eta c_s^2  (Sec. 3)
    h.eta = (p.M_cst + p.M_deg) / (h.gamma[1] * (p.tau_phi - 0.5) * p.d0);
    d.nx = p.nx;
    d.ny = p.ny;
    d.px = p.periodic_x ? 1 : 0;
    d.py = p.periodic_y ? 1 : 0;
    d.has_s = (p.rho[1] != p.rho[2]) ? 1 : 0;
    d.bh_zero = (2.0 - 4.0 * p.d0 == 0.0) ? 1 : 0;
    d.open_x = p.open_x ? 1 : 0;
    d.inlet_type = p.inlet_type;
    fill_kconst<double>(p, h, d.kd);
    fill_kconst<float>(p, h, d.kf);
}

// ---------------------------------------------------------------------------
// Arena layout
// ---------------------------------------------------------------------------
static size_t domain_bytes(const HostDomain& h, int prec) {
    const size_t e = prec == 32 ? 4 : 8;
    const size_t N = (size_t)pitch_of(h.p.nx) * h.p.ny;   // fields: rows of pitch elements
    const bool S = h.p.rho[1] != h.p.rho[2];
    size_t b = 0;
    b += align_up(4 * 9 * N * e, 256);       // f[2], g[2]
    b += align_up(N * e, 256);               // phi0
    b += align_up(2 * N * e, 256);           // A
    b += align_up(N * e, 256);               // B
    if (S) b += align_up(3 * N * e, 256) + align_up(2 * N * e, 256);  // C, psi[2]
    b += align_up((size_t)h.p.nx * h.p.ny * 8, 256);  // snap (float64, [ny][nx])
    if (h.p.open_x) b += align_up(2 * kBndFields * (size_t)h.p.ny * e, 256);  // bnd
    return b;
}

// Capacity of the tile table: every domain at its own largest tile count
// (domains may run different codes).
static void count_tiles(const tpf_ctx* c, size_t& max_tiles) {
    max_tiles = 0;
    for (auto& h : c->doms) {
        size_t m = 0;
        for (int i = 0; i < kNumTiles; ++i)
            m = std::max(m, (size_t)((h.p.nx + kTiles[i].tx - 1) / kTiles[i].tx) *
                                ((h.p.ny + kTiles[i].ty - 1) / kTiles[i].ty));
        max_tiles += m;
    }
}

static size_t max_nodes(const tpf_ctx* c) {
    size_t m = 0;
    for (auto& h : c->doms) m = std::max(m, (size_t)h.p.nx * h.p.ny);
    return m;
}

static size_t total_bytes(tpf_ctx* c) {
    size_t b = 0;
    for (auto& h : c->doms) b += domain_bytes(h, c->precision);
    size_t nd = c->doms.size();
    size_t mt;
    count_tiles(c, mt);
    b += align_up(nd * sizeof(DomDev), 256);
    b += align_up(mt * sizeof(int4), 256);
    b += align_up(nd * sizeof(int), 256);
    b += align_up(nd * sizeof(int), 256);  // open-domain list
    b += align_up(nd * kRedMaxBlocks * 7 * sizeof(double), 256);
    b += align_up(nd * 4 * sizeof(double), 256);
    b += align_up(18 * max_nodes(c) * sizeof(double), 256);
    b += align_up(3 * sizeof(int), 256) + 4 * align_up(nd * sizeof(int), 256);
    return b;
}

// ---------------------------------------------------------------------------
// Launch helpers (the kernel instances live in tpf_launch_f32/f64.hip)
// ---------------------------------------------------------------------------
// Launches the step (or moments) kernel once per group of the tile table,
// each with the instance of its tile code and S flag.
static hipError_t launch_step(tpf_ctx* c, int mode, const std::vector<TileGroup>& groups, int offset,
                              double* mom) {
    auto run = c->precision == 32 ? launch_tiles_f32 : launch_tiles_f64;
    for (const TileGroup& g : groups) {
        TileLaunch a{c->stream, c->d_doms, c->d_tiles + g.begin, g.count, offset, mom};
        hipError_t e = run(g.code, g.s, mode, a);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Host -> device upload of all descriptors (small; issued on the stream).
static int upload_descriptors(tpf_ctx* c) {
    std::vector<DomDev> v;
    v.reserve(c->doms.size());
    for (auto& h : c->doms) v.push_back(h.dev);
    HIP_OK(hipMemcpyAsync(c->d_doms, v.data(), v.size() * sizeof(DomDev), hipMemcpyHostToDevice,
                          c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    return TPF_OK;
}

// Tile table for a set of domains (all live ones, or one for moments),
// grouped by (tile code, S) in increasing code order, domains without the
// flux S first within a code, so each group runs one kernel instance.
static int build_tiles(tpf_ctx* c, const std::vector<int>& which, std::vector<int4>& out,
                       std::vector<TileGroup>& groups) {
    std::map<std::pair<int, int>, std::vector<int>> by;
    for (int di : which) by[{eff_code(c, c->doms[di]), c->doms[di].dev.has_s ? 1 : 0}].push_back(di);
    out.clear();
    groups.clear();
    for (auto& kv : by) {
        const TileShape* ts = find_tile(kv.first.first);
        if (!ts) return TPF_EINVAL;
        TileGroup g{kv.first.first, kv.first.second != 0, (int)out.size(), 0};
        for (int di : kv.second) {
            const auto& h = c->doms[di];
            for (int y = 0; y < h.p.ny; y += ts->ty)
                for (int x = 0; x < h.p.nx; x += ts->tx) out.push_back(make_int4(di, x, y, 0));
        }
        g.count = (int)out.size() - g.begin;
        groups.push_back(g);
    }
    if (out.size() > c->max_tiles) return TPF_EINVAL;
    if (!out.empty())
        HIP_OK(hipMemcpyAsync(c->d_tiles, out.data(), out.size() * sizeof(int4),
                              hipMemcpyHostToDevice, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    return TPF_OK;
}

static int refresh_live(tpf_ctx* c) {
    std::vector<int> live;
    for (size_t i = 0; i < c->doms.size(); ++i)
        if (stepping(c->doms[i])) live.push_back((int)i);
    if (live != c->live_list || c->tiles_dirty || c->tiles_code_built != c->tile_code) {
        c->live_list = live;
        int rc = build_tiles(c, live, c->tiles, c->groups);
        if (rc) return rc;
        c->tiles_code_built = c->tile_code;
        c->tiles_dirty = false;
    }
    return TPF_OK;
}

// The persistent launch runs one tile code with a persistent form (strips
// 8-10, groups 17, 20-24) for every live domain, and no open ends.
static bool persistent_ok(const tpf_ctx* c) {
    if (c->launch_mode != 1 || c->groups.empty() || c->n_open > 0) return false;
    const int code = c->groups[0].code;
    for (const TileGroup& g : c->groups)
        if (g.code != code) return false;
    return persistent_code(code);
}

// n steps of all live domains in persistent launches (chunks keep the item
// count within 31 bits).  check_every > 0: the residual checks of
// tpf_run_to_residual run inside the launches (every check_every steps of
// the call and at its last step); a domain whose residual falls below tol,
// or that turns non-finite, leaves the queue at that check; each chunk
// starts from the domains still live.  The entry snapshot is the caller's.
// Returns TPF_EDEVICE if a wait ever timed out.
static int run_persistent(tpf_ctx* c, int64_t n, int check_every = 0, double tol = 0.0) {
    const int nd = (int)c->doms.size();
    // every domain starts the call live (-1) with its last check at call step 0
    // (the kernels read both arrays also when no checks run)
    std::vector<int> minus(nd, -1), zero(nd, 0);
    HIP_OK(hipMemcpyAsync(c->d_retired, minus.data(), nd * sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIP_OK(hipMemcpyAsync(c->d_lastchk, zero.data(), nd * sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    int64_t done_steps = 0;
    while (done_steps < n) {
        int rc = refresh_live(c);
        if (rc) return rc;
        if (c->live_list.empty()) break;
        const int ntiles = (int)c->tiles.size(), nlive = (int)c->live_list.size();
        std::vector<int> per(nd, 0);
        for (const int4& t : c->tiles) per[t.x]++;
        HIP_OK(hipMemcpyAsync(c->d_dom_tiles, per.data(), per.size() * sizeof(int), hipMemcpyHostToDevice,
                              c->stream));
        HIP_OK(hipMemcpyAsync(c->d_domlist, c->live_list.data(), nlive * sizeof(int), hipMemcpyHostToDevice,
                              c->stream));
        bool S = false;  // some live domain has S: the S-capable instance
        for (const TileGroup& g : c->groups) S = S || g.s;
        const int code = c->groups[0].code;
        const int64_t per_step = ntiles + (check_every > 0 ? nlive : 0);
        int64_t chunk = std::max<int64_t>(1, ((int64_t)1 << 30) / per_step);
        if (check_every > 0) chunk = std::max<int64_t>(check_every, chunk / check_every * check_every);
        if (chunk * per_step >= ((int64_t)1 << 31)) return TPF_EINVAL;   // a table beyond 2^31 items per chunk
        const int64_t m = std::min<int64_t>(n - done_steps, chunk);
        hipLaunchKernelGGL(zero_ints, dim3(1), dim3(64), 0, c->stream, c->d_ctl, 3);
        hipLaunchKernelGGL(zero_ints, dim3((nd + 255) / 256), dim3(256), 0, c->stream, c->d_done, nd);
        HIP_OK(hipGetLastError());
        HIP_OK(hipMemcpyAsync(c->d_ctl + 2, &nlive, sizeof(int), hipMemcpyHostToDevice, c->stream));
        hipEvent_t ea = nullptr, eb = nullptr;
        if (c->timing) {
            HIP_OK(hipEventCreate(&ea));
            HIP_OK(hipEventCreate(&eb));
            HIP_OK(hipEventRecord(ea, c->stream));
        }
        PersistArgs pa{c->d_tiles, ntiles, c->d_domlist, nlive, (int)m, (int)done_steps, (int)n, check_every, tol,
                       c->d_dom_tiles, c->d_ctl, c->d_done, c->d_retired, c->d_lastchk, c->d_red, 1 << 22};
        const PersistentLaunch pl{c->stream, c->d_doms, pa, c->n_cu};
        HIP_OK(c->precision == 32 ? launch_persistent_f32(code, S, pl) : launch_persistent_f64(code, S, pl));
        if (c->timing) {
            HIP_OK(hipEventRecord(eb, c->stream));
            c->ev_pool.push_back(ea);
            c->ev_pool.push_back(eb);
            c->ev_steps.push_back(m);
        }
        int ctl[3] = {0, 0, 0};
        std::vector<int> retired(nd, -1);
        std::vector<double> stats(4 * nd, 0.0);
        HIP_OK(hipMemcpyAsync(ctl, c->d_ctl, sizeof(ctl), hipMemcpyDeviceToHost, c->stream));
        if (check_every > 0) {
            HIP_OK(hipMemcpyAsync(retired.data(), c->d_retired, nd * sizeof(int), hipMemcpyDeviceToHost, c->stream));
            HIP_OK(hipMemcpyAsync(stats.data(), c->d_red, 4 * nd * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        }
        HIP_OK(hipStreamSynchronize(c->stream));
        if (ctl[1]) return TPF_EDEVICE;
        for (int di : c->live_list) {
            auto& h = c->doms[di];
            int64_t took = m;
            if (check_every > 0) {
                const int r = retired[di];
                if (r >= 0) took = r + 1;   // left at the check after its step r of this chunk
                // the domain's last check within this chunk (call-relative step cs), if any
                const int64_t first = done_steps + 1, last = done_steps + took;
                int64_t cs = -1;
                if (r >= 0 || last == n) cs = last;
                else if (last / check_every * check_every >= first) cs = last / check_every * check_every;
                if (cs >= 0) {
                    h.residual = stats[4 * di + 0];
                    h.mass = stats[4 * di + 1];
                    h.snap_step = h.steps + (cs - done_steps);
                }
                if (r >= 0) h.status = stats[4 * di + 3] != 0.0 ? TPF_ENAN : 1;
            }
            h.steps += took;
            h.dev.parity = (int)((h.dev.parity + took) & 1);
        }
        int urc = upload_descriptors(c);
        if (urc) return urc;
        done_steps += m;
    }
    return TPF_OK;
}

// Advances the live domains by n steps with one launch per step.  Domains
// share the step count within the call, so each one's buffer parity is
// (parity at entry + step index) & 1.
// Launch mode 2: the tile shape follows the live work.  Candidates from the
// largest tile down; the first whose tile table gives at least one
// wavefront per resident slot (16 per compute unit) is taken, else the
// smallest.  As domains retire, smaller tiles keep the device filled and a
// step's latency short.
static void adapt_tile(tpf_ctx* c) {
    static const int kLadder[] = {17, 9, 8, 2, 1};
    std::vector<int> live;
    for (size_t i = 0; i < c->doms.size(); ++i)
        if (stepping(c->doms[i])) live.push_back((int)i);
    const int64_t slots = (int64_t)16 * std::max(c->n_cu, 1);
    int pick = kLadder[sizeof(kLadder) / sizeof(kLadder[0]) - 1];
    for (int code : kLadder) {
        const TileShape* ts = find_tile(code);
        int64_t waves = 0;
        for (int di : live) {
            const auto& p = c->doms[di].p;
            waves += (int64_t)((p.nx + ts->tx - 1) / ts->tx) * ((p.ny + ts->ty - 1) / ts->ty) * (ts->threads / 64);
        }
        if (waves >= slots) {
            pick = code;
            break;
        }
    }
    if (pick != c->tile_code) c->tiles_dirty = true;
    c->tile_code = pick;
}

// Non-equilibrium extrapolation at the open ends of every open domain, after
// the step launched with the same step offset.
static hipError_t launch_open_bc(tpf_ctx* c, int offset) {
    int maxny = 1;
    for (auto& h : c->doms)
        if (h.p.open_x) maxny = std::max(maxny, h.p.ny);
    const dim3 grid((unsigned)((2 * maxny + 255) / 256), (unsigned)c->n_open);
    if (c->precision == 32)
        hipLaunchKernelGGL(open_bc_kernel<float>, grid, dim3(256), 0, c->stream, c->d_doms, c->d_open, c->n_open,
                           offset);
    else
        hipLaunchKernelGGL(open_bc_kernel<double>, grid, dim3(256), 0, c->stream, c->d_doms, c->d_open, c->n_open,
                           offset);
    return hipGetLastError();
}

static int run_steps(tpf_ctx* c, int64_t n) {
    if (n <= 0) return TPF_OK;
    if (c->launch_mode == 2) adapt_tile(c);
    int rc = refresh_live(c);
    if (rc) return rc;
    if (c->live_list.empty()) return TPF_OK;
    for (int di : c->live_list) {
        c->doms[di].dev.live = 1;
    }
    for (size_t i = 0; i < c->doms.size(); ++i)
        if (!stepping(c->doms[i])) c->doms[i].dev.live = 0;
    rc = upload_descriptors(c);
    if (rc) return rc;
    if (persistent_ok(c)) return run_persistent(c, n);
    // timing: one event pair around the call's n back-to-back launches (an
    // event between every two launches measurably slowed the run: 282 against
    // 275 us per step on the 4096 x 2048 workload), so the average per launch
    // includes the short gaps between launches
    hipEvent_t ta = nullptr, tb = nullptr;
    if (c->timing) {
        HIP_OK(hipEventCreate(&ta));
        HIP_OK(hipEventCreate(&tb));
        HIP_OK(hipEventRecord(ta, c->stream));
    }
    for (int64_t s = 0; s < n; ++s) {
        HIP_OK(launch_step(c, kModeStep, c->groups, (int)(s & 1), nullptr));
        if (c->n_open > 0) HIP_OK(launch_open_bc(c, (int)(s & 1)));
    }
    if (c->timing) {
        HIP_OK(hipEventRecord(tb, c->stream));
        c->ev_pool.push_back(ta);
        c->ev_pool.push_back(tb);
        c->ev_steps.push_back(n);
    }
    for (int di : c->live_list) {
        auto& h = c->doms[di];
        h.steps += n;
        h.dev.parity = (int)((h.dev.parity + n) & 1);
    }
    return upload_descriptors(c);
}

// Mass and residual of the given domains (FP64, compensated).
static int reduce(tpf_ctx* c, const std::vector<int>& which, bool update_snap) {
    if (which.empty()) return TPF_OK;
    HIP_OK(hipMemcpyAsync(c->d_domlist, which.data(), which.size() * sizeof(int),
                          hipMemcpyHostToDevice, c->stream));
    int maxny = 1;
    for (int di : which) maxny = std::max(maxny, c->doms[di].p.ny);
    const int nblk = std::min(kRedMaxBlocks, maxny);
    dim3 grid(nblk, (unsigned)which.size());
    if (c->precision == 32)
        hipLaunchKernelGGL(reduce_partials<float>, grid, dim3(kRedThreads), 0, c->stream, c->d_doms,
                           c->d_domlist, update_snap ? 1 : 0, c->d_partials);
    else
        hipLaunchKernelGGL(reduce_partials<double>, grid, dim3(kRedThreads), 0, c->stream, c->d_doms,
                           c->d_domlist, update_snap ? 1 : 0, c->d_partials);
    HIP_OK(hipGetLastError());
    hipLaunchKernelGGL(reduce_final, dim3((which.size() + 63) / 64), dim3(64), 0, c->stream,
                       c->d_domlist, (int)which.size(), nblk, c->d_partials, c->d_red);
    HIP_OK(hipGetLastError());
    std::vector<double> red(4 * c->doms.size());
    HIP_OK(hipMemcpyAsync(red.data(), c->d_red, red.size() * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    for (int di : which) {
        auto& h = c->doms[di];
        h.mass = red[4 * di + 0];
        const double d2 = red[4 * di + 1], n2 = red[4 * di + 2], bad = red[4 * di + 3];
        if (bad > 0 || !std::isfinite(h.mass)) h.status = TPF_ENAN;
        if (update_snap) {
            if (h.snap_step >= 0 && h.steps > h.snap_step && n2 > 0)
                h.residual = std::sqrt(d2) / ((double)(h.steps - h.snap_step) * std::sqrt(n2));
            h.snap_step = h.steps;
        }
    }
    return TPF_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" int tpf_create(tpf_ctx** out, int32_t precision, void* hip_stream) {
    if (!out || (precision != 32 && precision != 64)) return TPF_EINVAL;
    tpf_ctx* c = new tpf_ctx();  // no device work before tpf_finalize
    c->precision = precision;
    c->stream = (hipStream_t)hip_stream;
    *out = c;
    return TPF_OK;
}

extern "C" int tpf_add_domain(tpf_ctx* c, const tpf_domain_params* p, const double* phi0,
                              const double* phi1, int32_t* id) {
    if (!c || !p || !phi0 || !phi1) return TPF_EINVAL;
    if (c->finalized) return TPF_ESTATE;
    int rc = validate(*p);
    if (rc) return rc;
    HostDomain h;
    h.p = *p;
    const size_t N = (size_t)p->nx * p->ny;
    h.phi0.assign(phi0, phi0 + N);
    h.phi1.assign(phi1, phi1 + N);
    fill_constants(h);
    c->doms.push_back(std::move(h));
    if (id) *id = (int32_t)c->doms.size() - 1;
    return TPF_OK;
}

extern "C" int tpf_arena_bytes(tpf_ctx* c, uint64_t* bytes) {
    if (!c || !bytes) return TPF_EINVAL;
    if (c->doms.empty()) return TPF_ESTATE;
    *bytes = total_bytes(c);
    return TPF_OK;
}

static int init_domain(tpf_ctx* c, int di, const double* phi1) {
    auto& h = c->doms[di];
    const size_t N = (size_t)h.p.nx * h.p.ny;
    HIP_OK(hipMemcpyAsync(c->d_scratch, phi1, N * sizeof(double), hipMemcpyHostToDevice, c->stream));
    const int nb = (int)((N + 255) / 256);
    if (c->precision == 32)
        hipLaunchKernelGGL(init_kernel<float>, dim3(nb), dim3(256), 0, c->stream, c->d_doms, di,
                           (const double*)c->d_scratch);
    else
        hipLaunchKernelGGL(init_kernel<double>, dim3(nb), dim3(256), 0, c->stream, c->d_doms, di,
                           (const double*)c->d_scratch);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(c->stream));
    h.steps = 0;
    h.status = TPF_OK;
    h.residual = NAN;
    h.snap_step = -1;
    return TPF_OK;
}

template <typename T>
static int upload_phi0(tpf_ctx* c, HostDomain& h) {
    const int nx = h.p.nx, ny = h.p.ny, ld = pitch_of(nx);
    std::vector<T> v((size_t)ld * ny, T(0));   // rows of pitch elements, zero padding
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) v[(size_t)y * ld + x] = T(h.phi0[(size_t)y * nx + x]);
    HIP_OK(hipMemcpyAsync(h.dev.phi0, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    return TPF_OK;
}

extern "C" int tpf_finalize(tpf_ctx* c, void* arena, uint64_t arena_bytes) {
    if (!c) return TPF_EINVAL;
    if (c->finalized) return TPF_ESTATE;
    if (c->doms.empty()) return TPF_ESTATE;
    {
        int ndev = 0;
        const hipError_t e = hipGetDeviceCount(&ndev);
        if (e != hipSuccess || ndev <= 0) {
            std::fprintf(stderr, "tpf: no usable device (%s, %d devices)\n", hipGetErrorString(e), ndev);
            return TPF_EDEVICE;
        }
    }
    const uint64_t need = total_bytes(c);
    if (arena) {
        if (arena_bytes < need || ((uintptr_t)arena & 255)) return TPF_EINVAL;
        c->arena = (char*)arena;
        c->own_arena = false;
    } else {
        void* p = nullptr;
        HIP_OK(hipMalloc(&p, need));
        c->arena = (char*)p;
        c->own_arena = true;
    }
    c->arena_bytes = need;
    const size_t e = c->precision == 32 ? 4 : 8;
    size_t off = 0;
    auto take = [&](size_t b) {
        char* p = c->arena + off;
        off += align_up(b, 256);
        return (void*)p;
    };
    for (auto& h : c->doms) {
        const size_t N = (size_t)pitch_of(h.p.nx) * h.p.ny;
        DomDev& d = h.dev;
        d.pitch = pitch_of(h.p.nx);
        char* base = (char*)take(4 * 9 * N * e);
        d.f[0] = base;
        d.f[1] = base + 9 * N * e;
        d.g[0] = base + 18 * N * e;
        d.g[1] = base + 27 * N * e;
        d.phi0 = take(N * e);
        d.lagA = take(2 * N * e);
        d.lagB = take(N * e);
        if (d.has_s) {
            d.lagC = take(3 * N * e);
            char* ps = (char*)take(2 * N * e);
            d.psi[0] = ps;
            d.psi[1] = ps + N * e;
        } else {
            d.lagC = nullptr;
            d.psi[0] = d.psi[1] = nullptr;
        }
        d.snap = (double*)take((size_t)h.p.nx * h.p.ny * 8);
        d.bnd = h.p.open_x ? take(2 * kBndFields * (size_t)h.p.ny * e) : nullptr;
        d.parity = 0;
        d.live = 1;
    }
    size_t nd = c->doms.size();
    count_tiles(c, c->max_tiles);
    c->d_doms = (DomDev*)take(nd * sizeof(DomDev));
    c->d_tiles = (int4*)take(c->max_tiles * sizeof(int4));
    c->d_domlist = (int*)take(nd * sizeof(int));
    c->d_open = (int*)take(nd * sizeof(int));
    c->d_partials = (double*)take(nd * kRedMaxBlocks * 7 * sizeof(double));
    c->d_red = (double*)take(nd * 4 * sizeof(double));
    c->d_scratch = (double*)take(18 * max_nodes(c) * sizeof(double));
    c->d_ctl = (int*)take(3 * sizeof(int));
    c->d_retired = (int*)take(nd * sizeof(int));
    c->d_lastchk = (int*)take(nd * sizeof(int));
    c->d_done = (int*)take(nd * sizeof(int));
    c->d_dom_tiles = (int*)take(nd * sizeof(int));
    if (off > need) return TPF_EINVAL;
    {
        int dev = 0;
        HIP_OK(hipGetDevice(&dev));
        hipDeviceProp_t prop;
        HIP_OK(hipGetDeviceProperties(&prop, dev));
        c->n_cu = prop.multiProcessorCount;
        c->device = std::string(prop.gcnArchName) + ":" + std::to_string(prop.multiProcessorCount);
    }
    {
        std::vector<int> open;
        for (size_t i = 0; i < c->doms.size(); ++i)
            if (c->doms[i].p.open_x) open.push_back((int)i);
        c->n_open = (int)open.size();
        if (!open.empty())
            HIP_OK(hipMemcpyAsync(c->d_open, open.data(), open.size() * sizeof(int), hipMemcpyHostToDevice,
                                  c->stream));
    }
    int rc = upload_descriptors(c);
    if (rc) return rc;
    for (size_t i = 0; i < c->doms.size(); ++i) {
        rc = c->precision == 32 ? upload_phi0<float>(c, c->doms[i]) : upload_phi0<double>(c, c->doms[i]);
        if (rc) return rc;
        rc = init_domain(c, (int)i, c->doms[i].phi1.data());
        if (rc) return rc;
    }
    c->finalized = true;
    c->tiles_dirty = true;
    std::vector<int> all(c->doms.size());
    for (size_t i = 0; i < all.size(); ++i) all[i] = (int)i;
    return reduce(c, all, true);
}

extern "C" int tpf_step(tpf_ctx* c, int64_t nsteps) {
    if (!c || nsteps < 0) return TPF_EINVAL;
    if (!c->finalized) return TPF_ESTATE;
    return run_steps(c, nsteps);
}

extern "C" int tpf_run_to_residual(tpf_ctx* c, double tol, int32_t check_every, int64_t max_steps,
                                   int64_t* steps_out) {
    if (!c || check_every <= 0 || max_steps < 0 || !(tol >= 0)) return TPF_EINVAL;
    if (!c->finalized) return TPF_ESTATE;
    std::vector<int64_t> start(c->doms.size());
    for (size_t i = 0; i < c->doms.size(); ++i) start[i] = c->doms[i].steps;
    std::vector<int> live;
    for (size_t i = 0; i < c->doms.size(); ++i)
        if (stepping(c->doms[i])) live.push_back((int)i);
    int rc = reduce(c, live, true);  // snapshot at entry
    if (rc) return rc;
    int64_t done = 0;
    bool budget = false;
    // launch mode 1 with a tile code that has a persistent form: the checks
    // run inside the persistent launches and converged domains leave there
    bool in_launch = false;
    if (c->launch_mode == 1 && max_steps > 0 && max_steps < (int64_t)1 << 30) {
        rc = refresh_live(c);
        if (rc) return rc;
        in_launch = persistent_ok(c);
    }
    if (in_launch) {
        for (auto& h : c->doms) h.dev.live = stepping(h) ? 1 : 0;
        rc = upload_descriptors(c);
        if (rc) return rc;
        rc = run_persistent(c, max_steps, check_every, tol);
        if (rc) return rc;
        for (auto& h : c->doms)
            if (stepping(h)) budget = true;
    }
    while (!in_launch) {
        live.clear();
        for (size_t i = 0; i < c->doms.size(); ++i)
            if (stepping(c->doms[i])) live.push_back((int)i);
        if (live.empty()) break;
        if (done >= max_steps) {
            budget = true;
            break;
        }
        const int64_t n = std::min<int64_t>(check_every, max_steps - done);
        rc = run_steps(c, n);
        if (rc) return rc;
        done += n;
        rc = reduce(c, live, true);
        if (rc) return rc;
        for (int di : live) {
            auto& h = c->doms[di];
            if (h.status == TPF_OK && std::isfinite(h.residual) && h.residual < tol) h.status = 1;
        }
    }
    bool nan = false;
    for (size_t i = 0; i < c->doms.size(); ++i) {
        if (steps_out) steps_out[i] = c->doms[i].steps - start[i];
        if (c->doms[i].status == TPF_ENAN) nan = true;
        if (c->doms[i].status == 1) c->doms[i].status = TPF_OK;  // retired domains stay usable
    }
    // retired domains become live again for later calls
    c->tiles_dirty = true;
    if (nan) return TPF_ENAN;
    return budget ? TPF_EBUDGET : TPF_OK;
}

extern "C" int tpf_read_moments(tpf_ctx* c, int32_t id, double* phi1, double* ux, double* uy, double* p) {
    if (!c || id < 0 || id >= (int)c->doms.size()) return TPF_EINVAL;
    if (!c->finalized) return TPF_ESTATE;
    auto& h = c->doms[id];
    const size_t N = (size_t)h.p.nx * h.p.ny;
    std::vector<int4> t;
    std::vector<TileGroup> grp;
    std::vector<int> one = {id};
    int rc = build_tiles(c, one, t, grp);
    if (rc) return rc;
    c->tiles_dirty = true;
    HIP_OK(launch_step(c, kModeMoments, grp, 0, c->d_scratch));
    std::vector<double> buf(4 * N);
    HIP_OK(hipMemcpyAsync(buf.data(), c->d_scratch, 4 * N * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    if (phi1) std::memcpy(phi1, buf.data(), N * sizeof(double));
    if (ux) std::memcpy(ux, buf.data() + N, N * sizeof(double));
    if (uy) std::memcpy(uy, buf.data() + 2 * N, N * sizeof(double));
    if (p) std::memcpy(p, buf.data() + 3 * N, N * sizeof(double));
    return TPF_OK;
}

extern "C" int tpf_flow_rates(tpf_ctx* c, int32_t id, double* q) {
    if (!c || !q || id < 0 || id >= (int)c->doms.size()) return TPF_EINVAL;
    if (!c->finalized) return TPF_ESTATE;
    std::vector<int4> t;
    std::vector<TileGroup> grp;
    std::vector<int> one = {id};
    int rc = build_tiles(c, one, t, grp);
    if (rc) return rc;
    c->tiles_dirty = true;
    HIP_OK(launch_step(c, kModeMoments, grp, 0, c->d_scratch));
    const int N = c->doms[id].p.nx * c->doms[id].p.ny;
    const int nblk = std::max(1, std::min(kRedMaxBlocks, (N + kRedThreads - 1) / kRedThreads));
    if (c->precision == 32)
        hipLaunchKernelGGL(flow_partials<float>, dim3(nblk), dim3(kRedThreads), 0, c->stream, c->d_doms, id,
                           c->d_scratch, c->d_partials);
    else
        hipLaunchKernelGGL(flow_partials<double>, dim3(nblk), dim3(kRedThreads), 0, c->stream, c->d_doms, id,
                           c->d_scratch, c->d_partials);
    HIP_OK(hipGetLastError());
    hipLaunchKernelGGL(flow_final, dim3(1), dim3(64), 0, c->stream, c->d_partials, nblk, c->d_red + 4 * id);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(q, c->d_red + 4 * id, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    return TPF_OK;
}

extern "C" int tpf_read_diag(tpf_ctx* c, int32_t id, double* mass, double* residual, int32_t* status,
                             int64_t* steps) {
    if (!c || id < 0 || id >= (int)c->doms.size()) return TPF_EINVAL;
    if (!c->finalized) return TPF_ESTATE;
    std::vector<int> one = {id};
    int rc = reduce(c, one, false);
    if (rc) return rc;
    auto& h = c->doms[id];
    if (mass) *mass = h.mass;
    if (residual) *residual = h.residual;
    if (status) *status = h.status;
    if (steps) *steps = h.steps;
    return TPF_OK;
}

extern "C" int tpf_set_active(tpf_ctx* c, int32_t id, int32_t active) {
    if (!c || id < 0 || id >= (int)c->doms.size() || (active != 0 && active != 1)) return TPF_EINVAL;
    if (!c->finalized) return TPF_ESTATE;
    c->doms[id].active = active != 0;
    c->tiles_dirty = true;
    return TPF_OK;
}

extern "C" int tpf_set_phi1(tpf_ctx* c, int32_t id, const double* phi1) {
    if (!c || !phi1 || id < 0 || id >= (int)c->doms.size()) return TPF_EINVAL;
    if (!c->finalized) return TPF_ESTATE;
    int rc = init_domain(c, id, phi1);
    if (rc) return rc;
    c->tiles_dirty = true;
    std::vector<int> one = {id};
    return reduce(c, one, true);
}

extern "C" int tpf_get_populations(tpf_ctx* c, int32_t id, double* f, double* g) {
    if (!c || id < 0 || id >= (int)c->doms.size()) return TPF_EINVAL;
    if (!c->finalized) return TPF_ESTATE;
    auto& h = c->doms[id];
    const size_t N = (size_t)h.p.nx * h.p.ny;
    if (c->precision == 32)
        hipLaunchKernelGGL(export_populations<float>, dim3(1024), dim3(256), 0, c->stream, c->d_doms,
                           id, c->d_scratch);
    else
        hipLaunchKernelGGL(export_populations<double>, dim3(1024), dim3(256), 0, c->stream, c->d_doms,
                           id, c->d_scratch);
    HIP_OK(hipGetLastError());
    std::vector<double> buf(18 * N);
    HIP_OK(hipMemcpyAsync(buf.data(), c->d_scratch, 18 * N * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    if (f) std::memcpy(f, buf.data(), 9 * N * sizeof(double));
    if (g) std::memcpy(g, buf.data() + 9 * N, 9 * N * sizeof(double));
    return TPF_OK;
}

// Checkpoint: a header, then per domain its host bookkeeping and its whole
// arena slice (populations of both buffers, phi0, lagged fields, snapshot).
static const char kMagic[8] = {'T', 'P', 'F', 'C', 'K', 'P', 'T', '4'};

static size_t domain_slice_bytes(const tpf_ctx* c, const HostDomain& h) {
    return domain_bytes(h, c->precision);
}

extern "C" int tpf_save(tpf_ctx* c, const char* path) {
    if (!c || !path) return TPF_EINVAL;
    if (!c->finalized) return TPF_ESTATE;
    FILE* fp = std::fopen(path, "wb");
    if (!fp) return TPF_EIO;
    int32_t hdr[3] = {c->precision, (int32_t)c->doms.size(), (int32_t)sizeof(tpf_domain_params)};
    bool ok = std::fwrite(kMagic, 1, 8, fp) == 8 && std::fwrite(hdr, sizeof(hdr), 1, fp) == 1;
    for (auto& h : c->doms) {
        if (!ok) break;
        const size_t b = domain_slice_bytes(c, h);
        std::vector<char> buf(b);
        if (hipMemcpyAsync(buf.data(), h.dev.f[0], b, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess) {
            std::fclose(fp);
            return TPF_EDEVICE;
        }
        int64_t meta_i[3] = {h.steps, h.snap_step, (int64_t)h.status};
        double meta_d[2] = {h.residual, h.mass};
        int32_t par = h.dev.parity;
        ok = std::fwrite(&h.p, sizeof(h.p), 1, fp) == 1 && std::fwrite(meta_i, sizeof(meta_i), 1, fp) == 1 &&
             std::fwrite(meta_d, sizeof(meta_d), 1, fp) == 1 && std::fwrite(&par, 4, 1, fp) == 1 &&
             std::fwrite(buf.data(), 1, b, fp) == b;
    }
    ok = (std::fclose(fp) == 0) && ok;
    return ok ? TPF_OK : TPF_EIO;
}

extern "C" int tpf_load(tpf_ctx* c, const char* path) {
    if (!c || !path) return TPF_EINVAL;
    if (!c->finalized) return TPF_ESTATE;
    FILE* fp = std::fopen(path, "rb");
    if (!fp) return TPF_EIO;
    // Pass 1 validates the whole file before any device memory changes: the
    // header, every domain's full parameter set against the context's, and
    // the presence of every data block (skipped with fseek).
    char magic[8];
    int32_t hdr[3];
    bool ok = std::fread(magic, 1, 8, fp) == 8 && std::fread(hdr, sizeof(hdr), 1, fp) == 1;
    if (!ok) {
        std::fclose(fp);
        return TPF_EIO;
    }
    if (std::memcmp(magic, kMagic, 8) != 0 || hdr[0] != c->precision || hdr[1] != (int32_t)c->doms.size() ||
        hdr[2] != (int32_t)sizeof(tpf_domain_params)) {
        std::fclose(fp);
        return TPF_EINVAL;
    }
    const long data_start = std::ftell(fp);
    const size_t meta_bytes = 3 * sizeof(int64_t) + 2 * sizeof(double) + sizeof(int32_t);
    for (auto& h : c->doms) {
        tpf_domain_params p;
        if (std::fread(&p, sizeof(p), 1, fp) != 1) {
            std::fclose(fp);
            return TPF_EIO;
        }
        if (std::memcmp(&p, &h.p, sizeof(p)) != 0) {
            std::fclose(fp);
            return TPF_EINVAL;
        }
        const size_t skip = meta_bytes + domain_slice_bytes(c, h);
        // the last byte of the block must be readable
        if (std::fseek(fp, (long)skip - 1, SEEK_CUR) != 0 || std::fgetc(fp) == EOF) {
            std::fclose(fp);
            return TPF_EIO;
        }
    }
    // Pass 2 reads and uploads domain by domain.
    if (std::fseek(fp, data_start, SEEK_SET) != 0) {
        std::fclose(fp);
        return TPF_EIO;
    }
    for (auto& h : c->doms) {
        tpf_domain_params p;
        int64_t meta_i[3];
        double meta_d[2];
        int32_t par;
        const size_t b = domain_slice_bytes(c, h);
        std::vector<char> buf(b);
        ok = std::fread(&p, sizeof(p), 1, fp) == 1 && std::fread(meta_i, sizeof(meta_i), 1, fp) == 1 &&
             std::fread(meta_d, sizeof(meta_d), 1, fp) == 1 && std::fread(&par, 4, 1, fp) == 1 &&
             std::fread(buf.data(), 1, b, fp) == b;
        if (!ok) break;  // only if the file changed between the passes
        if (hipMemcpyAsync(h.dev.f[0], buf.data(), b, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess) {
            std::fclose(fp);
            return TPF_EDEVICE;
        }
        h.steps = meta_i[0];
        h.snap_step = meta_i[1];
        h.status = (int32_t)meta_i[2];
        h.residual = meta_d[0];
        h.mass = meta_d[1];
        h.dev.parity = par & 1;
    }
    std::fclose(fp);
    if (!ok) return TPF_EIO;
    c->tiles_dirty = true;
    return upload_descriptors(c);
}

extern "C" int tpf_tile_codes(int32_t* n, int32_t* codes, int32_t* tx, int32_t* ty) {
    if (!n) return TPF_EINVAL;
    *n = kNumTiles;
    for (int i = 0; i < kNumTiles; ++i) {
        if (codes) codes[i] = kTiles[i].code;
        if (tx) tx[i] = kTiles[i].tx;
        if (ty) ty[i] = kTiles[i].ty;
    }
    return TPF_OK;
}

extern "C" int tpf_set_tile(tpf_ctx* c, int32_t code) {
    if (!c) return TPF_EINVAL;
    if (code != 0 && !find_tile(code)) return TPF_EINVAL;
    for (auto& h : c->doms) h.tile = 0;  // one code for all domains again
    c->tiles_dirty = true;
    if (code == 0) {
        c->tile_from_user = false;
        c->tuned = false;
        return TPF_OK;
    }
    c->tile_code = code;
    c->tile_from_user = true;
    return TPF_OK;
}

extern "C" int tpf_get_tile(tpf_ctx* c, int32_t* code, int32_t* tx, int32_t* ty) {
    if (!c) return TPF_EINVAL;
    const TileShape* t = find_tile(c->tile_code);
    if (code) *code = t->code;
    if (tx) *tx = t->tx;
    if (ty) *ty = t->ty;
    return TPF_OK;
}

extern "C" int tpf_domain_tile(tpf_ctx* c, int32_t id, int32_t* code) {
    if (!c || !code || id < 0 || id >= (int)c->doms.size()) return TPF_EINVAL;
    *code = eff_code(c, c->doms[id]);
    return TPF_OK;
}

// Device state of every domain and its bookkeeping, saved before timing runs
// and put back afterwards.
struct SavedState {
    std::vector<std::vector<char>> slices;
    std::vector<HostDomain> meta;
};

static int save_state(tpf_ctx* c, SavedState& st) {
    st.slices.assign(c->doms.size(), {});
    st.meta = c->doms;
    for (size_t i = 0; i < c->doms.size(); ++i) {
        const size_t b = domain_slice_bytes(c, c->doms[i]);
        st.slices[i].resize(b);
        HIP_OK(hipMemcpyAsync(st.slices[i].data(), c->doms[i].dev.f[0], b, hipMemcpyDeviceToHost, c->stream));
    }
    HIP_OK(hipStreamSynchronize(c->stream));
    return TPF_OK;
}

static int restore_state(tpf_ctx* c, const SavedState& st) {
    for (size_t i = 0; i < c->doms.size(); ++i) {
        HIP_OK(hipMemcpyAsync(c->doms[i].dev.f[0], st.slices[i].data(), st.slices[i].size(), hipMemcpyHostToDevice,
                              c->stream));
        auto& h = c->doms[i];
        const auto& m = st.meta[i];
        h.steps = m.steps;
        h.dev.parity = m.dev.parity;
        h.status = m.status;
        h.active = m.active;
        h.residual = m.residual;
        h.snap_step = m.snap_step;
        h.mass = m.mass;
    }
    HIP_OK(hipStreamSynchronize(c->stream));
    c->tiles_dirty = true;
    return upload_descriptors(c);
}

// Average time per step of `steps` steps of the live domains with their
// current codes (after two untimed steps that also build the tile table).
static int time_steps(tpf_ctx* c, int32_t steps, double* per_step_ms) {
    c->tiles_dirty = true;
    int rc = run_steps(c, 2);
    if (rc) return rc;
    hipEvent_t a, b;
    HIP_OK(hipEventCreate(&a));
    HIP_OK(hipEventCreate(&b));
    HIP_OK(hipEventRecord(a, c->stream));
    rc = run_steps(c, steps);
    if (rc) return rc;
    HIP_OK(hipEventRecord(b, c->stream));
    HIP_OK(hipEventSynchronize(b));
    float ms = 0;
    HIP_OK(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *per_step_ms = ms / steps;
    return TPF_OK;
}

extern "C" int tpf_autotune(tpf_ctx* c, int32_t steps, double* best_ms) {
    if (!c || steps <= 0) return TPF_EINVAL;
    if (!c->finalized) return TPF_ESTATE;
    SavedState st;
    int rc = save_state(c, st);
    if (rc) return rc;
    for (auto& h : c->doms) h.tile = 0;
    int best = c->tile_code;
    double best_t = 1e300;
    for (int i = 0; i < kNumTiles; ++i) {
        c->tile_code = kTiles[i].code;
        double per = 0;
        rc = time_steps(c, steps, &per);
        if (rc) return rc;
        if (per < best_t) {
            best_t = per;
            best = kTiles[i].code;
        }
    }
    c->tile_code = best;
    c->tuned = true;
    if (best_ms) *best_ms = best_t;
    return restore_state(c, st);
}

// ---------------------------------------------------------------------------
// Per-size-class autotuning with a JSON cache
// ---------------------------------------------------------------------------
static int pow2_at_least(int v) {
    int p = 1;
    while (p < v && p < (1 << 30)) p <<= 1;
    return p;
}

static std::string size_class(int precision, int nx, int ny, bool has_s) {
    char buf[64];
    std::snprintf(buf, sizeof(buf), "p%d_s%d_w%d_h%d", precision, has_s ? 1 : 0, pow2_at_least(nx),
                  pow2_at_least(ny));
    return buf;
}

extern "C" int tpf_size_class(int32_t precision, int32_t nx, int32_t ny, int32_t has_s, char* buf, int32_t len) {
    if (!buf || len <= 0 || (precision != 32 && precision != 64) || nx < 1 || ny < 1) return TPF_EINVAL;
    const std::string k = size_class(precision, nx, ny, has_s != 0);
    if ((int)k.size() + 1 > len) return TPF_EINVAL;
    std::memcpy(buf, k.c_str(), k.size() + 1);
    return TPF_OK;
}

struct CacheEntry {
    int code;
    double ms;
};

static const char kCacheFormat[] = "tpf-autotune-1";

// Reads the entries of a cache file written by write_cache for this device;
// a missing file, another format or another device give no entries.  Entries
// naming a tile code this build does not have are dropped.
static void read_cache(const char* path, const std::string& device, std::map<std::string, CacheEntry>& out) {
    out.clear();
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[512];
    bool format_ok = false, device_ok = false;
    std::map<std::string, CacheEntry> tmp;
    while (std::fgets(line, sizeof(line), f)) {
        char key[128], val[128];
        int code = 0;
        double ms = 0;
        if (std::sscanf(line, " \"format\": \"%127[^\"]\"", val) == 1) format_ok = std::strcmp(val, kCacheFormat) == 0;
        else if (std::sscanf(line, " \"device\": \"%127[^\"]\"", val) == 1) device_ok = device == val;
        else if (std::sscanf(line, " \"%127[^\"]\": {\"code\": %d, \"ms_per_step\": %lf}", key, &code, &ms) == 3 &&
                 find_tile(code))
            tmp[key] = CacheEntry{code, ms};
    }
    std::fclose(f);
    if (format_ok && device_ok) out = tmp;
}

static bool write_cache(const char* path, const std::string& device, const std::map<std::string, CacheEntry>& e) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return false;
    std::fprintf(f, "{\n  \"format\": \"%s\",\n  \"device\": \"%s\",\n  \"entries\": {\n", kCacheFormat,
                 device.c_str());
    size_t i = 0;
    for (const auto& kv : e)
        std::fprintf(f, "    \"%s\": {\"code\": %d, \"ms_per_step\": %.6g}%s\n", kv.first.c_str(), kv.second.code,
                     kv.second.ms, ++i < e.size() ? "," : "");
    std::fprintf(f, "  }\n}\n");
    const bool ok = std::fclose(f) == 0;
    return ok && std::rename(tmp.c_str(), path) == 0;
}

extern "C" int tpf_autotune_classes(tpf_ctx* c, int32_t steps, const char* cache_path, int32_t* n_timed) {
    if (!c || steps <= 0) return TPF_EINVAL;
    if (!c->finalized) return TPF_ESTATE;
    if (c->launch_mode == 2) return TPF_EINVAL;  // mode 2 chooses the code itself
    // classes of the domains that take part in the steps
    std::map<std::string, std::vector<int>> classes;
    for (size_t i = 0; i < c->doms.size(); ++i) {
        const auto& h = c->doms[i];
        if (!stepping(h)) continue;
        classes[size_class(c->precision, h.p.nx, h.p.ny, h.dev.has_s != 0)].push_back((int)i);
    }
    std::map<std::string, CacheEntry> cache;
    if (cache_path) read_cache(cache_path, c->device, cache);
    SavedState st;
    int rc = save_state(c, st);
    if (rc) return rc;
    int timed = 0;
    std::map<std::string, int> chosen;
    for (const auto& kv : classes) {
        auto it = cache.find(kv.first);
        if (it != cache.end()) {
            chosen[kv.first] = it->second.code;
            continue;
        }
        // time this class alone: every other domain sits out
        for (size_t i = 0; i < c->doms.size(); ++i) c->doms[i].active = false;
        for (int di : kv.second) c->doms[di].active = true;
        int best = kTiles[0].code;
        double best_t = 1e300;
        for (int t = 0; t < kNumTiles; ++t) {
            for (int di : kv.second) c->doms[di].tile = kTiles[t].code;
            double per = 0;
            rc = time_steps(c, steps, &per);
            if (rc) return rc;
            if (per < best_t) {
                best_t = per;
                best = kTiles[t].code;
            }
        }
        chosen[kv.first] = best;
        cache[kv.first] = CacheEntry{best, best_t};
        ++timed;
        rc = restore_state(c, st);  // also brings back the active flags
        if (rc) return rc;
    }
    for (const auto& kv : classes)
        for (int di : kv.second) c->doms[di].tile = chosen[kv.first];
    c->tuned = true;
    rc = restore_state(c, st);
    if (rc) return rc;
    if (n_timed) *n_timed = timed;
    if (cache_path && timed > 0 && !write_cache(cache_path, c->device, cache)) return TPF_EIO;
    return TPF_OK;
}

extern "C" int tpf_set_launch_mode(tpf_ctx* c, int32_t mode) {
    if (!c || mode < 0 || mode > 2) return TPF_EINVAL;
    c->launch_mode = mode;
    return TPF_OK;
}

extern "C" int tpf_bytes_per_node(tpf_ctx* c, int32_t id, double* bytes) {
    if (!c || !bytes || id < 0 || id >= (int)c->doms.size()) return TPF_EINVAL;
    const double e = c->precision == 32 ? 4.0 : 8.0;
    // 18 population reads + 18 writes, phi0, lagged A (2) and B (1) read + written,
    // and with S: C (3) and psi (1) read + written
    const double lag = c->doms[id].dev.has_s ? 7.0 : 3.0;
    *bytes = e * (36.0 + 1.0 + 2.0 * lag);
    return TPF_OK;
}

extern "C" int tpf_num_domains(tpf_ctx* c, int32_t* n) {
    if (!c || !n) return TPF_EINVAL;
    *n = (int32_t)c->doms.size();
    return TPF_OK;
}

extern "C" int tpf_domain_size(tpf_ctx* c, int32_t id, int32_t* nx, int32_t* ny) {
    if (!c || id < 0 || id >= (int)c->doms.size()) return TPF_EINVAL;
    if (nx) *nx = c->doms[id].p.nx;
    if (ny) *ny = c->doms[id].p.ny;
    return TPF_OK;
}

extern "C" int tpf_derived(tpf_ctx* c, int32_t id, double* k, double* gamma3, double* gammaT, double* eta) {
    if (!c || id < 0 || id >= (int)c->doms.size()) return TPF_EINVAL;
    auto& h = c->doms[id];
    double kk, g[3], gT;
    derive_gamma(h.p, kk, g, gT);
    if (k) *k = kk;
    if (gamma3) std::memcpy(gamma3, g, sizeof(g));
    if (gammaT) *gammaT = gT;
    if (eta) *eta = (h.p.M_cst + h.p.M_deg) / (g[1] * (h.p.tau_phi - 0.5) * h.p.d0);
    return TPF_OK;
}

extern "C" int tpf_kernel_timing(tpf_ctx* c, int32_t enable, double* avg_ms, int64_t* launches) {
    if (!c) return TPF_EINVAL;
    double acc = 0;
    int64_t n = 0;
    if (!c->ev_pool.empty()) {
        HIP_OK(hipStreamSynchronize(c->stream));
        for (size_t i = 0; i + 1 < c->ev_pool.size(); i += 2) {
            float ms = 0;
            HIP_OK(hipEventElapsedTime(&ms, c->ev_pool[i], c->ev_pool[i + 1]));
            acc += ms;
            n += c->ev_steps[i / 2];
        }
        for (auto e : c->ev_pool) (void)hipEventDestroy(e);
        c->ev_pool.clear();
        c->ev_steps.clear();
    }
    if (avg_ms) *avg_ms = n ? acc / n : 0.0;
    if (launches) *launches = n;
    c->timing = enable != 0;
    return TPF_OK;
}

// Device copy used as the achievable-bandwidth reference of the roofline.
typedef float v4f __attribute__((ext_vector_type(4)));

template <bool NT>
static __global__ void __launch_bounds__(256) copy16_k(const v4f* __restrict__ a, v4f* __restrict__ b, size_t n) {
    for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        if constexpr (NT) __builtin_nontemporal_store(__builtin_nontemporal_load(a + i), b + i);
        else b[i] = a[i];
    }
}

extern "C" int tpf_copy_bandwidth(const void* src, void* dst, uint64_t bytes, int32_t nontemporal, int32_t reps,
                                  void* hip_stream, double* ms_per_copy) {
    if (!src || !dst || !ms_per_copy || bytes == 0 || bytes % 16 || reps < 1 || (nontemporal != 0 && nontemporal != 1))
        return TPF_EINVAL;
    if ((uintptr_t)src % 16 || (uintptr_t)dst % 16) return TPF_EINVAL;
    const char* s0 = (const char*)src;
    const char* d0 = (const char*)dst;
    if (s0 < d0 + bytes && d0 < s0 + bytes) return TPF_EINVAL;
    const size_t n = bytes / 16;
    const unsigned grid = (unsigned)std::min<size_t>(65536, (n + 255) / 256);
    hipStream_t st = (hipStream_t)hip_stream;
    auto launch = [&]() {
        if (nontemporal)
            hipLaunchKernelGGL(copy16_k<true>, dim3(grid), dim3(256), 0, st, (const v4f*)src, (v4f*)dst, n);
        else
            hipLaunchKernelGGL(copy16_k<false>, dim3(grid), dim3(256), 0, st, (const v4f*)src, (v4f*)dst, n);
    };
    hipEvent_t a = nullptr, b = nullptr;
    float ms = 0;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) {
        launch();
        launch();
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(a, st);
    if (e == hipSuccess) {
        for (int r = 0; r < reps; ++r) launch();
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(b, st);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (e != hipSuccess) {
        std::fprintf(stderr, "tpf: tpf_copy_bandwidth failed: %s\n", hipGetErrorString(e));
        return TPF_EDEVICE;
    }
    *ms_per_copy = ms / reps;
    return TPF_OK;
}

extern "C" const char* tpf_strerror(int32_t s) {
    switch (s) {
        case TPF_OK: return "ok";
        case TPF_EINVAL: return "invalid argument";
        case TPF_EDEVICE: return "device error";
        case TPF_ENAN: return "non-finite values in a domain";
        case TPF_EBUDGET: return "step budget exhausted";
        case TPF_ESTATE: return "call not valid in this state";
        case TPF_EIO: return "checkpoint i/o error";
    }
    return "unknown status";
}

extern "C" void tpf_destroy(tpf_ctx* c) {
    if (!c) return;
    if (!c->ev_pool.empty()) {
        (void)hipStreamSynchronize(c->stream);
        for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    }
    if (c->own_arena && c->arena) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(c->arena);
    }
    delete c;
}
