// Host side of the 3D C ABI declared in include/tpf3.h: domains, per-domain
// constants (Sec. 2.2-3 with the 3D pressure constants), arena layout, the
// tile table of the fused D3Q15 kernel, the FP64 mass sum and read-out.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "tpf.h"
#include "tpf3.h"
#include "tpf3_kernels.h"
#include "tpf3_launch.h"

using namespace tpf3;

namespace {

struct HostDomain3 {
    tpf3_domain_params p;
    std::vector<double> phi0, phi1;
    DomDev3 dev;
    int64_t steps = 0;
    double gamma[3] = {0, 0, 0}, gammaT = 0, eta = 0, k = 0;
};

constexpr int kMassBlocks = 512;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
bool has_s(const tpf3_domain_params& p) { return p.rho[1] != p.rho[2]; }

}  // namespace

struct tpf3_ctx {
    int precision = 64;
    hipStream_t stream = nullptr;
    std::vector<HostDomain3> doms;
    bool finalized = false;
    char* arena = nullptr;
    uint64_t arena_bytes = 0;
    bool own_arena = false;
    DomDev3* d_doms = nullptr;
    int4* d_tiles = nullptr;
    double* d_part = nullptr;
    double* d_scratch = nullptr;   // max over domains of 30 N doubles
    int ty = 0;                    // 0 = automatic
    std::vector<int4> tiles;
    int tiles_noS = 0;
    bool tiles_dirty = true;
    bool timing = false;
    std::vector<hipEvent_t> ev;
    std::vector<int64_t> ev_steps;
};

#define HIP3_OK(expr)                                                                     \
    do {                                                                                  \
        hipError_t _e = (expr);                                                           \
        if (_e != hipSuccess) {                                                           \
            std::fprintf(stderr, "tpf3: %s failed: %s\n", #expr, hipGetErrorString(_e)); \
            return TPF_EDEVICE;                                                           \
        }                                                                                 \
    } while (0)

extern "C" void tpf3_default_params(tpf3_domain_params* p, int32_t nx, int32_t ny, int32_t nz) {
    std::memset(p, 0, sizeof(*p));
    p->nx = nx;
    p->ny = ny;
    p->nz = nz;
    p->periodic[0] = 1;
    p->periodic[1] = 1;
    p->periodic[2] = 0;
    p->d0 = 0.4;
    p->D = 4.0;
    p->sigma12 = 0.01;
    p->theta = M_PI / 3.0;
    for (int i = 0; i < 3; ++i) {
        p->rho[i] = 1.0;
        p->mu[i] = 0.15;
    }
    p->M_deg = 0.004;
    p->tau_phi = 0.8;
    for (int i = 0; i < 4; ++i) p->s_phi[i] = p->s_g[i] = 1.0;
    p->s_g[2] = p->s_g[3] = 0.5;   // NS s3, s4 (reading: 1 diverges beside a saturated diffuse solid)
}

// k(theta, kappa) of Eq. (eq-kk), Young's law and the spreading coefficients.
static void derive_gamma3(const tpf3_domain_params& p, double& k, double g[3], double& gT) {
    const double th = p.theta;
    const double sg = (th > 0.5 * M_PI) ? 1.0 : (th < 0.5 * M_PI ? -1.0 : 0.0);
    const double sn = std::sin(0.25 * M_PI * std::cos(th));
    k = 9.0 / (1.0 + p.kappa) * (1.0 + 2.0 * sg * sn * sn);
    const double s12 = p.sigma12, s01 = k * s12, s02 = s01 + s12 * std::cos(th);
    g[0] = s01 + s02 - s12;
    g[1] = s01 + s12 - s02;
    g[2] = s02 + s12 - s01;
    gT = 3.0 / (1.0 / g[0] + 1.0 / g[1] + 1.0 / g[2]);
}

static int validate3(const tpf3_domain_params& p) {
    if (p.nx < 3 || p.ny < 3 || p.nz < 3) return TPF_EINVAL;
    if ((int64_t)p.nx * p.ny * p.nz * 15 >= ((int64_t)1 << 31)) return TPF_EINVAL;
    if (!(p.theta > 0.0 && p.theta < M_PI) || !(p.d0 > 0.0 && p.d0 < 1.0) || !(p.tau_phi > 0.5)) return TPF_EINVAL;
    if (!(p.D > 0.0) || !(p.sigma12 > 0.0) || !(p.kappa > -1.0)) return TPF_EINVAL;
    for (int i = 0; i < 3; ++i)
        if (!(p.rho[i] > 0.0) || !(p.mu[i] > 0.0) || !std::isfinite(p.Fb[i]) || !std::isfinite(p.u_wall[i]))
            return TPF_EINVAL;
    if (!(p.M_cst >= 0.0 && p.M_deg >= 0.0 && p.M_cst + p.M_deg > 0.0)) return TPF_EINVAL;
    for (int i = 0; i < 4; ++i)
        if (!(p.s_phi[i] > 0.0 && p.s_phi[i] < 2.0) || !(p.s_g[i] > 0.0 && p.s_g[i] < 2.0)) return TPF_EINVAL;
    double k, g[3], gT;
    derive_gamma3(p, k, g, gT);
    return (g[0] > 0 && g[1] > 0 && g[2] > 0) ? TPF_OK : TPF_EINVAL;
}

template <typename T>
static void fill_kconst3(const tpf3_domain_params& p, const HostDomain3& h, KConst3<T>& K) {
    const double c2 = p.d0;
    const double w0 = 1.0 - 3.0 * c2 + 2.0 * c2 * c2;
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
    K.inv_cfa = (T)(2.0 / (1.0 - c2));
    K.inv_cfb = (T)(1.0 / c2);
    K.Fbx = (T)p.Fb[0];
    K.Fby = (T)p.Fb[1];
    K.Fbz = (T)p.Fb[2];
    K.uwx = (T)p.u_wall[0];
    K.uwy = (T)p.u_wall[1];
    K.uwz = (T)p.u_wall[2];
    K.gauge = (T)p.rho_gauge;
    // p = c_s^2/(1 - w0) [ sum_{i != 0} g_i + (1/2 + H) u.grad(rho) - w0 B/(c^2 - c_s^2)
    //      + (K/c^2)(dt/2) d_t B ],  3D: K = 1 - 2 d0,
    //      H = K [ (1 - d0)/s0 - (3 - 7 d0)/s2a + (1 - 3 d0) ]   (Sec. 3)
    const double Kp = 1.0 - 2.0 * c2;
    K.pfac = (T)(c2 / (1.0 - w0));
    K.pw = (T)(w0 / (1.0 - c2));
    K.Kp = (T)Kp;
    K.AH = (T)(Kp * ((1.0 - c2) / p.s_g[0] + (1.0 - 3.0 * c2)));
    K.BH = (T)(Kp * (3.0 - 7.0 * c2));
}

static void fill_constants3(HostDomain3& h) {
    const tpf3_domain_params& p = h.p;
    derive_gamma3(p, h.k, h.gamma, h.gammaT);
    h.eta = (p.M_cst + p.M_deg) / (h.gamma[1] * (p.tau_phi - 0.5) * p.d0);
    DomDev3& d = h.dev;
    d.nx = p.nx;
    d.ny = p.ny;
    d.nz = p.nz;
    d.px = p.periodic[0] ? 1 : 0;
    d.py = p.periodic[1] ? 1 : 0;
    d.pz = p.periodic[2] ? 1 : 0;
    d.has_s = has_s(p) ? 1 : 0;
    // the s2a term of H vanishes with its coefficient K (3 - 7 d0) (reading R11')
    d.bh_zero = ((1.0 - 2.0 * p.d0) * (3.0 - 7.0 * p.d0) == 0.0) ? 1 : 0;
    fill_kconst3<double>(p, h, d.kd);
    fill_kconst3<float>(p, h, d.kf);
}

static size_t nodes(const tpf3_domain_params& p) { return (size_t)p.nx * p.ny * p.nz; }

static size_t domain_bytes3(const tpf3_domain_params& p, int prec) {
    const size_t e = prec == 32 ? 4 : 8, N = nodes(p);
    size_t b = align_up(60 * N * e, 256) + align_up(N * e, 256) + align_up(3 * N * e, 256) + align_up(N * e, 256);
    if (has_s(p)) b += align_up(6 * N * e, 256) + align_up(6 * N * e, 256);
    return b;
}

static int auto_ty(const tpf3_ctx* c) {
    bool anyS = false;
    for (auto& h : c->doms) anyS |= has_s(h.p);
    if (c->precision == 32) return anyS ? 4 : 8;
    return anyS ? 2 : 4;
}

static int cur_ty(const tpf3_ctx* c) { return c->ty ? c->ty : auto_ty(c); }

static size_t max_tiles3(const tpf3_ctx* c) {
    size_t t = 0;
    for (auto& h : c->doms)
        t += (size_t)((h.p.nx + 63) / 64) * ((h.p.ny + 1) / 2) * ((h.p.nz + kTileZ3 - 1) / kTileZ3);
    return t;
}

static size_t total_bytes3(const tpf3_ctx* c) {
    size_t b = 0, maxn = 0;
    for (auto& h : c->doms) {
        b += domain_bytes3(h.p, c->precision);
        maxn = std::max(maxn, nodes(h.p));
    }
    b += align_up(c->doms.size() * sizeof(DomDev3), 256);
    b += align_up(max_tiles3(c) * sizeof(int4), 256);
    b += align_up(2 * kMassBlocks * sizeof(double) + 8, 256);
    b += align_up(30 * maxn * sizeof(double), 256);
    return b;
}

static int upload3(tpf3_ctx* c) {
    std::vector<DomDev3> v;
    for (auto& h : c->doms) v.push_back(h.dev);
    HIP3_OK(hipMemcpyAsync(c->d_doms, v.data(), v.size() * sizeof(DomDev3), hipMemcpyHostToDevice, c->stream));
    HIP3_OK(hipStreamSynchronize(c->stream));
    return TPF_OK;
}

// Tile table of the given domains: domains without S first, then with S.
static int build_tiles3(tpf3_ctx* c, const std::vector<int>& which, std::vector<int4>& out, int* n_noS) {
    const int ty = cur_ty(c);
    out.clear();
    int split = 0;
    for (int pass = 0; pass < 2; ++pass) {
        for (int di : which) {
            const auto& p = c->doms[di].p;
            if (has_s(p) != (pass == 1)) continue;
            for (int z = 0; z < p.nz; z += kTileZ3)
                for (int y = 0; y < p.ny; y += ty)
                    for (int x = 0; x < p.nx; x += 64) out.push_back(make_int4(di, x, y, z));
        }
        if (pass == 0) split = (int)out.size();
    }
    *n_noS = split;
    if (out.size() > max_tiles3(c)) return TPF_EINVAL;
    if (!out.empty())
        HIP3_OK(hipMemcpyAsync(c->d_tiles, out.data(), out.size() * sizeof(int4), hipMemcpyHostToDevice, c->stream));
    HIP3_OK(hipStreamSynchronize(c->stream));
    return TPF_OK;
}

static hipError_t launch_split(tpf3_ctx* c, int mode, int ntiles, int n_noS, int offset, double* mom) {
    auto run = c->precision == 32 ? launch3_f32 : launch3_f64;
    const int ty = cur_ty(c);
    Tile3Launch a{c->stream, c->d_doms, c->d_tiles, n_noS, offset, mom};
    hipError_t e = run(ty, false, mode, a);
    if (e != hipSuccess) return e;
    a.tiles = c->d_tiles + n_noS;
    a.ntiles = ntiles - n_noS;
    return run(ty, true, mode, a);
}

extern "C" int tpf3_create(tpf3_ctx** out, int32_t precision, void* hip_stream) {
    if (!out || (precision != 32 && precision != 64)) return TPF_EINVAL;
    tpf3_ctx* c = new tpf3_ctx();  // no device work before tpf3_finalize
    c->precision = precision;
    c->stream = (hipStream_t)hip_stream;
    *out = c;
    return TPF_OK;
}

extern "C" int tpf3_add_domain(tpf3_ctx* c, const tpf3_domain_params* p, const double* phi0, const double* phi1,
                               int32_t* id) {
    if (!c || !p || !phi0 || !phi1) return TPF_EINVAL;
    if (c->finalized) return TPF_ESTATE;
    const int rc = validate3(*p);
    if (rc) return rc;
    HostDomain3 h;
    h.p = *p;
    const size_t N = nodes(*p);
    h.phi0.assign(phi0, phi0 + N);
    h.phi1.assign(phi1, phi1 + N);
    c->doms.push_back(std::move(h));
    if (id) *id = (int32_t)c->doms.size() - 1;
    return TPF_OK;
}

extern "C" int tpf3_arena_bytes(tpf3_ctx* c, uint64_t* bytes) {
    if (!c || !bytes) return TPF_EINVAL;
    *bytes = total_bytes3(c);
    return TPF_OK;
}

extern "C" int tpf3_finalize(tpf3_ctx* c, void* arena, uint64_t arena_bytes) {
    if (!c) return TPF_EINVAL;
    if (c->finalized || c->doms.empty()) return TPF_ESTATE;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return TPF_EDEVICE;
    const size_t need = total_bytes3(c);
    if (arena) {
        if (arena_bytes < need || ((uintptr_t)arena & 255)) return TPF_EINVAL;
        c->arena = (char*)arena;
    } else {
        HIP3_OK(hipMalloc((void**)&c->arena, need));
        c->own_arena = true;
    }
    c->arena_bytes = need;
    const size_t e = c->precision == 32 ? 4 : 8;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = c->arena + off;
        off += align_up(bytes, 256);
        return (void*)p;
    };
    for (auto& h : c->doms) {
        fill_constants3(h);
        const size_t N = nodes(h.p);
        DomDev3& d = h.dev;
        char* pops = (char*)take(60 * N * e);
        d.f[0] = pops;
        d.f[1] = pops + 15 * N * e;
        d.g[0] = pops + 30 * N * e;
        d.g[1] = pops + 45 * N * e;
        d.phi0 = take(N * e);
        d.lagA = take(3 * N * e);
        d.lagB = take(N * e);
        d.lagC = nullptr;
        d.psi[0] = d.psi[1] = nullptr;
        if (has_s(h.p)) {
            d.lagC = take(6 * N * e);
            char* ps = (char*)take(6 * N * e);
            d.psi[0] = ps;
            d.psi[1] = ps + 3 * N * e;
        }
        d.parity = 0;
        d.live = 1;
    }
    c->d_doms = (DomDev3*)take(c->doms.size() * sizeof(DomDev3));
    c->d_tiles = (int4*)take(max_tiles3(c) * sizeof(int4));
    c->d_part = (double*)take(2 * kMassBlocks * sizeof(double) + 8);
    size_t maxn = 0;
    for (auto& h : c->doms) maxn = std::max(maxn, nodes(h.p));
    c->d_scratch = (double*)take(30 * maxn * sizeof(double));
    if (off > need) return TPF_EDEVICE;
    int rc = upload3(c);
    if (rc) return rc;
    for (size_t i = 0; i < c->doms.size(); ++i) {
        auto& h = c->doms[i];
        const size_t N = nodes(h.p);
        // phi0 in the storage precision; the initial phi1 through the scratch
        if (c->precision == 32) {
            std::vector<float> f0(h.phi0.begin(), h.phi0.end());
            HIP3_OK(hipMemcpyAsync(h.dev.phi0, f0.data(), N * 4, hipMemcpyHostToDevice, c->stream));
            HIP3_OK(hipMemcpyAsync(c->d_scratch, h.phi1.data(), N * 8, hipMemcpyHostToDevice, c->stream));
            hipLaunchKernelGGL(init3_kernel<float>, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, c->stream,
                               c->d_doms, (int)i, c->d_scratch);
        } else {
            HIP3_OK(hipMemcpyAsync(h.dev.phi0, h.phi0.data(), N * 8, hipMemcpyHostToDevice, c->stream));
            HIP3_OK(hipMemcpyAsync(c->d_scratch, h.phi1.data(), N * 8, hipMemcpyHostToDevice, c->stream));
            hipLaunchKernelGGL(init3_kernel<double>, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, c->stream,
                               c->d_doms, (int)i, c->d_scratch);
        }
        HIP3_OK(hipGetLastError());
        HIP3_OK(hipStreamSynchronize(c->stream));
    }
    c->finalized = true;
    c->tiles_dirty = true;
    return TPF_OK;
}

extern "C" int tpf3_step(tpf3_ctx* c, int64_t nsteps) {
    if (!c || nsteps < 0) return TPF_EINVAL;
    if (!c->finalized) return TPF_ESTATE;
    if (nsteps == 0) return TPF_OK;
    if (c->tiles_dirty) {
        std::vector<int> all(c->doms.size());
        for (size_t i = 0; i < all.size(); ++i) all[i] = (int)i;
        int rc = build_tiles3(c, all, c->tiles, &c->tiles_noS);
        if (rc) return rc;
        c->tiles_dirty = false;
    }
    hipEvent_t a = nullptr, b = nullptr;
    if (c->timing) {
        HIP3_OK(hipEventCreate(&a));
        HIP3_OK(hipEventCreate(&b));
        HIP3_OK(hipEventRecord(a, c->stream));
    }
    const int nt = (int)c->tiles.size();
    for (int64_t s = 0; s < nsteps; ++s) HIP3_OK(launch_split(c, 0, nt, c->tiles_noS, (int)(s & 1), nullptr));
    if (c->timing) {
        HIP3_OK(hipEventRecord(b, c->stream));
        c->ev.push_back(a);
        c->ev.push_back(b);
        c->ev_steps.push_back(nsteps);
    }
    for (auto& h : c->doms) {
        h.steps += nsteps;
        h.dev.parity = (int)((h.dev.parity + nsteps) & 1);
    }
    return upload3(c);
}

extern "C" int tpf3_read_moments(tpf3_ctx* c, int32_t id, double* phi1, double* ux, double* uy, double* uz, double* p) {
    if (!c || id < 0 || id >= (int32_t)c->doms.size()) return TPF_EINVAL;
    if (!c->finalized) return TPF_ESTATE;
    std::vector<int4> t;
    int n_noS = 0;
    int rc = build_tiles3(c, {id}, t, &n_noS);
    if (rc) return rc;
    HIP3_OK(launch_split(c, 1, (int)t.size(), n_noS, 0, c->d_scratch));
    const size_t N = nodes(c->doms[id].p);
    double* outs[5] = {phi1, ux, uy, uz, p};
    for (int k = 0; k < 5; ++k)
        if (outs[k])
            HIP3_OK(hipMemcpyAsync(outs[k], c->d_scratch + k * N, N * 8, hipMemcpyDeviceToHost, c->stream));
    HIP3_OK(hipStreamSynchronize(c->stream));
    c->tiles_dirty = true;   // the step table was overwritten
    return TPF_OK;
}

extern "C" int tpf3_read_mass(tpf3_ctx* c, int32_t id, double* mass) {
    if (!c || !mass || id < 0 || id >= (int32_t)c->doms.size()) return TPF_EINVAL;
    if (!c->finalized) return TPF_ESTATE;
    if (c->precision == 32)
        hipLaunchKernelGGL(mass3_partials<float>, dim3(kMassBlocks), dim3(256), 0, c->stream, c->d_doms, id, c->d_part);
    else
        hipLaunchKernelGGL(mass3_partials<double>, dim3(kMassBlocks), dim3(256), 0, c->stream, c->d_doms, id, c->d_part);
    HIP3_OK(hipGetLastError());
    hipLaunchKernelGGL(mass3_final, dim3(1), dim3(64), 0, c->stream, c->d_part, kMassBlocks,
                       c->d_part + 2 * kMassBlocks);
    HIP3_OK(hipGetLastError());
    HIP3_OK(hipMemcpyAsync(mass, c->d_part + 2 * kMassBlocks, 8, hipMemcpyDeviceToHost, c->stream));
    HIP3_OK(hipStreamSynchronize(c->stream));
    return TPF_OK;
}

extern "C" int tpf3_get_populations(tpf3_ctx* c, int32_t id, double* f, double* g) {
    if (!c || id < 0 || id >= (int32_t)c->doms.size()) return TPF_EINVAL;
    if (!c->finalized) return TPF_ESTATE;
    const size_t n = 15 * nodes(c->doms[id].p);
    if (c->precision == 32)
        hipLaunchKernelGGL(export3_populations<float>, dim3(1024), dim3(256), 0, c->stream, c->d_doms, id,
                           c->d_scratch);
    else
        hipLaunchKernelGGL(export3_populations<double>, dim3(1024), dim3(256), 0, c->stream, c->d_doms, id,
                           c->d_scratch);
    HIP3_OK(hipGetLastError());
    if (f) HIP3_OK(hipMemcpyAsync(f, c->d_scratch, n * 8, hipMemcpyDeviceToHost, c->stream));
    if (g) HIP3_OK(hipMemcpyAsync(g, c->d_scratch + n, n * 8, hipMemcpyDeviceToHost, c->stream));
    HIP3_OK(hipStreamSynchronize(c->stream));
    return TPF_OK;
}

extern "C" int tpf3_set_tile(tpf3_ctx* c, int32_t ty) {
    if (!c) return TPF_EINVAL;
    if (ty != 0) {
        bool anyS = false;
        for (auto& h : c->doms) anyS |= has_s(h.p);
        const bool ok = c->precision == 32 ? (ty == 4 || (ty == 8 && !anyS)) : (ty == 2 || (ty == 4 && !anyS));
        if (!ok) return TPF_EINVAL;
    }
    c->ty = ty;
    c->tiles_dirty = true;
    return TPF_OK;
}

extern "C" int tpf3_get_tile(tpf3_ctx* c, int32_t* tx, int32_t* ty, int32_t* tz) {
    if (!c) return TPF_EINVAL;
    if (tx) *tx = 64;
    if (ty) *ty = cur_ty(c);
    if (tz) *tz = kTileZ3;
    return TPF_OK;
}

extern "C" int tpf3_bytes_per_node(tpf3_ctx* c, int32_t id, double* bytes) {
    if (!c || !bytes || id < 0 || id >= (int32_t)c->doms.size()) return TPF_EINVAL;
    const double e = c->precision == 32 ? 4.0 : 8.0;
    // 30 population reads + 30 writes, phi0, lagged phi1 u (3) and B read and
    // written; with S also sym(Su) (6) and S x u (3)
    double fields = 60 + 1 + 2 * 4;
    if (has_s(c->doms[id].p)) fields += 2 * 9;
    *bytes = fields * e;
    return TPF_OK;
}

extern "C" int tpf3_kernel_timing(tpf3_ctx* c, int32_t enable, double* avg_ms, int64_t* launches) {
    if (!c) return TPF_EINVAL;
    double acc = 0.0;
    int64_t n = 0;
    if (!c->ev.empty()) {
        HIP3_OK(hipStreamSynchronize(c->stream));
        for (size_t k = 0; k < c->ev_steps.size(); ++k) {
            float ms = 0.f;
            HIP3_OK(hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]));
            acc += ms;
            n += c->ev_steps[k];
            (void)hipEventDestroy(c->ev[2 * k]);
            (void)hipEventDestroy(c->ev[2 * k + 1]);
        }
        c->ev.clear();
        c->ev_steps.clear();
    }
    if (avg_ms) *avg_ms = n ? acc / (double)n : 0.0;
    if (launches) *launches = n;
    c->timing = enable != 0;
    return TPF_OK;
}

extern "C" void tpf3_destroy(tpf3_ctx* c) {
    if (!c) return;
    for (auto e : c->ev) (void)hipEventDestroy(e);
    if (c->own_arena && c->arena) (void)hipFree(c->arena);
    delete c;
}
