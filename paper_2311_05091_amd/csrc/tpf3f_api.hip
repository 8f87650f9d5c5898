// Host side of the 3f-model C ABI declared in include/tpf3f.h: domains,
// per-domain constants (Sec. 2.1 spreading coefficients from the pairwise
// tensions, Sec. 3 eta_p and the 2D pressure constants), arena layout, the
// tile table of the fused kernel, the FP64 phase masses and read-out.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "tpf.h"
#include "tpf3f.h"
#include "tpf3f_kernels.h"

using namespace tpf3f;

namespace {

constexpr int kChunk3F = 32;  // rows per strip tile
constexpr int kMassBlocks3F = 512;

struct HostDomain3F {
    tpf3f_domain_params p;
    std::vector<double> phi0, phi1;
    DomDev3F dev;
    double gamma[3] = {0, 0, 0}, gammaT = 0, eta[2] = {0, 0};
};

size_t align_up3f(size_t v, size_t a) { return (v + a - 1) / a * a; }
size_t nodes3f(const tpf3f_domain_params& p) { return (size_t)p.nx * p.ny; }
bool has_s3f(const tpf3f_domain_params& p) { return !(p.rho[0] == p.rho[2] && p.rho[1] == p.rho[2]); }

}  // namespace

struct tpf3f_ctx {
    int precision = 64;
    hipStream_t stream = nullptr;
    std::vector<HostDomain3F> doms;
    bool finalized = false;
    char* arena = nullptr;
    uint64_t arena_bytes = 0;
    bool own_arena = false;
    DomDev3F* d_doms = nullptr;
    int4* d_tiles = nullptr;
    double* d_part = nullptr;
    double* d_scratch = nullptr;  // max over domains of 27 N doubles
    std::vector<int4> tiles;
    int tiles_noS = 0;
    bool tiles_dirty = true;
    bool timing = false;
    std::vector<hipEvent_t> ev;
    std::vector<int64_t> ev_steps;
};

#define HIP3F_OK(expr)                                                                     \
    do {                                                                                   \
        hipError_t _e = (expr);                                                            \
        if (_e != hipSuccess) {                                                            \
            std::fprintf(stderr, "tpf3f: %s failed: %s\n", #expr, hipGetErrorString(_e)); \
            return TPF_EDEVICE;                                                            \
        }                                                                                  \
    } while (0)

// gamma_p from the pairwise tensions (Sec. 2.1).
static void derive_gamma3f(const tpf3f_domain_params& p, double g[3], double& gT) {
    g[0] = p.sigma01 + p.sigma02 - p.sigma12;
    g[1] = p.sigma01 + p.sigma12 - p.sigma02;
    g[2] = p.sigma02 + p.sigma12 - p.sigma01;
    gT = 3.0 / (1.0 / g[0] + 1.0 / g[1] + 1.0 / g[2]);
}

static int validate3f(const tpf3f_domain_params& p) {
    if (p.nx < 3 || p.ny < 3) return TPF_EINVAL;
    if ((int64_t)p.nx * p.ny * 9 >= ((int64_t)1 << 31)) return TPF_EINVAL;
    if (!(p.d0 > 0.0 && p.d0 < 1.0) || !(p.tau_phi > 0.5) || !(p.D > 0.0)) return TPF_EINVAL;
    for (int i = 0; i < 3; ++i)
        if (!(p.rho[i] > 0.0) || !(p.mu[i] > 0.0)) return TPF_EINVAL;
    if (!std::isfinite(p.Fb[0]) || !std::isfinite(p.Fb[1]) || !std::isfinite(p.rho_gauge)) return TPF_EINVAL;
    if (!(p.M_cst >= 0.0 && p.M_deg >= 0.0 && p.M_cst + p.M_deg > 0.0)) return TPF_EINVAL;
    for (int i = 0; i < 4; ++i)
        if (!(p.s_phi[i] > 0.0 && p.s_phi[i] < 2.0) || !(p.s_g[i] > 0.0 && p.s_g[i] < 2.0)) return TPF_EINVAL;
    double g[3], gT;
    derive_gamma3f(p, g, gT);
    return (g[0] > 0 && g[1] > 0 && g[2] > 0) ? TPF_OK : TPF_EINVAL;
}

template <typename T>
static void fill_kconst3f(const tpf3f_domain_params& p, const HostDomain3F& h, KConst3F<T>& K) {
    const double c2 = p.d0, w0 = (1.0 - c2) * (1.0 - c2);
    K.c2 = (T)c2;
    K.w0 = (T)w0;
    for (int i = 0; i < 3; ++i) {
        K.gam[i] = (T)h.gamma[i];
        K.inv_gam[i] = (T)(1.0 / h.gamma[i]);
    }
    K.gT3 = (T)(h.gammaT / 3.0);
    K.c12D = (T)(12.0 / p.D);
    K.c3D4 = (T)(0.75 * p.D);
    K.eta0 = (T)h.eta[0];
    K.eta1 = (T)h.eta[1];
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
    K.Sfac0 = (T)((p.rho[0] - p.rho[2]) / h.gamma[0]);
    K.Sfac1 = (T)((p.rho[1] - p.rho[2]) / h.gamma[1]);
    K.sg0 = (T)p.s_g[0];
    K.sg1 = (T)p.s_g[1];
    K.sg3 = (T)p.s_g[2];
    K.sg4 = (T)p.s_g[3];
    // mu/rho = (1/s2a - 1/2)(c^2 - c_s^2)/2 = (1/s2b - 1/2) c_s^2 (Sec. 3, no solid factor)
    K.inv_cfa = (T)(2.0 / (1.0 - c2));
    K.inv_cfb = (T)(1.0 / c2);
    K.Fbx = (T)p.Fb[0];
    K.Fby = (T)p.Fb[1];
    K.gauge = (T)p.rho_gauge;
    // 2D pressure: K = 1 - d0, H = K [ (1 - d0)/s0 - (2 - 4 d0)/s2a + (1 - 3 d0)/2 ]
    K.pfac = (T)(c2 / (1.0 - w0));
    K.pw = (T)(w0 / (1.0 - c2));
    K.Kp = (T)(1.0 - c2);
    K.AH = (T)((1.0 - c2) / p.s_g[0] + 0.5 * (1.0 - 3.0 * c2));
    K.BH = (T)(2.0 - 4.0 * c2);
}

static void fill_constants3f(HostDomain3F& h) {
    const auto& p = h.p;
    derive_gamma3f(p, h.gamma, h.gammaT);
    for (int q = 0; q < 2; ++q) h.eta[q] = (p.M_cst + p.M_deg) / (h.gamma[q] * (p.tau_phi - 0.5) * p.d0);
    DomDev3F& d = h.dev;
    d.nx = p.nx;
    d.ny = p.ny;
    d.px = p.periodic_x ? 1 : 0;
    d.py = p.periodic_y ? 1 : 0;
    d.has_s = has_s3f(p) ? 1 : 0;
    d.bh_zero = (2.0 - 4.0 * p.d0) == 0.0 ? 1 : 0;
    fill_kconst3f<double>(p, h, d.kd);
    fill_kconst3f<float>(p, h, d.kf);
}

static size_t domain_bytes3f(const tpf3f_domain_params& p, int prec) {
    const size_t e = prec == 32 ? 4 : 8, N = nodes3f(p);
    size_t b = align_up3f(54 * N * e, 256) + align_up3f(4 * N * e, 256) + align_up3f(N * e, 256);
    if (has_s3f(p)) b += align_up3f(3 * N * e, 256) + align_up3f(2 * N * e, 256);
    return b;
}

static size_t max_tiles3f(const tpf3f_ctx* c) {
    size_t t = 0;
    for (auto& h : c->doms) t += (size_t)((h.p.nx + 63) / 64) * ((h.p.ny + kChunk3F - 1) / kChunk3F);
    return t;
}

static size_t total_bytes3f(const tpf3f_ctx* c) {
    size_t b = 0, maxn = 0;
    for (auto& h : c->doms) {
        b += domain_bytes3f(h.p, c->precision);
        maxn = std::max(maxn, nodes3f(h.p));
    }
    b += align_up3f(c->doms.size() * sizeof(DomDev3F), 256);
    b += align_up3f(max_tiles3f(c) * sizeof(int4), 256);
    b += align_up3f(2 * kMassBlocks3F * sizeof(double) + 16, 256);
    b += align_up3f(27 * maxn * sizeof(double), 256);
    return b;
}

static int upload3f(tpf3f_ctx* c) {
    std::vector<DomDev3F> v;
    for (auto& h : c->doms) v.push_back(h.dev);
    HIP3F_OK(hipMemcpyAsync(c->d_doms, v.data(), v.size() * sizeof(DomDev3F), hipMemcpyHostToDevice, c->stream));
    HIP3F_OK(hipStreamSynchronize(c->stream));
    return TPF_OK;
}

// Tile table of the given domains: domains without S first, then with S.
static int build_tiles3f(tpf3f_ctx* c, const std::vector<int>& which, std::vector<int4>& out, int* n_noS) {
    out.clear();
    int split = 0;
    for (int pass = 0; pass < 2; ++pass) {
        for (int di : which) {
            const auto& p = c->doms[di].p;
            if (has_s3f(p) != (pass == 1)) continue;
            for (int y = 0; y < p.ny; y += kChunk3F)
                for (int x = 0; x < p.nx; x += 64) out.push_back(make_int4(di, x, y, 0));
        }
        if (pass == 0) split = (int)out.size();
    }
    *n_noS = split;
    if (out.size() > max_tiles3f(c)) return TPF_EINVAL;
    if (!out.empty())
        HIP3F_OK(hipMemcpyAsync(c->d_tiles, out.data(), out.size() * sizeof(int4), hipMemcpyHostToDevice, c->stream));
    HIP3F_OK(hipStreamSynchronize(c->stream));
    return TPF_OK;
}

template <typename T, bool S, int MODE>
static hipError_t launch3f_t(hipStream_t st, const DomDev3F* doms, const int4* tiles, int n, int offset, double* mom) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((step3f_kernel<T, kChunk3F, S, MODE>), dim3(n), dim3(64), 0, st, doms, tiles, n, offset, mom);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch3f_prec(tpf3f_ctx* c, int mode, int ntiles, int n_noS, int offset, double* mom) {
    const int4* t = c->d_tiles;
    hipError_t e;
    if (mode == kMode3FStep) {
        e = launch3f_t<T, false, kMode3FStep>(c->stream, c->d_doms, t, n_noS, offset, mom);
        if (e == hipSuccess) e = launch3f_t<T, true, kMode3FStep>(c->stream, c->d_doms, t + n_noS, ntiles - n_noS, offset, mom);
    } else {
        e = launch3f_t<T, false, kMode3FMoments>(c->stream, c->d_doms, t, n_noS, offset, mom);
        if (e == hipSuccess)
            e = launch3f_t<T, true, kMode3FMoments>(c->stream, c->d_doms, t + n_noS, ntiles - n_noS, offset, mom);
    }
    return e;
}

static hipError_t launch3f(tpf3f_ctx* c, int mode, int ntiles, int n_noS, int offset, double* mom) {
    return c->precision == 32 ? launch3f_prec<float>(c, mode, ntiles, n_noS, offset, mom)
                              : launch3f_prec<double>(c, mode, ntiles, n_noS, offset, mom);
}

extern "C" void tpf3f_default_params(tpf3f_domain_params* p, int32_t nx, int32_t ny) {
    std::memset(p, 0, sizeof(*p));
    p->nx = nx;
    p->ny = ny;
    p->periodic_x = 1;
    p->periodic_y = 0;
    p->d0 = 0.5;
    p->D = 4.0;
    p->sigma01 = p->sigma02 = p->sigma12 = 0.01;
    for (int i = 0; i < 3; ++i) {
        p->rho[i] = 1.0;
        p->mu[i] = 0.15;
    }
    p->M_deg = 0.01;
    p->tau_phi = 0.8;
    for (int i = 0; i < 4; ++i) p->s_phi[i] = p->s_g[i] = 1.0;
}

extern "C" int tpf3f_create(tpf3f_ctx** out, int32_t precision, void* hip_stream) {
    if (!out || (precision != 32 && precision != 64)) return TPF_EINVAL;
    tpf3f_ctx* c = new tpf3f_ctx();  // no device work before tpf3f_finalize
    c->precision = precision;
    c->stream = (hipStream_t)hip_stream;
    *out = c;
    return TPF_OK;
}

extern "C" int tpf3f_add_domain(tpf3f_ctx* c, const tpf3f_domain_params* p, const double* phi0, const double* phi1,
                                int32_t* id) {
    if (!c || !p || !phi0 || !phi1) return TPF_EINVAL;
    if (c->finalized) return TPF_ESTATE;
    const int rc = validate3f(*p);
    if (rc) return rc;
    HostDomain3F h;
    h.p = *p;
    const size_t N = nodes3f(*p);
    h.phi0.assign(phi0, phi0 + N);
    h.phi1.assign(phi1, phi1 + N);
    c->doms.push_back(std::move(h));
    if (id) *id = (int32_t)c->doms.size() - 1;
    return TPF_OK;
}

extern "C" int tpf3f_arena_bytes(tpf3f_ctx* c, uint64_t* bytes) {
    if (!c || !bytes) return TPF_EINVAL;
    if (c->doms.empty()) return TPF_ESTATE;
    *bytes = total_bytes3f(c);
    return TPF_OK;
}

extern "C" int tpf3f_finalize(tpf3f_ctx* c, void* arena, uint64_t arena_bytes) {
    if (!c) return TPF_EINVAL;
    if (c->finalized || c->doms.empty()) return TPF_ESTATE;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return TPF_EDEVICE;
    const size_t need = total_bytes3f(c);
    if (arena) {
        if (arena_bytes < need || ((uintptr_t)arena & 255)) return TPF_EINVAL;
        c->arena = (char*)arena;
    } else {
        HIP3F_OK(hipMalloc((void**)&c->arena, need));
        c->own_arena = true;
    }
    c->arena_bytes = need;
    const size_t e = c->precision == 32 ? 4 : 8;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* q = c->arena + off;
        off += align_up3f(bytes, 256);
        return (void*)q;
    };
    for (auto& h : c->doms) {
        fill_constants3f(h);
        const size_t N = nodes3f(h.p);
        DomDev3F& d = h.dev;
        char* pops = (char*)take(54 * N * e);
        d.f0[0] = pops;
        d.f0[1] = pops + 9 * N * e;
        d.f1[0] = pops + 18 * N * e;
        d.f1[1] = pops + 27 * N * e;
        d.g[0] = pops + 36 * N * e;
        d.g[1] = pops + 45 * N * e;
        d.lagA = take(4 * N * e);
        d.lagB = take(N * e);
        d.lagC = nullptr;
        d.psi[0] = d.psi[1] = nullptr;
        if (has_s3f(h.p)) {
            d.lagC = take(3 * N * e);
            char* ps = (char*)take(2 * N * e);
            d.psi[0] = ps;
            d.psi[1] = ps + N * e;
        }
        d.parity = 0;
        d.live = 1;
    }
    c->d_doms = (DomDev3F*)take(c->doms.size() * sizeof(DomDev3F));
    c->d_tiles = (int4*)take(max_tiles3f(c) * sizeof(int4));
    c->d_part = (double*)take(2 * kMassBlocks3F * sizeof(double) + 16);
    size_t maxn = 0;
    for (auto& h : c->doms) maxn = std::max(maxn, nodes3f(h.p));
    c->d_scratch = (double*)take(27 * maxn * sizeof(double));
    if (off > need) return TPF_EDEVICE;
    int rc = upload3f(c);
    if (rc) return rc;
    for (size_t i = 0; i < c->doms.size(); ++i) {
        auto& h = c->doms[i];
        const size_t N = nodes3f(h.p);
        HIP3F_OK(hipMemcpyAsync(c->d_scratch, h.phi0.data(), N * 8, hipMemcpyHostToDevice, c->stream));
        HIP3F_OK(hipMemcpyAsync(c->d_scratch + N, h.phi1.data(), N * 8, hipMemcpyHostToDevice, c->stream));
        if (c->precision == 32)
            hipLaunchKernelGGL(init3f_kernel<float>, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, c->stream,
                               c->d_doms, (int)i, c->d_scratch);
        else
            hipLaunchKernelGGL(init3f_kernel<double>, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, c->stream,
                               c->d_doms, (int)i, c->d_scratch);
        HIP3F_OK(hipGetLastError());
        HIP3F_OK(hipStreamSynchronize(c->stream));
    }
    c->finalized = true;
    c->tiles_dirty = true;
    return TPF_OK;
}

extern "C" int tpf3f_step(tpf3f_ctx* c, int64_t nsteps) {
    if (!c || nsteps < 0) return TPF_EINVAL;
    if (!c->finalized) return TPF_ESTATE;
    if (nsteps == 0) return TPF_OK;
    if (c->tiles_dirty) {
        std::vector<int> all(c->doms.size());
        for (size_t i = 0; i < all.size(); ++i) all[i] = (int)i;
        int rc = build_tiles3f(c, all, c->tiles, &c->tiles_noS);
        if (rc) return rc;
        c->tiles_dirty = false;
    }
    hipEvent_t a = nullptr, b = nullptr;
    if (c->timing) {
        HIP3F_OK(hipEventCreate(&a));
        HIP3F_OK(hipEventCreate(&b));
        HIP3F_OK(hipEventRecord(a, c->stream));
    }
    const int nt = (int)c->tiles.size();
    for (int64_t s = 0; s < nsteps; ++s) HIP3F_OK(launch3f(c, kMode3FStep, nt, c->tiles_noS, (int)(s & 1), nullptr));
    if (c->timing) {
        HIP3F_OK(hipEventRecord(b, c->stream));
        c->ev.push_back(a);
        c->ev.push_back(b);
        c->ev_steps.push_back(nsteps);
    }
    for (auto& h : c->doms) h.dev.parity = (int)((h.dev.parity + nsteps) & 1);
    return upload3f(c);
}

extern "C" int tpf3f_read_moments(tpf3f_ctx* c, int32_t id, double* phi0, double* phi1, double* ux, double* uy,
                                  double* p) {
    if (!c || id < 0 || id >= (int32_t)c->doms.size()) return TPF_EINVAL;
    if (!c->finalized) return TPF_ESTATE;
    std::vector<int4> t;
    int n_noS = 0;
    int rc = build_tiles3f(c, {id}, t, &n_noS);
    if (rc) return rc;
    c->tiles_dirty = true;  // the step table was overwritten
    HIP3F_OK(launch3f(c, kMode3FMoments, (int)t.size(), n_noS, 0, c->d_scratch));
    const size_t N = nodes3f(c->doms[id].p);
    double* outs[5] = {phi0, phi1, ux, uy, p};
    for (int k = 0; k < 5; ++k)
        if (outs[k]) HIP3F_OK(hipMemcpyAsync(outs[k], c->d_scratch + k * N, N * 8, hipMemcpyDeviceToHost, c->stream));
    HIP3F_OK(hipStreamSynchronize(c->stream));
    return TPF_OK;
}

extern "C" int tpf3f_read_mass(tpf3f_ctx* c, int32_t id, double mass[2]) {
    if (!c || !mass || id < 0 || id >= (int32_t)c->doms.size()) return TPF_EINVAL;
    if (!c->finalized) return TPF_ESTATE;
    if (c->precision == 32)
        hipLaunchKernelGGL(mass3f_partials<float>, dim3(kMassBlocks3F), dim3(256), 0, c->stream, c->d_doms, id,
                           c->d_part);
    else
        hipLaunchKernelGGL(mass3f_partials<double>, dim3(kMassBlocks3F), dim3(256), 0, c->stream, c->d_doms, id,
                           c->d_part);
    HIP3F_OK(hipGetLastError());
    hipLaunchKernelGGL(mass3f_final, dim3(1), dim3(64), 0, c->stream, c->d_part, kMassBlocks3F,
                       c->d_part + 2 * kMassBlocks3F);
    HIP3F_OK(hipGetLastError());
    HIP3F_OK(hipMemcpyAsync(mass, c->d_part + 2 * kMassBlocks3F, 16, hipMemcpyDeviceToHost, c->stream));
    HIP3F_OK(hipStreamSynchronize(c->stream));
    return TPF_OK;
}

extern "C" int tpf3f_get_populations(tpf3f_ctx* c, int32_t id, double* f0, double* f1, double* g) {
    if (!c || id < 0 || id >= (int32_t)c->doms.size()) return TPF_EINVAL;
    if (!c->finalized) return TPF_ESTATE;
    const size_t n = 9 * nodes3f(c->doms[id].p);
    if (c->precision == 32)
        hipLaunchKernelGGL(export3f_populations<float>, dim3(1024), dim3(256), 0, c->stream, c->d_doms, id,
                           c->d_scratch);
    else
        hipLaunchKernelGGL(export3f_populations<double>, dim3(1024), dim3(256), 0, c->stream, c->d_doms, id,
                           c->d_scratch);
    HIP3F_OK(hipGetLastError());
    double* outs[3] = {f0, f1, g};
    for (int k = 0; k < 3; ++k)
        if (outs[k]) HIP3F_OK(hipMemcpyAsync(outs[k], c->d_scratch + k * n, n * 8, hipMemcpyDeviceToHost, c->stream));
    HIP3F_OK(hipStreamSynchronize(c->stream));
    return TPF_OK;
}

extern "C" int tpf3f_bytes_per_node(tpf3f_ctx* c, int32_t id, double* bytes) {
    if (!c || !bytes || id < 0 || id >= (int32_t)c->doms.size()) return TPF_EINVAL;
    const double e = c->precision == 32 ? 4.0 : 8.0;
    // 27 population reads + 27 writes, lagged phi0 u, phi1 u (4) and B read and
    // written; with S also sym(Su) (3) and psi read and written
    double fields = 54 + 2 * 5;
    if (has_s3f(c->doms[id].p)) fields += 2 * 4;
    *bytes = fields * e;
    return TPF_OK;
}

extern "C" int tpf3f_kernel_timing(tpf3f_ctx* c, int32_t enable, double* avg_ms, int64_t* launches) {
    if (!c) return TPF_EINVAL;
    double acc = 0.0;
    int64_t n = 0;
    if (!c->ev.empty()) {
        HIP3F_OK(hipStreamSynchronize(c->stream));
        for (size_t k = 0; k < c->ev_steps.size(); ++k) {
            float ms = 0.f;
            HIP3F_OK(hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]));
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

extern "C" void tpf3f_destroy(tpf3f_ctx* c) {
    if (!c) return;
    for (auto e : c->ev) (void)hipEventDestroy(e);
    if (c->own_arena && c->arena) (void)hipFree(c->arena);
    delete c;
}
