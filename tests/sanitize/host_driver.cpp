// Host-sanitizer driver of the library's host code (test infrastructure):
// tpf_api.hip and tpf3_api.hip built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host side, run without a device through
// every call that needs none: parameter validation, the derived constants,
// the arena layout, the size classes, and finalize reporting the missing
// device.
#include <cmath>
#include <cstdio>
#include <vector>

#include "tpf.h"
#include "tpf3.h"

static int check(bool ok, const char* what) {
    if (!ok) std::printf("FAILED: %s\n", what);
    return ok ? 0 : 1;
}

int main() {
    int bad = 0;
    for (int prec : {32, 64}) {
        tpf_ctx* c = nullptr;
        bad |= check(tpf_create(&c, prec, nullptr) == TPF_OK && c, "tpf_create");
        std::vector<std::pair<int, int>> sizes = {{3, 3}, {67, 23}, {300, 200}};
        for (auto [nx, ny] : sizes) {
            tpf_domain_params p;
            tpf_default_params(&p, nx, ny);
            std::vector<double> phi0(nx * ny, 0.0), phi1(nx * ny, 0.3);
            int32_t id = -1;
            bad |= check(tpf_add_domain(c, &p, phi0.data(), phi1.data(), &id) == TPF_OK, "add");
            p.rho[2] = 0.1;  // S flux
            bad |= check(tpf_add_domain(c, &p, phi0.data(), phi1.data(), &id) == TPF_OK, "add S");
            p.theta = 4.0;  // outside (0, pi)
            bad |= check(tpf_add_domain(c, &p, phi0.data(), phi1.data(), &id) == TPF_EINVAL, "reject theta");
            p.theta = 1.0;
            p.tau_phi = 0.5;
            bad |= check(tpf_add_domain(c, &p, phi0.data(), phi1.data(), &id) == TPF_EINVAL, "reject tau");
        }
        int32_t n = 0;
        bad |= check(tpf_num_domains(c, &n) == TPF_OK && n == 6, "num domains");
        uint64_t bytes = 0;
        bad |= check(tpf_arena_bytes(c, &bytes) == TPF_OK && bytes > 0, "arena bytes");
        for (int i = 0; i < n; ++i) {
            double k, g[3], gT, eta, bpn;
            bad |= check(tpf_derived(c, i, &k, g, &gT, &eta) == TPF_OK && std::isfinite(eta), "derived");
            bad |= check(tpf_bytes_per_node(c, i, &bpn) == TPF_OK && bpn > 0, "bytes per node");
            int32_t nx, ny;
            bad |= check(tpf_domain_size(c, i, &nx, &ny) == TPF_OK, "domain size");
        }
        bad |= check(tpf_finalize(c, nullptr, 0) == TPF_EDEVICE, "finalize without device");
        tpf_destroy(c);
    }
    char buf[64];
    bad |= check(tpf_size_class(32, 300, 200, 0, buf, sizeof(buf)) == TPF_OK, "size class");
    bad |= check(tpf_size_class(32, 300, 200, 0, buf, 4) == TPF_EINVAL, "size class short buffer");
    int32_t ncodes = 0;
    int32_t codes[64], tx[64], ty[64];
    bad |= check(tpf_tile_codes(&ncodes, codes, tx, ty) == TPF_OK && ncodes > 0 && ncodes <= 64, "tile codes");
    for (int s = 0; s > -8; --s) bad |= check(tpf_strerror(s) != nullptr, "strerror");

    tpf3_ctx* c3 = nullptr;
    bad |= check(tpf3_create(&c3, 32, nullptr) == TPF_OK, "tpf3_create");
    tpf3_domain_params q;
    tpf3_default_params(&q, 17, 9, 11);
    std::vector<double> a(17 * 9 * 11, 0.0), b(17 * 9 * 11, 0.4);
    int32_t id = -1;
    bad |= check(tpf3_add_domain(c3, &q, a.data(), b.data(), &id) == TPF_OK, "tpf3 add");
    q.d0 = 1.5;
    bad |= check(tpf3_add_domain(c3, &q, a.data(), b.data(), &id) == TPF_EINVAL, "tpf3 reject d0");
    uint64_t bytes3 = 0;
    bad |= check(tpf3_arena_bytes(c3, &bytes3) == TPF_OK && bytes3 > 0, "tpf3 arena");
    bad |= check(tpf3_finalize(c3, nullptr, 0) == TPF_EDEVICE, "tpf3 finalize without device");
    tpf3_destroy(c3);
    std::printf("host sanitized run %s\n", bad ? "FAILED" : "ok");
    return bad;
}
