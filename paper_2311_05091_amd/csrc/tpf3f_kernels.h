// Kernels of the 3f model ("three fluids", arXiv 2311.05091 Sec. 2.1, 3, 4,
// 4.1) on the D2Q9 lattice: two CH lattices (phi0, phi1; phi2 = 1 - phi0 -
// phi1) and the NS lattice without solid terms.
//
// step3f_kernel: one wavefront per (domain, 64-column strip, CH-row chunk).
// Lane l owns column x0 + l; the wavefront marches rows y0 - 2 .. y0 + CH + 1.
// Iteration r
//   A. pulls both CH lattices of row y0 - 2 + r for its column (kept in a
//      three-deep register ring) and, on lanes 0..3, for the halo columns
//      x0 - 2, x0 - 1, x0 + 64, x0 + 65; writes phi0, phi1 into five-row LDS
//      rings;
//   B. computes mubar_0, mubar_1 (and stages psi = S_x u_y - S_y u_x) of the
//      row below on the columns x0 - 1 .. x0 + 64 (three-row rings);
//   C. updates the row two below: stencils, chemical potentials, S, forces,
//      u, p and the three Hermite-space collisions.
// Every population of an owned column is read once from memory.
#pragma once
#include "tpf_device.h"

namespace tpf3f {

using tpf::at_bytes;
using tpf::chem;
using tpf::fdiv;
using tpf::from_hermite;
using tpf::gp;
using tpf::gpc;
using tpf::gptr;
using tpf::kCx;
using tpf::kCy;
using tpf::kOpp;
using tpf::map_index;
using tpf::nat_moments;
using tpf::pull;
using tpf::to_hermite;
using tpf::xcd_tile;

enum { kMode3FStep = 0, kMode3FMoments = 1 };

template <typename T>
struct KConst3F {
    T c2, w0;
    T gam[3], inv_gam[3], gT3;   // spreading coefficients (Sec. 2.1), gamma^T/3
    T c12D, c3D4;                // 12/D, 3D/4
    T eta0, eta1;                // per CH lattice
    T Mcst, Mdeg, Mdeg_frac;
    T s0, s1, s2, s3, s4;        // CH rates (both lattices)
    T rho0, rho1, rho2, muv0, muv1, muv2;
    T drho0, drho1;              // rho0 - rho2, rho1 - rho2
    T Sfac0, Sfac1;              // (rho0 - rho2)/gamma0, (rho1 - rho2)/gamma1
    T sg0, sg1, sg3, sg4;        // NS rates (s2a, s2b per node)
    T inv_cfa, inv_cfb;          // 2/(1 - c_s^2), 1/c_s^2
    T Fbx, Fby, gauge;
    T pfac, pw, Kp, AH, BH;      // 2D pressure constants, H = Kp (AH - BH/s2a)
};

struct DomDev3F {
    int32_t nx, ny, px, py;
    int32_t parity, live, has_s, bh_zero;
    void* f0[2];     // [9][ny][nx] CH populations of phi0 (ping-pong)
    void* f1[2];     // [9][ny][nx] CH populations of phi1
    void* g[2];      // [9][ny][nx] NS populations
    void* lagA;      // [4][ny][nx] phi0 u, phi1 u of the previous step
    void* lagB;      // [ny][nx]    (rho u - S).u
    void* lagC;      // [3][ny][nx] sym(S u) (has_s)
    void* psi[2];    // [ny][nx]    S_x u_y - S_y u_x (has_s, ping-pong)
    KConst3F<double> kd;
    KConst3F<float> kf;
};

template <typename T>
__device__ __forceinline__ const KConst3F<T>& kconst3f(const DomDev3F& d);
template <>
__device__ __forceinline__ const KConst3F<double>& kconst3f<double>(const DomDev3F& d) { return d.kd; }
template <>
__device__ __forceinline__ const KConst3F<float>& kconst3f<float>(const DomDev3F& d) { return d.kf; }

// Isotropic 9-point gradient and Laplacian from three row arrays (below,
// centre, above) at column index i.
template <typename T>
__device__ __forceinline__ void st3(const T* lo, const T* mid, const T* hi, int i, T& gx, T& gy, T& lap) {
    const T C = mid[i], E = mid[i + 1], W = mid[i - 1], Nn = hi[i], S = lo[i];
    const T NE = hi[i + 1], NW = hi[i - 1], SE = lo[i + 1], SW = lo[i - 1];
    gx = (T(4) * (E - W) + (NE - NW + SE - SW)) * T(1.0 / 12.0);
    gy = (T(4) * (Nn - S) + (NE - SE + NW - SW)) * T(1.0 / 12.0);
    lap = (T(4) * (E + W + Nn + S) + (NE + NW + SE + SW) - T(20) * C) * T(1.0 / 6.0);
}

template <typename T>
__device__ __forceinline__ void gr3(const T* lo, const T* mid, const T* hi, int i, T& gx, T& gy) {
    const T E = mid[i + 1], W = mid[i - 1], Nn = hi[i], S = lo[i];
    const T NE = hi[i + 1], NW = hi[i - 1], SE = lo[i + 1], SW = lo[i - 1];
    gx = (T(4) * (E - W) + (NE - NW + SE - SW)) * T(1.0 / 12.0);
    gy = (T(4) * (Nn - S) + (NE - SE + NW - SW)) * T(1.0 / 12.0);
}

template <typename T>
__device__ __forceinline__ T lp3(const T* lo, const T* mid, const T* hi, int i) {
    return (T(4) * (mid[i + 1] + mid[i - 1] + hi[i] + lo[i]) + (hi[i + 1] + hi[i - 1] + lo[i + 1] + lo[i - 1]) -
            T(20) * mid[i]) * T(1.0 / 6.0);
}

// mu_p of the three phases (Sec. 2.1) and mubar_0, mubar_1 (Eq. eq-CHmodel):
// mubar_p = (gamma^T/3) sum_{q != p} (mu_p - mu_q)/gamma_q.
template <typename T>
__device__ __forceinline__ void chem3f(const KConst3F<T>& K, T ph0, T ph1, T lap0, T lap1, T& mu0, T& mu1, T& mu2,
                                       T& mb0, T& mb1) {
    mu0 = chem(K.gam[0], K.c12D, K.c3D4, ph0, lap0);
    mu1 = chem(K.gam[1], K.c12D, K.c3D4, ph1, lap1);
    mu2 = chem(K.gam[2], K.c12D, K.c3D4, T(1) - ph0 - ph1, -lap0 - lap1);
    mb0 = K.gT3 * ((mu0 - mu1) * K.inv_gam[1] + (mu0 - mu2) * K.inv_gam[2]);
    mb1 = K.gT3 * ((mu1 - mu0) * K.inv_gam[0] + (mu1 - mu2) * K.inv_gam[2]);
}

// CH collision of one lattice in Hermite space (Sec. 3, 4): phase field ph,
// eta mubar, velocity u, d_t(ph u) by explicit Euler, a eta grad(mubar).
template <typename T>
__device__ __forceinline__ void ch_collide(const KConst3F<T>& K, const T* fp, T ph, T emu, T ux, T uy, T lAx, T lAy,
                                           T aeg_x, T aeg_y, T (&fo)[9]) {
    const T c2 = K.c2;
    T m[9], h[9];
    nat_moments(fp, m);
    to_hermite(m, h, c2);
    const T Ax = ph * ux, Ay = ph * uy;
    const T Wx = (Ax - lAx) + c2 * aeg_x, Wy = (Ay - lAy) + c2 * aeg_y;
    const T e3 = c2 * (emu - ph);
    h[0] = h[0] - K.s0 * (h[0] - ph);
    h[1] = h[1] - K.s1 * (h[1] - Ax) + (T(1) - T(0.5) * K.s1) * Wx;
    h[2] = h[2] - K.s1 * (h[2] - Ay) + (T(1) - T(0.5) * K.s1) * Wy;
    h[3] = h[3] - K.s2 * (h[3] - e3);
    h[4] = h[4] - K.s2 * (h[4] - e3);
    h[5] = h[5] - K.s2 * h[5];
    h[6] = h[6] - K.s3 * h[6];
    h[7] = h[7] - K.s3 * h[7];
    h[8] = h[8] - K.s4 * (h[8] - c2 * c2 * (ph - emu));
    from_hermite(h, fo, c2);
}

// Lagged fields of one node, read before its update.
template <typename T>
struct Lag3F {
    T A0x, A0y, A1x, A1y, B, Cxx, Cyy, Cxy;
};

template <typename T, int MODE>
__device__ __forceinline__ void node_update3f(const DomDev3F& d, const KConst3F<T>& K, bool dS, int id, int N, T ph0,
                                              T ph1, T gx0, T gy0, T lap0, T gx1, T gy1, T lap1, T mb0, T mb1,
                                              T gm0x, T gm0y, T gm1x, T gm1y, T dpx, T dpy, const T* f0p,
                                              const T* f1p, const T (&gq)[9], const Lag3F<T>& L, int cur,
                                              double* __restrict__ mom_out) {
    const T c2 = K.c2;
    T mu0, mu1, mu2, mbu0, mbu1;
    chem3f<T>(K, ph0, ph1, lap0, lap1, mu0, mu1, mu2, mbu0, mbu1);
    (void)mbu0;
    (void)mbu1;
    const T ph2 = T(1) - ph0 - ph1;
    // degenerate mobility of the 3f model (Sec. 4)
    const T fdeg = (T(1) - ph0) * (T(1) - ph1) * (T(1) - ph2);
    const T a = K.Mdeg_frac * (T(1) - fdeg);
    const T rho = K.rho0 * ph0 + K.rho1 * ph1 + K.rho2 * ph2;
    const T muv = K.muv0 * ph0 + K.muv1 * ph1 + K.muv2 * ph2;
    const T drx = K.drho0 * gx0 + K.drho1 * gx1;
    const T dry = K.drho0 * gy0 + K.drho1 * gy1;
    T Fx = mu0 * gx0 + mu1 * gx1 - mu2 * (gx0 + gx1);
    T Fy = mu0 * gy0 + mu1 * gy1 - mu2 * (gy0 + gy1);
    T Sx = T(0), Sy = T(0);
    if (dS) {
        // S = sum_p rho_p M grad(mubar_p)/gamma_p over the three phases
        const T Mob = K.Mcst + K.Mdeg * fdeg;
        Sx = Mob * (K.Sfac0 * gm0x + K.Sfac1 * gm1x);
        Sy = Mob * (K.Sfac0 * gm0y + K.Sfac1 * gm1y);
        Fx += T(-0.5) * dpy;
        Fy += T(0.5) * dpx;
    }
    Fx += K.Fbx;
    Fy += K.Fby;
    T mg[9];
    nat_moments(gq, mg);
    const T inv_rho = fdiv(T(1), rho);
    // no solid: u = u*, effective viscosity mu
    const T ux = (mg[1] + T(0.5) * Fx) * inv_rho;
    const T uy = (mg[2] + T(0.5) * Fy) * inv_rho;
    const T s2a = fdiv(T(1), muv * inv_rho * K.inv_cfa + T(0.5));
    const T s2b = fdiv(T(1), muv * inv_rho * K.inv_cfb + T(0.5));
    const T Q = ux * drx + uy * dry;
    const T Bn = (rho * ux - Sx) * ux + (rho * uy - Sy) * uy;
    const T H = K.Kp * (K.AH - (d.bh_zero ? T(0) : fdiv(K.BH, s2a)));
    const T p = K.pfac * ((mg[0] - gq[0]) + (T(0.5) + H) * Q - K.pw * Bn + T(0.5) * K.Kp * (Bn - L.B));

    if constexpr (MODE == kMode3FMoments) {
        mom_out[id] = double(ph0);
        mom_out[N + id] = double(ph1);
        mom_out[2 * N + id] = double(ux);
        mom_out[3 * N + id] = double(uy);
        mom_out[4 * N + id] = double(p);
        return;
    }
    // ---- the two CH collisions ----
    {
        T fo[9];
        ch_collide<T>(K, f0p, ph0, K.eta0 * mb0, ux, uy, L.A0x, L.A0y, a * K.eta0 * gm0x, a * K.eta0 * gm0y, fo);
        gptr<T> o = gp<T>(d.f0[cur ^ 1]);
#pragma unroll
        for (int q = 0; q < 9; ++q) __builtin_nontemporal_store(fo[q], o + (q * N + id));
        ch_collide<T>(K, f1p, ph1, K.eta1 * mb1, ux, uy, L.A1x, L.A1y, a * K.eta1 * gm1x, a * K.eta1 * gm1y, fo);
        o = gp<T>(d.f1[cur ^ 1]);
#pragma unroll
        for (int q = 0; q < 9; ++q) __builtin_nontemporal_store(fo[q], o + (q * N + id));
        gptr<T> lA = gp<T>(d.lagA);
        lA[id] = ph0 * ux;
        lA[N + id] = ph0 * uy;
        lA[2 * N + id] = ph1 * ux;
        lA[3 * N + id] = ph1 * uy;
    }
    // ---- NS collision (G = F: no fluid-structure force) ----
    {
        const T Jx = rho * ux, Jy = rho * uy;
        const T Pxx = rho * ux * ux - Sx * ux;
        const T Pyy = rho * uy * uy - Sy * uy;
        const T Pxy = rho * ux * uy - T(0.5) * (Sx * uy + ux * Sy);
        T Cxx = T(0), Cyy = T(0), Cxy = T(0), dCxx = T(0), dCyy = T(0), dCxy = T(0);
        if (dS) {
            Cxx = Sx * ux;
            Cyy = Sy * uy;
            Cxy = T(0.5) * (Sx * uy + Sy * ux);
            dCxx = Cxx - L.Cxx;
            dCyy = Cyy - L.Cyy;
            dCxy = Cxy - L.Cxy;
        }
        const T q3 = (T(1) - T(3) * c2) * Q;
        const T Mxx = T(2) * ux * Fx - dCxx + T(2) * c2 * ux * drx + q3;
        const T Myy = T(2) * uy * Fy - dCyy + T(2) * c2 * uy * dry + q3;
        const T Mxy = ux * Fy + Fx * uy - dCxy + c2 * (ux * dry + drx * uy);
        T h[9];
        to_hermite(mg, h, c2);
        const T gauge = K.gauge;
        h[0] = h[0] - K.sg0 * (h[0] - gauge) + (T(1) - T(0.5) * K.sg0) * Q;
        h[1] = h[1] - K.sg1 * (h[1] - Jx) + (T(1) - T(0.5) * K.sg1) * Fx;
        h[2] = h[2] - K.sg1 * (h[2] - Jy) + (T(1) - T(0.5) * K.sg1) * Fy;
        h[3] = h[3] - s2a * (h[3] - (p + Pxx - c2 * gauge)) + (T(1) - T(0.5) * s2a) * Mxx;
        h[4] = h[4] - s2a * (h[4] - (p + Pyy - c2 * gauge)) + (T(1) - T(0.5) * s2a) * Myy;
        h[5] = h[5] - s2b * (h[5] - Pxy) + (T(1) - T(0.5) * s2b) * Mxy;
        h[6] = h[6] - K.sg3 * h[6];
        h[7] = h[7] - K.sg3 * h[7];
        h[8] = h[8] - K.sg4 * (h[8] - (c2 * c2 * gauge - c2 * p));
        T go[9];
        from_hermite(h, go, c2);
        gptr<T> o = gp<T>(d.g[cur ^ 1]);
#pragma unroll
        for (int q = 0; q < 9; ++q) __builtin_nontemporal_store(go[q], o + (q * N + id));
        gp<T>(d.lagB)[id] = Bn;
        if (dS) {
            gptr<T> lC = gp<T>(d.lagC);
            lC[id] = Cxx;
            lC[N + id] = Cyy;
            lC[2 * N + id] = Cxy;
            gp<T>(d.psi[cur ^ 1])[id] = Sx * uy - Sy * ux;
        }
    }
}

template <typename T, bool HAS_S>
struct Ring3F {
    static constexpr int WX = 68, VX = 66;
    T phi0[5][WX];
    T phi1[5][WX];
    T mb0[3][VX];
    T mb1[3][VX];
    T psi[HAS_S ? 3 : 1][HAS_S ? VX : 1];
};

// Both CH lattices pulled at node (x, y) into p[0..8] (phi0) and p[9..17].
template <typename T>
__device__ __forceinline__ void pull18(const DomDev3F& d, int cur, int x, int y, T* p) {
    const int nx = d.nx, ny = d.ny, N = nx * ny;
    gptr<const T> a = gpc<T>(d.f0[cur]);
    gptr<const T> b = gpc<T>(d.f1[cur]);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        p[q] = pull<T>(a, q, x, y, nx, ny, d.px, d.py, N, nx);
        p[9 + q] = pull<T>(b, q, x, y, nx, ny, d.px, d.py, N, nx);
    }
}

template <typename T, bool HAS_S, int MODE>
__device__ __forceinline__ void iter3f(const DomDev3F& d, const KConst3F<T>& K, Ring3F<T, HAS_S>& sh, int r,
                                       int x0, int y0, int lane, int cur, bool dS, T (&FL)[18], const T (&FU)[18],
                                       double* __restrict__ mom_out) {
    constexpr int WX = Ring3F<T, HAS_S>::WX, VX = Ring3F<T, HAS_S>::VX;
    const int nx = d.nx, ny = d.ny, N = nx * ny;
    const int yr = y0 - 2 + r;
    const int sy = map_index(yr, ny, d.py);
    const int s5 = r % 5;
    // ---- A. pull both CH lattices of row yr ----
    // (at the highest wavefront priority, so that a memory-bound wavefront
    // gets its loads out before the others' arithmetic)
    __builtin_amdgcn_s_setprio(3);
    {
        const int sx = map_index(x0 + lane, nx, d.px);
        pull18<T>(d, cur, sx, sy, FL);
        T a = FL[0], b = FL[9];
#pragma unroll
        for (int q = 1; q < 9; ++q) {
            a += FL[q];
            b += FL[9 + q];
        }
        sh.phi0[s5][lane + 2] = a;
        sh.phi1[s5][lane + 2] = b;
    }
    if (lane < 4) {
        const int cell = lane < 2 ? lane : 64 + lane;
        const int hx = map_index(x0 - 2 + cell, nx, d.px);
        T hp[18];
        pull18<T>(d, cur, hx, sy, hp);
        T a = hp[0], b = hp[9];
#pragma unroll
        for (int q = 1; q < 9; ++q) {
            a += hp[q];
            b += hp[9 + q];
        }
        sh.phi0[s5][cell] = a;
        sh.phi1[s5][cell] = b;
    }
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();
    // ---- B. mubar_0, mubar_1 (and psi) of row yr - 1 on columns x0 - 1 .. x0 + 64 ----
    const int s3 = r % 3;
    if (r >= 2) {
        const T* pl = sh.phi0[(r + 3) % 5];
        const T* pm = sh.phi0[(r + 4) % 5];
        const T* ph = sh.phi0[s5];
        const T* ql = sh.phi1[(r + 3) % 5];
        const T* qm = sh.phi1[(r + 4) % 5];
        const T* qh = sh.phi1[s5];
        const int yb = map_index(yr - 1, ny, d.py);
        for (int c = lane; c < VX; c += 64) {
            const int i = c + 1;
            T mu0, mu1, mu2, m0, m1;
            chem3f<T>(K, pm[i], qm[i], lp3(pl, pm, ph, i), lp3(ql, qm, qh, i), mu0, mu1, mu2, m0, m1);
            sh.mb0[s3][c] = m0;
            sh.mb1[s3][c] = m1;
            if constexpr (HAS_S) {
                if (dS) sh.psi[s3][c] = gpc<T>(d.psi[cur])[yb * nx + map_index(x0 - 1 + c, nx, d.px)];
            }
        }
    }
    __syncthreads();
    // ---- C. update row yu = yr - 2 ----
    const int yu = yr - 2;
    const int x = x0 + lane;
    if (r >= 4 && yu < ny && x < nx) {
        const int i = lane + 2, j = lane + 1;
        const int id = yu * nx + x;
        T gx0, gy0, lap0, gx1, gy1, lap1, gm0x, gm0y, gm1x, gm1y;
        st3(sh.phi0[(r + 2) % 5], sh.phi0[(r + 3) % 5], sh.phi0[(r + 4) % 5], i, gx0, gy0, lap0);
        st3(sh.phi1[(r + 2) % 5], sh.phi1[(r + 3) % 5], sh.phi1[(r + 4) % 5], i, gx1, gy1, lap1);
        gr3(sh.mb0[(r + 1) % 3], sh.mb0[(r + 2) % 3], sh.mb0[s3], j, gm0x, gm0y);
        gr3(sh.mb1[(r + 1) % 3], sh.mb1[(r + 2) % 3], sh.mb1[s3], j, gm1x, gm1y);
        T dpx = T(0), dpy = T(0);
        if constexpr (HAS_S) {
            if (dS) gr3(sh.psi[(r + 1) % 3], sh.psi[(r + 2) % 3], sh.psi[s3], j, dpx, dpy);
        }
        T gq[9];
        gptr<const T> gin = gpc<T>(d.g[cur]);
#pragma unroll
        for (int q = 0; q < 9; ++q) gq[q] = pull<T>(gin, q, x, yu, nx, ny, d.px, d.py, N, nx);
        Lag3F<T> L;
        gptr<const T> lA = gpc<T>(d.lagA);
        L.A0x = lA[id];
        L.A0y = lA[N + id];
        L.A1x = lA[2 * N + id];
        L.A1y = lA[3 * N + id];
        L.B = gpc<T>(d.lagB)[id];
        L.Cxx = L.Cyy = L.Cxy = T(0);
        if (dS) {
            gptr<const T> lC = gpc<T>(d.lagC);
            L.Cxx = lC[id];
            L.Cyy = lC[N + id];
            L.Cxy = lC[2 * N + id];
        }
        node_update3f<T, MODE>(d, K, dS, id, N, sh.phi0[(r + 3) % 5][i], sh.phi1[(r + 3) % 5][i], gx0, gy0, lap0,
                               gx1, gy1, lap1, sh.mb0[(r + 2) % 3][j], sh.mb1[(r + 2) % 3][j], gm0x, gm0y, gm1x,
                               gm1y, dpx, dpy, FU, FU + 9, gq, L, cur, mom_out);
    }
}

template <typename T, int CH, bool HAS_S, int MODE>
__global__ void __launch_bounds__(64)
step3f_kernel(const DomDev3F* __restrict__ doms, const int4* __restrict__ tiles, int ntiles, int step_offset,
              double* __restrict__ mom_out) {
    __shared__ Ring3F<T, HAS_S> sh;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    if (t >= ntiles) return;
    const int4 tile = tiles[t];
    const DomDev3F& d = doms[tile.x];
    if (!d.live && MODE == kMode3FStep) return;
    const KConst3F<T> K = kconst3f<T>(d);
    const int cur = (d.parity + step_offset) & 1;
    const bool dS = HAS_S && d.has_s;
    const int lane = threadIdx.x;
    const int x0 = tile.y, y0 = tile.z;
    T F0[18], F1[18], F2[18];
    constexpr int R = CH + 4;
    for (int r = 0; r < R; r += 3) {
        iter3f<T, HAS_S, MODE>(d, K, sh, r, x0, y0, lane, cur, dS, F0, F1, mom_out);
        if (r + 1 < R) iter3f<T, HAS_S, MODE>(d, K, sh, r + 1, x0, y0, lane, cur, dS, F1, F2, mom_out);
        if (r + 2 < R) iter3f<T, HAS_S, MODE>(d, K, sh, r + 2, x0, y0, lane, cur, dS, F2, F0, mom_out);
    }
}

// Initial state: f_p = f^eq(phi_p, eta_p mubar_p, u = 0) for p = 0, 1, g =
// g^eq(P = 0, u = 0) = gauge delta_q0, lagged fields zero.  phi_in: float64
// [2][ny][nx] (phi0, phi1).
template <typename T>
__global__ void init3f_kernel(const DomDev3F* __restrict__ doms, int dom, const double* __restrict__ phi_in) {
    const DomDev3F& d = doms[dom];
    const int nx = d.nx, ny = d.ny, N = nx * ny;
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= N) return;
    const int x = id % nx, y = id / nx;
    T v0[9], v1[9];
    int k = 0;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx, ++k) {
            const int sx = map_index(x + dx, nx, d.px), sy = map_index(y + dy, ny, d.py);
            v0[k] = T(phi_in[sy * nx + sx]);
            v1[k] = T(phi_in[N + sy * nx + sx]);
        }
    const KConst3F<T> K = kconst3f<T>(d);
    T mu0, mu1, mu2, mb0, mb1;
    chem3f<T>(K, v0[4], v1[4], tpf::lap9(v0, 4, 3), tpf::lap9(v1, 4, 3), mu0, mu1, mu2, mb0, mb1);
    const T c2 = K.c2, w0 = K.w0;
    const T w1 = (c2 - c2 * c2) * T(0.5), w5 = c2 * c2 * T(0.25);
    const int par = d.parity;
    const T emu[2] = {K.eta0 * mb0, K.eta1 * mb1};
    const T ph[2] = {v0[4], v1[4]};
    for (int p = 0; p < 2; ++p) {
        gptr<T> f = gp<T>(p == 0 ? d.f0[par] : d.f1[par]);
        f[id] = ph[p] + (w0 - T(1)) * emu[p];
        for (int q = 1; q <= 4; ++q) f[q * N + id] = w1 * emu[p];
        for (int q = 5; q <= 8; ++q) f[q * N + id] = w5 * emu[p];
    }
    gptr<T> g = gp<T>(d.g[par]);
    g[id] = K.gauge;
    for (int q = 1; q < 9; ++q) g[q * N + id] = T(0);
    gptr<T> A = gp<T>(d.lagA);
    for (int q = 0; q < 4; ++q) A[q * N + id] = T(0);
    gp<T>(d.lagB)[id] = T(0);
    if (d.has_s) {
        gptr<T> Cl = gp<T>(d.lagC);
        Cl[id] = T(0);
        Cl[N + id] = T(0);
        Cl[2 * N + id] = T(0);
        gp<T>(d.psi[0])[id] = T(0);
        gp<T>(d.psi[1])[id] = T(0);
    }
}

// Phase masses: per-block compensated FP64 sums of the post-collision
// populations of both CH lattices, then a fixed-order final sum.
template <typename T>
__global__ void __launch_bounds__(256) mass3f_partials(const DomDev3F* __restrict__ doms, int dom,
                                                      double* __restrict__ part) {
    const DomDev3F& d = doms[dom];
    const int64_t n = (int64_t)9 * d.nx * d.ny;
    __shared__ double red[2][256];
    for (int p = 0; p < 2; ++p) {
        gptr<const T> f = gpc<T>(p == 0 ? d.f0[d.parity] : d.f1[d.parity]);
        double s = 0.0, c = 0.0;
        for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) {
            const double y = double(f[k]) - c;
            const double t = s + y;
            c = (t - s) - y;
            s = t;
        }
        red[p][threadIdx.x] = s;
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = red[0][0];
        part[gridDim.x + blockIdx.x] = red[1][0];
    }
}

__global__ void mass3f_final(const double* __restrict__ part, int nblk, double* __restrict__ out) {
    if (threadIdx.x < 2) {
        double s = 0.0, c = 0.0;
        for (int b = 0; b < nblk; ++b) {
            const double y = part[threadIdx.x * nblk + b] - c;
            const double t = s + y;
            c = (t - s) - y;
            s = t;
        }
        out[threadIdx.x] = s;
    }
}

// Populations of the current state as float64: [f0; f1; g], 9 N each.
template <typename T>
__global__ void export3f_populations(const DomDev3F* __restrict__ doms, int dom, double* __restrict__ out) {
    const DomDev3F& d = doms[dom];
    const int64_t n = (int64_t)9 * d.nx * d.ny;
    gptr<const T> a = gpc<T>(d.f0[d.parity]);
    gptr<const T> b = gpc<T>(d.f1[d.parity]);
    gptr<const T> g = gpc<T>(d.g[d.parity]);
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        out[k] = double(a[k]);
        out[n + k] = double(b[k]);
        out[2 * n + k] = double(g[k]);
    }
}

}  // namespace tpf3f
