// Kernels of the coupled ternary phase-field LB step (arXiv 2311.05091, 2f1s
// model, D2Q9, Hermite-moment collision).
//
// step_kernel: one workgroup per (domain, TX x TY tile).  In one pass it
//   1. pulls the CH populations over the tile plus a 2-node halo and sums
//      them into phi1 (LDS), next to phi0 (LDS);
//   2. computes mubar1 on the tile plus a 1-node halo (LDS) and, when the
//      flux S is active, stages the previous psi (LDS);
//   3. per interior node: pulls f and g, forms grad/lap of phi0, phi1,
//      grad(mubar1), the forces, u, p, relaxes both lattices in Hermite-moment
//      space and writes the post-collision populations and lagged fields.
// All global accesses are SoA rows with x fastest, so a wavefront of 64 lanes
// touches 64 consecutive nodes.
#pragma once
#include <type_traits>

#include "tpf_device.h"

namespace tpf {

enum StepMode { kModeStep = 0, kModeMoments = 1 };

// Per-node part of the step, shared by the tile and strip kernels: given the
// stencil values of phi0, phi1, mubar1 (and psi), the pulled populations and
// the lagged fields of the node, forms the forces, u, p and writes either the
// post-collision populations and lagged fields or the moments.  The node's
// element index is row + cb / sizeof(T): a uniform part and a per-lane byte
// offset, so stores use scalar-base addressing.
template <typename T, int MODE>
__device__ __forceinline__ void node_update(const DomDev& d, const KConst<T>& K, bool dS, int64_t row, uint32_t cb,
                                            int N, int x, int y, T ph0, T ph1,
                                            T gx0, T gy0, T lap0, T gx1, T gy1, T lap1, T mub,
                                            T gmx, T gmy, T dpsix, T dpsiy, T (&fp)[9], T (&gq)[9],
                                            T lAx, T lAy, T lB, T lCxx, T lCyy, T lCxy, int cur,
                                            double* __restrict__ mom_out) {
    const T c2 = K.c2;
    T mu0, mu1, mu2;
    (void)mubar1<T>(K, ph0, ph1, lap0, lap1, mu0, mu1, mu2);

    // degenerate mobility, 2f1s form f = phi1 (1 - phi1)(1 - phi0) (Sec. 4)
    const T fdeg = ph1 * (T(1) - ph1) * (T(1) - ph0);
    const T a = K.Mdeg_frac * (T(1) - fdeg);

    // density, viscosity (linear in phi_p), grad(rho)
    const T ph2 = T(1) - ph0 - ph1;
    const T rho = K.rho0 * ph0 + K.rho1 * ph1 + K.rho2 * ph2;
    const T muv = K.muv0 * ph0 + K.muv1 * ph1 + K.muv2 * ph2;
    const T drx = K.drho0 * gx0 + K.drho1 * gx1;
    const T dry = K.drho0 * gy0 + K.drho1 * gy1;

    // surface tension F_s = sum_p mu_p grad(phi_p)
    T Fx = mu0 * gx0 + mu1 * gx1 + mu2 * (-gx0 - gx1);
    T Fy = mu0 * gy0 + mu1 * gy1 + mu2 * (-gy0 - gy1);
    T Sx = T(0), Sy = T(0);
    if (dS) {
        // S = (rho1 - rho2) M grad(mubar1)/gamma1; F_c from the previous psi
        const T Mob = K.Mcst + K.Mdeg * fdeg;
        Sx = K.Sfac * Mob * gmx;
        Sy = K.Sfac * Mob * gmy;
        Fx += T(-0.5) * dpsiy;
        Fy += T(0.5) * dpsix;
    }
    Fx += K.Fbx;
    Fy += K.Fby;

    // NS moments; velocity with the solid correction (Sec. 3)
    T mg[9];
    nat_moments(gq, mg);
    const T inv_rho = fdiv(T(1), rho);
    const T usx = (mg[1] + T(0.5) * Fx) * inv_rho;
    const T usy = (mg[2] + T(0.5) * Fy) * inv_rho;
    // rigid-body velocity of the solid point: translation plus rotation
    const T uwx = K.uwx - K.om * (T(y) - K.yc);
    const T uwy = K.uwy + K.om * (T(x) - K.xc);
    const T fsx = uwx - usx, fsy = uwy - usy;
    const T ux = usx + T(0.5) * ph0 * fsx;
    const T uy = usy + T(0.5) * ph0 * fsy;

    // per-node NS rates from mu/(rho (1 - phi0)) (Sec. 3)
    const T om = T(1) - ph0;
    const T s2a = fdiv(om, muv * inv_rho * K.inv_cfa + T(0.5) * om);
    const T s2b = fdiv(om, muv * inv_rho * K.inv_cfb + T(0.5) * om);

    // pressure (Sec. 3, 2D constants)
    const T Q = ux * drx + uy * dry;
    const T Bn = (rho * ux - Sx) * ux + (rho * uy - Sy) * uy;
    // the s2a term of H is zero where its coefficient is and at a saturated
    // solid node (phi0 = 1 in the working precision, s2a = 0)
    const T H = K.Kp * (K.AH - ((d.bh_zero || s2a == T(0)) ? T(0) : fdiv(K.BH, s2a)));
    const T p = K.pfac * ((mg[0] - gq[0]) + (T(0.5) + H) * Q - K.pw * Bn +
                             T(0.5) * K.Kp * (Bn - lB));

    if constexpr (MODE == kModeMoments) {
        // the moments in the caller's layout: [4][ny][nx], no row padding
        const int64_t id = (int64_t)y * d.nx + x, Nl = (int64_t)d.nx * d.ny;
        mom_out[id] = double(ph1);
        mom_out[Nl + id] = double(ux);
        mom_out[2 * Nl + id] = double(uy);
        mom_out[3 * Nl + id] = double(p);
        return;
    }
    // open ends: the inner neighbours of the inlet and outlet keep their
    // fields of this step for the non-equilibrium extrapolation
    if (d.open_x && (x == 1 || x == d.nx - 2)) {
        gptr<T> bnd = gp<T>(d.bnd) + (x == 1 ? 0 : kBndFields) * d.ny + y;
        bnd[kBndPhi1 * d.ny] = ph1;
        bnd[kBndMub * d.ny] = mub;
        bnd[kBndUx * d.ny] = ux;
        bnd[kBndUy * d.ny] = uy;
        bnd[kBndP * d.ny] = p;
        bnd[kBndSx * d.ny] = Sx;
        bnd[kBndSy * d.ny] = Sy;
    }
    gptr<T> fout = gp<T>(d.f[cur ^ 1]);
    gptr<T> gout = gp<T>(d.g[cur ^ 1]);

    // ---- CH collision in Hermite space ----
    {
        T m[9], h[9];
        nat_moments(fp, m);
        to_hermite(m, h, c2);
        const T Ax = ph1 * ux, Ay = ph1 * uy;
        const T emu = K.eta * mub;
        // d_t(phi u) by explicit Euler, plus the degenerate-mobility correction
        const T Wx = (Ax - lAx) + a * K.eta * c2 * gmx;
        const T Wy = (Ay - lAy) + a * K.eta * c2 * gmy;
        const T s0 = K.s0, s1 = K.s1, s2 = K.s2, s3 = K.s3, s4 = K.s4;
        const T e3 = c2 * (emu - ph1);
        h[0] = h[0] - s0 * (h[0] - ph1);
        h[1] = h[1] - s1 * (h[1] - Ax) + (T(1) - T(0.5) * s1) * Wx;
        h[2] = h[2] - s1 * (h[2] - Ay) + (T(1) - T(0.5) * s1) * Wy;
        h[3] = h[3] - s2 * (h[3] - e3);
        h[4] = h[4] - s2 * (h[4] - e3);
        h[5] = h[5] - s2 * h[5];
        h[6] = h[6] - s3 * h[6];
        h[7] = h[7] - s3 * h[7];
        h[8] = h[8] - s4 * (h[8] - c2 * c2 * (ph1 - emu));
        T fo[9];
        from_hermite(h, fo, c2);
#pragma unroll
        for (int q = 0; q < 9; ++q) __builtin_nontemporal_store(fo[q], at_bytes(fout + ((int64_t)q * N + row), cb));
        gptr<T> lagA = gp<T>(d.lagA);
        *at_bytes(lagA + row, cb) = Ax;
        *at_bytes(lagA + (N + row), cb) = Ay;
    }

    // ---- NS collision in Hermite space ----
    {
        const T Gx = Fx + ph0 * rho * fsx, Gy = Fy + ph0 * rho * fsy;
        const T Jx = rho * ux, Jy = rho * uy;
        const T Pxx = rho * ux * ux - Sx * ux;
        const T Pyy = rho * uy * uy - Sy * uy;
        const T Pxy = rho * ux * uy - T(0.5) * (Sx * uy + ux * Sy);
        // M2F = uF + Fu - d_t((Su + uS)/2) + c_s^2 (u grad rho + grad rho u)
        //       + (1 - 3 c_s^2)(u . grad rho) I
        T Cxx = T(0), Cyy = T(0), Cxy = T(0), dCxx = T(0), dCyy = T(0), dCxy = T(0);
        if (dS) {
            Cxx = Sx * ux;
            Cyy = Sy * uy;
            Cxy = T(0.5) * (Sx * uy + Sy * ux);
            dCxx = Cxx - lCxx;
            dCyy = Cyy - lCyy;
            dCxy = Cxy - lCxy;
        }
        const T q3 = (T(1) - T(3) * c2) * Q;
        const T Mxx = T(2) * ux * Fx - dCxx + T(2) * c2 * ux * drx + q3;
        const T Myy = T(2) * uy * Fy - dCyy + T(2) * c2 * uy * dry + q3;
        const T Mxy = ux * Fy + Fx * uy - dCxy + c2 * (ux * dry + drx * uy);
        T h[9];
        to_hermite(mg, h, c2);
        const T gauge = K.gauge;
        const T sg0 = K.sg0, sg1 = K.sg1, sg3 = K.sg3, sg4 = K.sg4;
        h[0] = h[0] - sg0 * (h[0] - gauge) + (T(1) - T(0.5) * sg0) * Q;
        h[1] = h[1] - sg1 * (h[1] - Jx) + (T(1) - T(0.5) * sg1) * Gx;
        h[2] = h[2] - sg1 * (h[2] - Jy) + (T(1) - T(0.5) * sg1) * Gy;
        h[3] = h[3] - s2a * (h[3] - (p + Pxx - c2 * gauge)) + (T(1) - T(0.5) * s2a) * Mxx;
        h[4] = h[4] - s2a * (h[4] - (p + Pyy - c2 * gauge)) + (T(1) - T(0.5) * s2a) * Myy;
        h[5] = h[5] - s2b * (h[5] - Pxy) + (T(1) - T(0.5) * s2b) * Mxy;
        h[6] = h[6] - sg3 * h[6];
        h[7] = h[7] - sg3 * h[7];
        h[8] = h[8] - sg4 * (h[8] - (c2 * c2 * gauge - c2 * p));
        T go[9];
        from_hermite(h, go, c2);
#pragma unroll
        for (int q = 0; q < 9; ++q) __builtin_nontemporal_store(go[q], at_bytes(gout + ((int64_t)q * N + row), cb));
        *at_bytes(gp<T>(d.lagB) + row, cb) = Bn;
        if (dS) {
            gptr<T> lagC = gp<T>(d.lagC);
            *at_bytes(lagC + row, cb) = Cxx;
            *at_bytes(lagC + (N + row), cb) = Cyy;
            *at_bytes(lagC + (2 * (int64_t)N + row), cb) = Cxy;
            *at_bytes(gp<T>(d.psi[cur ^ 1]) + row, cb) = Sx * uy - Sy * ux;
        }
    }
}

// Pulled populations of both lattices at node (x, y).
template <typename T>
__device__ __forceinline__ void pull9(gptr<const T> fin, int x, int y, int nx, int ny, int px,
                                      int py, int N, int ld, T (&out)[9]) {
#pragma unroll
    for (int q = 0; q < 9; ++q) out[q] = pull(fin, q, x, y, nx, ny, px, py, N, ld);
}

template <typename T, int TX, int TY, int NT, bool HAS_S, int MODE>
__global__ void __launch_bounds__(NT)
step_kernel(const DomDev* __restrict__ doms, const int4* __restrict__ tiles, int ntiles,
            int step_offset, double* __restrict__ mom_out) {
    constexpr int WX = TX + 4, WY = TY + 4;  // halo-2 window
    constexpr int VX = TX + 2, VY = TY + 2;  // halo-1 window
    __shared__ T s_phi0[WX * WY];
    __shared__ T s_phi1[WX * WY];
    __shared__ T s_mub[VX * VY];
    __shared__ T s_psi[HAS_S ? VX * VY : 1];

    const int t = xcd_tile(blockIdx.x, gridDim.x);
    if (t >= ntiles) return;
    const int4 tile = tiles[t];
    const DomDev& d = doms[tile.x];
    if (!d.live && MODE == kModeStep) return;
    const KConst<T> K = kconst<T>(d);
    const int nx = d.nx, ny = d.ny, px = d.px, py = d.py;
    const int ld = d.pitch, N = ld * ny;
    const int x0 = tile.y, y0 = tile.z;
    const int cur = (d.parity + step_offset) & 1;
    gptr<const T> fin = gpc<T>(d.f[cur]);
    gptr<const T> gin = gpc<T>(d.g[cur]);
    gptr<const T> phi0 = gpc<T>(d.phi0);
    const int tid = threadIdx.x;

    // ---- 1. phi0 and phi1 = sum_q f_q on the halo-2 window ----
    for (int k = tid; k < WX * WY; k += NT) {
        const int wx = k % WX, wy = k / WX;
        const int sx = map_index(x0 - 2 + wx, nx, px);
        const int sy = map_index(y0 - 2 + wy, ny, py);
        s_phi0[k] = phi0[sy * ld + sx];
        T s = pull(fin, 0, sx, sy, nx, ny, px, py, N, ld);
#pragma unroll
        for (int q = 1; q < 9; ++q) s += pull(fin, q, sx, sy, nx, ny, px, py, N, ld);
        s_phi1[k] = s;
    }
    __syncthreads();

    // ---- 2. mubar1 (and the previous psi) on the halo-1 window ----
    // HAS_S instances serve batches in which some domain has the flux S; the
    // per-domain flag selects the branch (uniform across the workgroup)
    const bool dS = HAS_S && d.has_s;
    gptr<const T> psi_in = dS ? gpc<T>(d.psi[cur]) : nullptr;
    for (int k = tid; k < VX * VY; k += NT) {
        const int vx = k % VX, vy = k / VX;
        const int i = (vy + 1) * WX + (vx + 1);
        T mu0, mu1, mu2;
        s_mub[k] = mubar1<T>(K, s_phi0[i], s_phi1[i], lap9(s_phi0, i, WX), lap9(s_phi1, i, WX),
                             mu0, mu1, mu2);
        if (dS) {
            const int sx = map_index(x0 - 1 + vx, nx, px);
            const int sy = map_index(y0 - 1 + vy, ny, py);
            s_psi[k] = psi_in[sy * ld + sx];
        }
    }
    __syncthreads();

    // ---- 3. per-node macroscopic fields and collisions ----
    gptr<const T> lagA = gpc<T>(d.lagA);
    gptr<const T> lagB = gpc<T>(d.lagB);
    gptr<const T> lagC = gpc<T>(d.lagC);
    for (int k = tid; k < TX * TY; k += NT) {
        const int lx = k % TX, ly = k / TX;
        const int x = x0 + lx, y = y0 + ly;
        if (x >= nx || y >= ny) continue;
        const int id = y * ld + x;
        const int ip = (ly + 2) * WX + (lx + 2);
        const int iv = (ly + 1) * VX + (lx + 1);
        T gx0, gy0, lap0, gx1, gy1, lap1, gmx, gmy, dpx = T(0), dpy = T(0);
        stencil9(s_phi0, ip, WX, gx0, gy0, lap0);
        stencil9(s_phi1, ip, WX, gx1, gy1, lap1);
        grad9(s_mub, iv, VX, gmx, gmy);
        T lCxx = T(0), lCyy = T(0), lCxy = T(0);
        if (dS) {
            grad9(s_psi, iv, VX, dpx, dpy);
            lCxx = lagC[id];
            lCyy = lagC[N + id];
            lCxy = lagC[2 * N + id];
        }
        T fp[9], gq[9];
        pull9(gin, x, y, nx, ny, px, py, N, ld, gq);
        pull9(fin, x, y, nx, ny, px, py, N, ld, fp);
        node_update<T, MODE>(d, K, dS, 0, (uint32_t)id * (uint32_t)sizeof(T), N, x, y, s_phi0[ip], s_phi1[ip], gx0, gy0, lap0, gx1, gy1, lap1,
                             s_mub[iv], gmx, gmy, dpx, dpy, fp, gq, lagA[id], lagA[N + id], lagB[id],
                             lCxx, lCyy, lCxy, cur, mom_out);
    }
}

// ---------------------------------------------------------------------------
// Strip kernel: one wavefront per (domain, 64-column strip, CH-row chunk).
// The wave marches down its chunk one row per iteration r:
//   A. loads the pulled CH populations of row y0 - 2 + r for its 64 columns
//      (kept in a 3-deep register ring) plus 4 halo columns, and writes
//      phi0, phi1 of that row into a 5-row LDS ring;
//   B. computes mubar1 (and stages psi) for the row above into a 3-row ring;
//   C. updates the row two above, whose populations are in registers.
// Each population is read once from memory apart from the 4 halo columns and
// the 4 halo rows of each chunk, which neighbouring waves share through L2.
// ---------------------------------------------------------------------------
template <typename T, bool HAS_S>
struct StripShared {
    T phi0[5][68];
    T phi1[5][68];
    T mub[3][66];
    T psi[HAS_S ? 3 : 1][66];
};

// The LDS rings as one strip sees them: cell i of a phi row is column
// x0 - 2 + i (i < 68), cell c of a mubar / psi row column x0 - 1 + c (c < 66).
// A strip alone owns its rings and produces their halo cells itself.
template <typename T, bool HAS_S>
struct SoloRing {
    StripShared<T, HAS_S>& s;
    bool own_left = true, own_right = true;
    __device__ T* phi0(int k) const { return s.phi0[k]; }
    __device__ T* phi1(int k) const { return s.phi1[k]; }
    __device__ T* mub(int k) const { return s.mub[k]; }
    __device__ T* psi(int k) const { return s.psi[k]; }
};

// The NW strips of a lockstep group share one ring per field, 64 NW + 4 (phi)
// or 64 NW + 2 (mubar, psi) cells wide: strip w's cells start at 64 w, so its
// halo cells are its neighbours' edge cells, written by them in the same
// phase of the same iteration.  Only the group's outer strips (and a strip
// whose right neighbour lies past the domain) produce halo cells.
template <typename T, bool HAS_S, int NW>
struct GroupShared {
    static constexpr int P = 64 * NW + 4, M = 64 * NW + 2;
    T phi0[5][P];
    T phi1[5][P];
    T mub[3][M];
    T psi[HAS_S ? 3 : 1][M];
};

template <typename T, bool HAS_S, int NW>
struct GroupRing {
    GroupShared<T, HAS_S, NW>& g;
    int base;                     // 64 w
    bool own_left, own_right;
    __device__ T* phi0(int k) const { return g.phi0[k] + base; }
    __device__ T* phi1(int k) const { return g.phi1[k] + base; }
    __device__ T* mub(int k) const { return g.mub[k] + base; }
    __device__ T* psi(int k) const { return g.psi[k] + base; }
};

// Load of a pulled population: non-temporal (NT) or plain.  Which is faster
// depends on the tiling: within lockstep groups of 64-row strips NT loads
// measured faster in FP32 (the DRAM streams run closer to copy speed, at the
// price of a few halo columns read twice); where neighbouring strips run in
// different workgroups the shared halo columns then miss the cache.
template <typename T, bool NT>
__device__ __forceinline__ T ld_pop(gptr<const T> p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// Pulled populations of a node whose source columns x - 1, x, x + 1 are given
// as byte offsets cb (wrapped periodically once per tile), in row y: the row
// part of every source address is uniform across the wave (scalar), the
// column part a per-lane offset.  A source row beyond a wall gives the
// opposite population of the node itself (half-way bounce-back).
template <typename T, bool NT>
__device__ __forceinline__ void pull9_cols(gptr<const T> fin, const uint32_t (&cb)[3], int y, int ld, int ny,
                                           int py, int N, T (&out)[9]) {
    int ym = y - 1, yp = y + 1;
    bool wall = false;
    if (py) {
        ym = ym < 0 ? ym + ny : ym;
        yp = yp >= ny ? yp - ny : yp;
    } else {
        wall = ym < 0 || yp >= ny;
    }
    if (!wall) {
        // source row of population q is y - cy_q: rows[1 - cy_q]
        gptr<const T> rows[3] = {fin + (int64_t)ym * ld, fin + (int64_t)y * ld, fin + (int64_t)yp * ld};
#pragma unroll
        for (int q = 0; q < 9; ++q) out[q] = ld_pop<T, NT>(at_bytes(rows[1 - cy_of(q)] + (int64_t)q * N, cb[1 - cx_of(q)]));
        return;
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int ys = y - cy_of(q);
        const bool w = ys < 0 || ys >= ny;
        const int64_t rowq = w ? (int64_t)opp_of(q) * N + (int64_t)y * ld : (int64_t)q * N + (int64_t)ys * ld;
        out[q] = *at_bytes(fin + rowq, w ? cb[1] : cb[1 - cx_of(q)]);
    }
}

// Byte offsets of the columns x - 1, x, x + 1 around column x (any integer),
// wrapped periodically.
template <typename T>
__device__ __forceinline__ void wrap_cols(int x, int nx, uint32_t (&cb)[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) cb[k] = (uint32_t)map_index(x - 1 + k, nx, 1) * (uint32_t)sizeof(T);
}

// One iteration r of the strip kernel.  PX: the domain is periodic in x, so
// each lane's source columns are fixed for the whole tile (cb: own column,
// hb: the halo column of lanes 0..3) and every load uses scalar-base
// addressing; otherwise the general pull with per-lane wall handling.
template <typename T, int CH, bool HAS_S, int MODE, bool PX, int NT, typename RG>
__device__ __forceinline__ void strip_iter(const DomDev& d, const KConst<T>& K, const RG& sh, int r, int x0,
                                           int y0, int lane, int cur, bool dS, const uint32_t (&cb)[3],
                                           const uint32_t (&hb)[3], T (&fL)[9], T (&fU)[9],
                                           double* __restrict__ mom_out) {
    const int nx = d.nx, ny = d.ny, px = d.px, py = d.py;
    const int ld = d.pitch, N = ld * ny;
    gptr<const T> fin = gpc<T>(d.f[cur]);
    gptr<const T> phi0 = gpc<T>(d.phi0);
    const int yr = y0 - 2 + r;          // phi row loaded in this iteration
    const int yu = yr - 2;              // row updated in this iteration
    const int x = x0 + lane;
    const bool do_update = (r >= 4) && (yu < ny) && (x < nx);
    const int64_t rowu = (int64_t)yu * ld;
    // byte offset of the updated node within its row (x < nx when updating)
    const uint32_t cu = PX ? cb[1] : (uint32_t)x * (uint32_t)sizeof(T);

    // A. loads of row yr: the pulled CH populations and phi0 of the own
    // column and (lanes 0..3) of the 4 halo columns; issued before the NS
    // prefetch below, so that waiting for them does not wait for that too
    const int slot5 = r % 5;
    const int sy = map_index(yr, ny, py);
    const int cxh = lane < 2 ? lane : 64 + lane;   // halo cells 0, 1, 66, 67 (lanes 0..3)
    // lanes 0, 1 produce the left halo cells, 2, 3 the right ones, where the
    // strip owns them
    const bool load_halo = lane < 2 ? sh.own_left : (lane < 4 && sh.own_right);
    T hF[9], p0v, h0v = T(0);
    // loads at the highest wavefront priority (until the NS prefetch below
    // is issued), so that a memory-bound wavefront gets its loads out before
    // the others' arithmetic
    __builtin_amdgcn_s_setprio(3);
    if constexpr (PX) {
        pull9_cols<T, (NT & 2) != 0>(fin, cb, sy, ld, ny, py, N, fL);
        p0v = *at_bytes(phi0 + (int64_t)sy * ld, cb[1]);
        if (load_halo) {
            // plain loads, not non-temporal: the halo cells are a
            // neighbouring strip's interior (another wavefront's or another
            // workgroup's), and lines loaded this way stay in the caches for
            // its read
            pull9_cols<T, false>(fin, hb, sy, ld, ny, py, N, hF);
            h0v = *at_bytes(phi0 + (int64_t)sy * ld, hb[1]);
        }
    } else {
        const int sx = map_index(x, nx, px);
        pull9(fin, sx, sy, nx, ny, px, py, N, ld, fL);
        p0v = phi0[sy * ld + sx];
        if (load_halo) {
            const int hx = map_index(x0 - 2 + cxh, nx, px);
            pull9(fin, hx, sy, nx, ny, px, py, N, ld, hF);
            h0v = phi0[sy * ld + hx];
        }
    }

    // prefetch the NS populations and lagged fields of the row to update
    // (used in C)
    T gpl[9];
    T lAx = T(0), lAy = T(0), lB = T(0), lCxx = T(0), lCyy = T(0), lCxy = T(0);
    if (do_update) {
        if constexpr (PX) pull9_cols<T, (NT & 1) != 0>(gpc<T>(d.g[cur]), cb, yu, ld, ny, py, N, gpl);
        else pull9(gpc<T>(d.g[cur]), x, yu, nx, ny, px, py, N, ld, gpl);
        lAx = *at_bytes(gpc<T>(d.lagA) + rowu, cu);
        lAy = *at_bytes(gpc<T>(d.lagA) + (N + rowu), cu);
        lB = *at_bytes(gpc<T>(d.lagB) + rowu, cu);
        if (dS) {
            lCxx = *at_bytes(gpc<T>(d.lagC) + rowu, cu);
            lCyy = *at_bytes(gpc<T>(d.lagC) + (N + rowu), cu);
            lCxy = *at_bytes(gpc<T>(d.lagC) + (2 * (int64_t)N + rowu), cu);
        }
    }
    __builtin_amdgcn_s_setprio(0);

    // phi1 = sum of the pulled populations, into the LDS ring with phi0
    {
        T s = fL[0];
#pragma unroll
        for (int q = 1; q < 9; ++q) s += fL[q];
        sh.phi1(slot5)[lane + 2] = s;
        sh.phi0(slot5)[lane + 2] = p0v;
        if (load_halo) {
            T t = hF[0];
#pragma unroll
            for (int q = 1; q < 9; ++q) t += hF[q];
            sh.phi1(slot5)[cxh] = t;
            sh.phi0(slot5)[cxh] = h0v;
        }
    }
    __syncthreads();

    // B. mubar1 (and psi) of row yr - 1 on 66 cells (x0 - 1 .. x0 + 64)
    const int slot3 = r % 3;
    if (r >= 2) {
        const T* pm = sh.phi1((r + 3) % 5);  // row yr - 2
        const T* p0 = sh.phi1((r + 4) % 5);  // row yr - 1
        const T* pp = sh.phi1(slot5);        // row yr
        const T* qm = sh.phi0((r + 3) % 5);
        const T* q0 = sh.phi0((r + 4) % 5);
        const T* qp = sh.phi0(slot5);
        for (int c = lane; c < 66; c += 64) {
            // the halo cells 0 and 65 only where the strip owns them
            if ((c == 0 && !sh.own_left) || (c == 65 && !sh.own_right)) continue;
            const int i = c + 1;
            const T l1 = (T(4) * (p0[i + 1] + p0[i - 1] + pp[i] + pm[i]) +
                          (pp[i + 1] + pp[i - 1] + pm[i + 1] + pm[i - 1]) - T(20) * p0[i]) * T(1.0 / 6.0);
            const T l0 = (T(4) * (q0[i + 1] + q0[i - 1] + qp[i] + qm[i]) +
                          (qp[i + 1] + qp[i - 1] + qm[i + 1] + qm[i - 1]) - T(20) * q0[i]) * T(1.0 / 6.0);
            T mu0, mu1, mu2;
            sh.mub(slot3)[c] = mubar1<T>(K, q0[i], p0[i], l0, l1, mu0, mu1, mu2);
            if constexpr (HAS_S) {
                if (dS) {
                    const int sx = map_index(x0 - 1 + c, nx, px);
                    const int sy = map_index(yr - 1, ny, py);
                    sh.psi(slot3)[c] = gpc<T>(d.psi[cur])[sy * ld + sx];
                }
            }
        }
    }
    __syncthreads();

    // C. update row yu = yr - 2 (phi rows yu-1..yu+1, mubar rows yu-1..yu+1)
    if (do_update) {
        const int i = lane + 2;   // phi cell of the node
        const int j = lane + 1;   // mubar cell of the node
        const T* pm = sh.phi1((r + 2) % 5);  // row yu - 1
        const T* p0 = sh.phi1((r + 3) % 5);  // row yu
        const T* pp = sh.phi1((r + 4) % 5);  // row yu + 1
        const T* qm = sh.phi0((r + 2) % 5);
        const T* q0 = sh.phi0((r + 3) % 5);
        const T* qp = sh.phi0((r + 4) % 5);
        const T* mm = sh.mub((r + 1) % 3);   // row yu - 1
        const T* m0 = sh.mub((r + 2) % 3);   // row yu
        const T* mp = sh.mub(slot3);         // row yu + 1
        const T gx1 = (T(4) * (p0[i + 1] - p0[i - 1]) + (pp[i + 1] - pp[i - 1] + pm[i + 1] - pm[i - 1])) * T(1.0 / 12.0);
        const T gy1 = (T(4) * (pp[i] - pm[i]) + (pp[i + 1] - pm[i + 1] + pp[i - 1] - pm[i - 1])) * T(1.0 / 12.0);
        const T lap1 = (T(4) * (p0[i + 1] + p0[i - 1] + pp[i] + pm[i]) +
                        (pp[i + 1] + pp[i - 1] + pm[i + 1] + pm[i - 1]) - T(20) * p0[i]) * T(1.0 / 6.0);
        const T gx0 = (T(4) * (q0[i + 1] - q0[i - 1]) + (qp[i + 1] - qp[i - 1] + qm[i + 1] - qm[i - 1])) * T(1.0 / 12.0);
        const T gy0 = (T(4) * (qp[i] - qm[i]) + (qp[i + 1] - qm[i + 1] + qp[i - 1] - qm[i - 1])) * T(1.0 / 12.0);
        const T lap0 = (T(4) * (q0[i + 1] + q0[i - 1] + qp[i] + qm[i]) +
                        (qp[i + 1] + qp[i - 1] + qm[i + 1] + qm[i - 1]) - T(20) * q0[i]) * T(1.0 / 6.0);
        const T gmx = (T(4) * (m0[j + 1] - m0[j - 1]) + (mp[j + 1] - mp[j - 1] + mm[j + 1] - mm[j - 1])) * T(1.0 / 12.0);
        const T gmy = (T(4) * (mp[j] - mm[j]) + (mp[j + 1] - mm[j + 1] + mp[j - 1] - mm[j - 1])) * T(1.0 / 12.0);
        T dpx = T(0), dpy = T(0);
        if constexpr (HAS_S) {
            if (dS) {
                const T* sm = sh.psi((r + 1) % 3);
                const T* s0 = sh.psi((r + 2) % 3);
                const T* sp = sh.psi(slot3);
                dpx = (T(4) * (s0[j + 1] - s0[j - 1]) + (sp[j + 1] - sp[j - 1] + sm[j + 1] - sm[j - 1])) * T(1.0 / 12.0);
                dpy = (T(4) * (sp[j] - sm[j]) + (sp[j + 1] - sm[j + 1] + sp[j - 1] - sm[j - 1])) * T(1.0 / 12.0);
            }
        }
        node_update<T, MODE>(d, K, dS, rowu, cu, N, x, yu, q0[i], p0[i], gx0, gy0, lap0, gx1, gy1, lap1, m0[j], gmx,
                             gmy, dpx, dpy, fU, gpl, lAx, lAy, lB, lCxx, lCyy, lCxy, cur, mom_out);
    }
}

// One (domain, strip, chunk) tile of the strip kernel at the given step offset.
template <typename T, int CH, bool HAS_S, int MODE, bool PX, int NT, typename RG>
__device__ __forceinline__ void strip_rows(const DomDev& d, const RG& sh, int x0, int y0, int step_offset,
                                           double* __restrict__ mom_out) {
    const KConst<T> K = kconst<T>(d);
    const int cur = (d.parity + step_offset) & 1;
    const bool dS = HAS_S && d.has_s;
    const int lane = threadIdx.x & 63;
    uint32_t cb[3] = {0, 0, 0}, hb[3] = {0, 0, 0};
    if constexpr (PX) {
        wrap_cols<T>(x0 + lane, d.nx, cb);
        const int cx = lane < 2 ? lane : 64 + lane;   // halo cells 0, 1, 66, 67 (lanes 0..3)
        wrap_cols<T>(x0 - 2 + cx, d.nx, hb);
    }
    T F0[9], F1[9], F2[9];
    // row ring: iteration r loads into F[r % 3] and updates with F[(r + 1) % 3]
    // (the row loaded two iterations earlier)
    constexpr int R = CH + 4;
    for (int r = 0; r < R; r += 3) {
        strip_iter<T, CH, HAS_S, MODE, PX, NT, RG>(d, K, sh, r, x0, y0, lane, cur, dS, cb, hb, F0, F1, mom_out);
        if (r + 1 < R)
            strip_iter<T, CH, HAS_S, MODE, PX, NT, RG>(d, K, sh, r + 1, x0, y0, lane, cur, dS, cb, hb, F1, F2, mom_out);
        if (r + 2 < R)
            strip_iter<T, CH, HAS_S, MODE, PX, NT, RG>(d, K, sh, r + 2, x0, y0, lane, cur, dS, cb, hb, F2, F0, mom_out);
    }
}

template <typename T, int CH, bool HAS_S, int MODE, int NT, typename RG>
__device__ __forceinline__ void strip_tile_r(const DomDev& d, const RG& ring, int x0, int y0, int step_offset,
                                             double* __restrict__ mom_out) {
    if (d.px) strip_rows<T, CH, HAS_S, MODE, true, NT, RG>(d, ring, x0, y0, step_offset, mom_out);
    else strip_rows<T, CH, HAS_S, MODE, false, NT, RG>(d, ring, x0, y0, step_offset, mom_out);
}

template <typename T, int CH, bool HAS_S, int MODE, int NT = 0>
__device__ __forceinline__ void strip_tile(const DomDev& d, StripShared<T, HAS_S>& sh, int x0, int y0,
                                           int step_offset, double* __restrict__ mom_out) {
    const SoloRing<T, HAS_S> ring{sh};
    strip_tile_r<T, CH, HAS_S, MODE, NT>(d, ring, x0, y0, step_offset, mom_out);
}

template <typename T, int CH, bool HAS_S, int MODE>
__device__ __forceinline__ void strip_body(const DomDev* __restrict__ doms, const int4* __restrict__ tiles,
                                           int ntiles, int step_offset, double* __restrict__ mom_out) {
    __shared__ StripShared<T, HAS_S> sh;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    if (t >= ntiles) return;
    const int4 tile = tiles[t];
    const DomDev& d = doms[tile.x];
    if (!d.live && MODE == kModeStep) return;
    strip_tile<T, CH, HAS_S, MODE>(d, sh, tile.y, tile.z, step_offset, mom_out);
}

// ---------------------------------------------------------------------------
// FP64 reductions with compensated (Neumaier/TwoSum) accumulation
// ---------------------------------------------------------------------------
struct CSum {
    double s, c;
};

__device__ __forceinline__ void csum_add(CSum& a, double v) {
    double t = a.s + v;
    if (fabs(a.s) >= fabs(v)) a.c += (a.s - t) + v;
    else a.c += (v - t) + a.s;
    a.s = t;
}

__device__ __forceinline__ void csum_merge(CSum& a, const CSum& b) {
    csum_add(a, b.s);
    a.c += b.c;
}

// Residual check of one domain inside the launch, by one workgroup: phi1 of
// the state after call step `cs` (pulled sums of the CH populations in
// buffer `buf`), sum (phi1 - snap)^2, sum phi1^2, sum phi1 and the
// non-finite count in FP64 (compensated per thread, then a fixed-order tree),
// snap <- phi1; the residual as in tpf_run_to_residual.  Returns the
// decision, the same in every thread: 0 live, 1 converged, 2 non-finite.
template <typename T, int NW>
__device__ int persist_check(const DomDev& d, int dom, int buf, int cs, double tol, int* __restrict__ last_check,
                             double* __restrict__ stats, double* red) {
    // snap in the [ny][nx] layout, populations in rows of pitch elements
    const int nx = d.nx, ny = d.ny, N = nx * ny, ld = d.pitch, Np = ld * ny;
    gptr<const T> fin = gpc<T>(d.f[buf]);
    gptr<double> snap = gp<double>(d.snap);
    CSum m = {0, 0}, r = {0, 0}, n2 = {0, 0};
    double bad = 0.0;
    for (int id = threadIdx.x; id < N; id += 64 * NW) {
        const int y = id / nx, x = id - y * nx;
        T sum = pull(fin, 0, x, y, nx, ny, d.px, d.py, Np, ld);
#pragma unroll
        for (int q = 1; q < 9; ++q) sum += pull(fin, q, x, y, nx, ny, d.px, d.py, Np, ld);
        const double v = double(sum);
        if (!isfinite(v)) bad += 1.0;
        csum_add(m, v);
        csum_add(n2, v * v);
        const double prev = snap[id];
        if (isfinite(prev)) csum_add(r, (v - prev) * (v - prev));
        snap[id] = v;
    }
    // fixed-order tree over the workgroup in LDS
    double* sh = red;  // [7][64 NW]
    const int T_ = 64 * NW;
    sh[0 * T_ + threadIdx.x] = m.s; sh[1 * T_ + threadIdx.x] = m.c;
    sh[2 * T_ + threadIdx.x] = r.s; sh[3 * T_ + threadIdx.x] = r.c;
    sh[4 * T_ + threadIdx.x] = n2.s; sh[5 * T_ + threadIdx.x] = n2.c;
    sh[6 * T_ + threadIdx.x] = bad;
    __syncthreads();
    for (int w = T_ / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const int o = threadIdx.x + w;
            for (int j = 0; j < 3; ++j) {
                CSum x = {sh[2 * j * T_ + threadIdx.x], sh[(2 * j + 1) * T_ + threadIdx.x]};
                csum_merge(x, CSum{sh[2 * j * T_ + o], sh[(2 * j + 1) * T_ + o]});
                sh[2 * j * T_ + threadIdx.x] = x.s;
                sh[(2 * j + 1) * T_ + threadIdx.x] = x.c;
            }
            sh[6 * T_ + threadIdx.x] += sh[6 * T_ + o];
        }
        __syncthreads();
    }
    const double mass = sh[0] + sh[T_], d2 = sh[2 * T_] + sh[3 * T_], nn = sh[4 * T_] + sh[5 * T_];
    const double nbad = sh[6 * T_];
    const int prev_check = last_check[dom];
    const double res = (nn > 0.0 && cs > prev_check) ? sqrt(d2) / ((double)(cs - prev_check) * sqrt(nn)) : NAN;
    __syncthreads();   // every thread has read the tree before the next item reuses it
    const int verdict = (nbad > 0.0 || !isfinite(mass)) ? 2 : ((isfinite(res) && res < tol) ? 1 : 0);
    if (threadIdx.x < 64) {   // wavefront 0, every lane the same values
        last_check[dom] = cs;
        stats[4 * dom + 0] = res;
        stats[4 * dom + 1] = mass;
        stats[4 * dom + 2] = nbad;
        stats[4 * dom + 3] = verdict == 2 ? 1.0 : 0.0;
    }
    return verdict;
}

// ---------------------------------------------------------------------------
// Persistent launcher: one launch advances every live domain by a.nsteps
// steps.  Work items are handed out in increasing order from a device
// counter.  Without residual checks step s holds the ntiles tile items of
// the table.  With checks every K = check_every steps, the items come in
// blocks of K steps: the K ntiles tile items (step by step), then one check
// item per live domain for the block's last step; the launch's last block
// may be shorter (the call's last step, which also gets a check).
// Before step s of a domain a workgroup waits until the domain's tiles of
// steps < s and its checks of earlier blocks have finished; a check item
// waits for the tiles of its own step (per-domain completion counters,
// release/acquire at device scope).  A workgroup only ever waits for items
// handed out before its own, held by running workgroups, so the queue cannot
// deadlock; a bounded spin sets a failure flag and lets every workgroup
// leave should a wait exceed the limit.  A domain whose check finds
// r < tol, or non-finite values, leaves: its later items are no-ops, and
// when no domain is left every workgroup leaves.
//   NW = 1: single strips (tile codes 8-10); NW > 1: lockstep groups of NW
//   strips (codes 17-24), as in strip_group_body.
// All control flow in the loop is uniform within each wavefront, and every
// wavefront meets the same barriers: wavefront 0 fetches, waits and
// decides, and broadcasts through LDS; the others take an acquire fence
// after the barrier that ends the wait.  (A "lane 0 only" branch around the
// item fetch once let lanes 1..63 of a one-wave workgroup run ahead into a
// loop of their own: a hang.)
// ---------------------------------------------------------------------------
template <typename T, int CH, bool HAS_S, int NW, int NT, bool SHARE>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && NW > 1 ? 3 : 1, 8)))
persistent_kernel(const DomDev* __restrict__ doms, PersistArgs a) {
    constexpr bool GROUP = NW > 1;
    using Shared = typename std::conditional<GROUP && SHARE, GroupShared<T, HAS_S, NW>,
                                             StripShared<T, HAS_S>>::type;
    __shared__ Shared rings[(GROUP && !SHARE) ? NW : 1];
    __shared__ double red[7 * 64 * NW];
    __shared__ int bc[4];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const bool checks = a.check_every > 0;
    const int K = checks ? a.check_every : a.nsteps;            // steps per block
    const int block_items = K * a.ntiles + (checks ? a.nlive : 0);
    const int full = a.nsteps / K, rem = a.nsteps - full * K;
    const int total = full * block_items + rem * a.ntiles + (checks && rem > 0 ? a.nlive : 0);
    for (;;) {
        // ---- fetch (wavefront 0) and broadcast ----
        if (w == 0) {
            const int item = __builtin_amdgcn_readfirstlane(atomicAdd(&a.ctl[0], lane == 0 ? 1 : 0));
            const int live = __builtin_amdgcn_readfirstlane(
                __hip_atomic_load(&a.ctl[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            bc[0] = item;
            bc[1] = live;
        }
        __syncthreads();
        const int item = bc[0], live_now = bc[1];
        __syncthreads();
        if (item >= total || live_now <= 0) break;
        const int b = item / block_items, r = item - b * block_items;
        const int steps_b = b < full ? K : rem;
        const bool is_check = r >= steps_b * a.ntiles;
        const int s = b * K + (is_check ? steps_b - 1 : r / a.ntiles);
        const int k = is_check ? r - steps_b * a.ntiles : r - (r / a.ntiles) * a.ntiles;
        const int dom = is_check ? a.live_doms[k] : a.tiles[k].x;
        const int tiles_d = a.dom_tiles[dom];
        // finished items of dom this item needs: tiles of steps < s (< s + 1
        // for a check) and the checks of earlier blocks
        const int need = tiles_d * (is_check ? s + 1 : s) + (checks ? s / K : 0);
        // ---- wait (wavefront 0) and vote ----
        if (w == 0) {
            int verdict = 0;   // 0 go on, 1 failure, 2 no domain left
            if (need > 0) {
                // relaxed polls (an acquire per poll would invalidate the
                // caches each time), one acquire fence once the count is met;
                // the live count and the failure flag every 32nd poll
                int it = 0;
                for (;;) {
                    const int got = __builtin_amdgcn_readfirstlane(
                        __hip_atomic_load(&a.done[dom], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                    if (got >= need) break;
                    ++it;
                    if ((it & 31) == 0) {
                        if (__builtin_amdgcn_readfirstlane(
                                __hip_atomic_load(&a.ctl[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) <= 0) {
                            verdict = 2;
                            break;
                        }
                        if (it > a.spin_limit || __builtin_amdgcn_readfirstlane(__hip_atomic_load(
                                                     &a.ctl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != 0) {
                            verdict = 1;
                            break;
                        }
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
                if (verdict == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            bc[2] = verdict;
        }
        __syncthreads();
        const int vote = bc[2];
        __syncthreads();
        if (vote == 1) {
            if (w == 0) __hip_atomic_store(&a.ctl[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        if (vote == 2) break;
        // the other wavefronts read what the awaited items wrote after the
        // barrier that follows wavefront 0's acquire (one compute unit, one
        // vector L1, invalidated by that acquire)
        const DomDev& d = doms[dom];
        const int rstep = a.retired[dom];
        const bool active = rstep < 0;   // a check of step s - 1 has been seen (acquire above)
        if (active) {
            if (is_check) {
                const int cs = a.step_base + s + 1;
                const int buf = (d.parity + s + 1) & 1;
                const int verdict = persist_check<T, NW>(d, dom, buf, cs, a.tol, a.last_check, a.stats, red);
                if (verdict != 0 && w == 0) {   // wavefront 0 as a whole
                    a.retired[dom] = s;
                    __hip_atomic_fetch_add(&a.ctl[2], lane == 0 ? -1 : 0, __ATOMIC_RELEASE,
                                           __HIP_MEMORY_SCOPE_AGENT);
                }
            } else {
                const int4 tile = a.tiles[k];
                if constexpr (!GROUP) {
                    strip_tile<T, CH, HAS_S, kModeStep, NT>(d, rings[0], tile.y, tile.z, s, nullptr);
                } else {
                    const int x0 = tile.y + 64 * w;
                    if (x0 >= d.nx) {
                        for (int r = 0; r < CH + 4; ++r) {
                            __syncthreads();
                            __syncthreads();
                        }
                    } else if constexpr (SHARE) {
                        const GroupRing<T, HAS_S, NW> ring{rings[0], 64 * w, w == 0, w == NW - 1 || x0 + 64 >= d.nx};
                        strip_tile_r<T, CH, HAS_S, kModeStep, NT>(d, ring, x0, tile.z, s, nullptr);
                    } else {
                        strip_tile<T, CH, HAS_S, kModeStep, NT>(d, rings[w], x0, tile.z, s, nullptr);
                    }
                }
            }
        }
        // every wavefront waits until its own stores have reached the L2
        // before wavefront 0's release (which writes the L2 back for the
        // other XCDs) publishes the item
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (w == 0) __hip_atomic_fetch_add(&a.done[dom], lane == 0 ? 1 : 0, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

static __global__ void zero_ints(int* __restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

template <typename T, int CH, bool HAS_S, int MODE>
__global__ void __launch_bounds__(64)
strip_kernel(const DomDev* __restrict__ doms, const int4* __restrict__ tiles, int ntiles,
             int step_offset, double* __restrict__ mom_out) {
    strip_body<T, CH, HAS_S, MODE>(doms, tiles, ntiles, step_offset, mom_out);
}

// NW wavefronts per workgroup, each marching its own 64-column strip of a
// (64 NW)-column tile.  The two barriers of every strip iteration are then
// workgroup barriers, so the NW strips advance row by row in lockstep and the
// columns that neighbouring strips share (their stencil and pull halos) are
// read while the other strip's wavefront holds the same cache lines.
template <typename T, int CH, bool HAS_S, int MODE, int NW, int NT, bool SHARE>
__device__ __forceinline__ void strip_group_body(const DomDev* __restrict__ doms, const int4* __restrict__ tiles,
                                                 int ntiles, int step_offset, double* __restrict__ mom_out) {
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    if (t >= ntiles) return;
    const int4 tile = tiles[t];
    const DomDev& d = doms[tile.x];
    if (!d.live && MODE == kModeStep) return;
    const int w = threadIdx.x >> 6;
    const int x0 = tile.y + 64 * w;
    if (x0 >= d.nx) {
        // strip entirely beyond the domain's last column (a ragged tile): no
        // work, but the wavefront keeps meeting the two barriers of every
        // row of its group
        for (int r = 0; r < CH + 4; ++r) {
            __syncthreads();
            __syncthreads();
        }
        return;
    }
    if constexpr (SHARE) {
        // one ring per field for the whole group: the outer strips of the
        // group, and a strip whose right neighbour lies past the domain's
        // last column, produce the halo cells on that side
        static_assert(sizeof(GroupShared<T, HAS_S, NW>) <= 65536, "LDS of a workgroup is limited to 64 KB");
        __shared__ GroupShared<T, HAS_S, NW> g;
        const GroupRing<T, HAS_S, NW> ring{g, 64 * w, w == 0, w == NW - 1 || x0 + 64 >= d.nx};
        strip_tile_r<T, CH, HAS_S, MODE, NT>(d, ring, x0, tile.z, step_offset, mom_out);
    } else {
        // a ring per strip, each with its own halo cells
        static_assert(sizeof(StripShared<T, HAS_S>) * NW <= 65536, "LDS of a workgroup is limited to 64 KB");
        __shared__ StripShared<T, HAS_S> sh[NW];
        strip_tile<T, CH, HAS_S, MODE, NT>(d, sh[w], x0, tile.z, step_offset, mom_out);
    }
}

// Compiled for four wavefronts per SIMD (at most 128 VGPRs).  SHARE: the
// strips share one LDS ring per field (halo cells from the neighbours).
template <typename T, int CH, bool HAS_S, int MODE, int NW, bool SHARE>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(4, 8)))
strip_group_kernel(const DomDev* __restrict__ doms, const int4* __restrict__ tiles, int ntiles,
                   int step_offset, double* __restrict__ mom_out) {
    strip_group_body<T, CH, HAS_S, MODE, NW, 0, SHARE>(doms, tiles, ntiles, step_offset, mom_out);
}

// The same groups with the register budget left to the compiler (the FP64
// step takes about 230 VGPRs, two wavefronts per SIMD), so the FP64 build
// gets the shared halos without spilling.  NT selects non-temporal loads of
// the pulled populations: bit 0 the NS lattice g, bit 1 the CH lattice f.
template <typename T, int CH, bool HAS_S, int MODE, int NW, int NT, bool SHARE>
__global__ void __launch_bounds__(64 * NW)
strip_group_kernel_wide(const DomDev* __restrict__ doms, const int4* __restrict__ tiles, int ntiles,
                        int step_offset, double* __restrict__ mom_out) {
    strip_group_body<T, CH, HAS_S, MODE, NW, NT, SHARE>(doms, tiles, ntiles, step_offset, mom_out);
}

// Initial state (per node): f = f^eq(phi1, eta mubar1, u = 0), g = g^eq(P = 0,
// u = 0) = gauge delta_q0, lagged fields zero.  phi1 comes from a float64 field.
template <typename T>
__global__ void init_kernel(const DomDev* __restrict__ doms, int dom, const double* __restrict__ phi1_in) {
    const DomDev& d = doms[dom];
    const int nx = d.nx, ny = d.ny, N = nx * ny;
    const int id = blockIdx.x * blockDim.x + threadIdx.x;   // node in the [ny][nx] layout of phi1_in and snap
    if (id >= N) return;
    const int x = id % nx, y = id / nx;
    const int ld = d.pitch, Np = ld * ny;
    const int o = y * ld + x;                                  // node in the fields' rows of pitch elements
    gptr<const T> phi0 = gpc<T>(d.phi0);
    T v0[9], v1[9];
    int k = 0;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx, ++k) {
            int sx = map_index(x + dx, nx, d.px), sy = map_index(y + dy, ny, d.py);
            v0[k] = phi0[sy * ld + sx];
            v1[k] = T(phi1_in[sy * nx + sx]);
        }
    // row-major 3x3 neighbourhood, centre at index 4, pitch 3
    const T lap0 = lap9(v0, 4, 3), lap1 = lap9(v1, 4, 3);
    T mu0, mu1, mu2;
    const KConst<T> K = kconst<T>(d);
    const T mub = mubar1<T>(K, v0[4], v1[4], lap0, lap1, mu0, mu1, mu2);
    const T c2 = K.c2, w0 = K.w0;
    const T w1 = (c2 - c2 * c2) * T(0.5), w5 = c2 * c2 * T(0.25);
    const T emu = K.eta * mub;
    const int par = d.parity;
    gptr<T> f = gp<T>(d.f[par]);
    gptr<T> g = gp<T>(d.g[par]);
    f[o] = v1[4] + (w0 - T(1)) * emu;
    for (int q = 1; q <= 4; ++q) f[q * Np + o] = w1 * emu;
    for (int q = 5; q <= 8; ++q) f[q * Np + o] = w5 * emu;
    g[o] = K.gauge;
    for (int q = 1; q < 9; ++q) g[q * Np + o] = T(0);
    gptr<T> A = gp<T>(d.lagA);
    A[o] = T(0);
    A[Np + o] = T(0);
    gp<T>(d.lagB)[o] = T(0);
    if (d.has_s) {
        gptr<T> Cl = gp<T>(d.lagC);
        Cl[o] = T(0);
        Cl[Np + o] = T(0);
        Cl[2 * Np + o] = T(0);
        gp<T>(d.psi[0])[o] = T(0);
        gp<T>(d.psi[1])[o] = T(0);
    }
    gp<double>(d.snap)[id] = __builtin_nan("");
}

constexpr int kRedMaxBlocks = 256;  // partial-sum blocks per domain (upper bound)
constexpr int kRedThreads = 256;

// Per domain (blockIdx.y), rows y = blockIdx.x + k gridDim.x, columns by
// thread: phi1 = sum of the pulled CH populations; accumulates sum phi1,
// sum (phi1 - snap)^2, sum phi1^2 and a non-finite count, and (when
// update_snap) stores phi1 into snap.  partials: [dom][gridDim.x][7].
template <typename T>
__global__ void __launch_bounds__(kRedThreads)
reduce_partials(const DomDev* __restrict__ doms, const int* __restrict__ dom_list, int update_snap,
                double* __restrict__ partials) {
    const int dom = dom_list[blockIdx.y];
    const DomDev& d = doms[dom];
    const int nx = d.nx, ny = d.ny, ld = d.pitch, Np = ld * ny;
    gptr<const T> fin = gpc<T>(d.f[d.parity]);
    gptr<double> snap = gp<double>(d.snap);   // [ny][nx]
    CSum m = {0, 0}, r = {0, 0}, n2 = {0, 0};
    double bad = 0.0;
    for (int y = blockIdx.x; y < ny; y += gridDim.x) {
        for (int x = threadIdx.x; x < nx; x += kRedThreads) {
            const int id = y * nx + x;
            T s = pull(fin, 0, x, y, nx, ny, d.px, d.py, Np, ld);
#pragma unroll
            for (int q = 1; q < 9; ++q) s += pull(fin, q, x, y, nx, ny, d.px, d.py, Np, ld);
            const double v = double(s);
            if (!isfinite(v)) bad += 1.0;
            csum_add(m, v);
            csum_add(n2, v * v);
            const double prev = snap[id];
            if (isfinite(prev)) csum_add(r, (v - prev) * (v - prev));
            if (update_snap) snap[id] = v;
        }
    }
    __shared__ double sh[7][kRedThreads];
    sh[0][threadIdx.x] = m.s; sh[1][threadIdx.x] = m.c;
    sh[2][threadIdx.x] = r.s; sh[3][threadIdx.x] = r.c;
    sh[4][threadIdx.x] = n2.s; sh[5][threadIdx.x] = n2.c;
    sh[6][threadIdx.x] = bad;
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const int o = threadIdx.x + w;
            for (int j = 0; j < 3; ++j) {
                CSum a = {sh[2 * j][threadIdx.x], sh[2 * j + 1][threadIdx.x]};
                CSum b = {sh[2 * j][o], sh[2 * j + 1][o]};
                csum_merge(a, b);
                sh[2 * j][threadIdx.x] = a.s;
                sh[2 * j + 1][threadIdx.x] = a.c;
            }
            sh[6][threadIdx.x] += sh[6][o];
        }
        __syncthreads();
    }
    if (threadIdx.x < 7)
        partials[((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 7 + threadIdx.x] = sh[threadIdx.x][0];
}

// One thread per domain: folds the partials in a fixed order.
// out: [dom][4] = mass, sum (phi1 - snap)^2, sum phi1^2, non-finite count.
static __global__ void reduce_final(const int* __restrict__ dom_list, int ndom, int nblk,
                             const double* __restrict__ partials, double* __restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ndom) return;
    CSum m = {0, 0}, r = {0, 0}, n2 = {0, 0};
    double bad = 0.0;
    for (int b = 0; b < nblk; ++b) {
        const double* p = partials + ((size_t)j * nblk + b) * 7;
        csum_merge(m, CSum{p[0], p[1]});
        csum_merge(r, CSum{p[2], p[3]});
        csum_merge(n2, CSum{p[4], p[5]});
        bad += p[6];
    }
    const int dom = dom_list[j];
    out[dom * 4 + 0] = m.s + m.c;
    out[dom * 4 + 1] = r.s + r.c;
    out[dom * 4 + 2] = n2.s + n2.c;
    out[dom * 4 + 3] = bad;
}

// Open ends in x by non-equilibrium extrapolation (Sec. 4): after a step,
// the inlet (x = 0) and outlet (x = nx - 1) nodes of each open domain take
// their equilibrium at the boundary values plus the non-equilibrium part of
// their inner neighbour n (x = 1, x = nx - 2) of that step.  With the
// equilibria written by their Hermite moments (the relaxation targets of the
// collisions), f(b) = f(n) + M^-1 [h^eq(b) - h^eq(n)], the same for g.
// Boundary values: inlet phi1 = phi1_in (1 - phi0), mubar1 = 0, S = 0, and
// p = p_in with u from n (inlet_type 0) or u = (u_in, 0) with p from n (1);
// outlet p = p_out, the rest from n.  The lagged fields of b are set from
// the same values.  Grid: x over the 2 ny (side, y) pairs, y over the open
// domains; step_offset as in the step just launched.
template <typename T>
__global__ void open_bc_kernel(const DomDev* __restrict__ doms, const int* __restrict__ open, int n_open,
                               int step_offset) {
    if ((int)blockIdx.y >= n_open) return;
    const DomDev& d = doms[open[blockIdx.y]];
    if (!d.live) return;
    const int nx = d.nx, ny = d.ny, ld = d.pitch, N = ld * ny;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * ny) return;
    const int side = t / ny, y = t - side * ny;
    const KConst<T> K = kconst<T>(d);
    const T c2 = K.c2;
    const int out = (d.parity + step_offset + 1) & 1;
    const int ib = y * ld + (side ? nx - 1 : 0), in = y * ld + (side ? nx - 2 : 1);
    gptr<const T> bn = gpc<T>(d.bnd) + side * kBndFields * ny + y;
    const T p1n = bn[kBndPhi1 * ny], mbn = bn[kBndMub * ny], uxn = bn[kBndUx * ny], uyn = bn[kBndUy * ny];
    const T pn = bn[kBndP * ny], Sxn = bn[kBndSx * ny], Syn = bn[kBndSy * ny];
    gptr<const T> phi0 = gpc<T>(d.phi0);
    const T p0n = phi0[in], p0b = phi0[ib];
    T p1b, mbb, uxb, uyb, pb, Sxb, Syb;
    if (side == 0) {
        p1b = K.phi1_in * (T(1) - p0b);
        mbb = T(0);
        Sxb = Syb = T(0);
        if (d.inlet_type == 0) {
            pb = K.p_in;
            uxb = uxn;
            uyb = uyn;
        } else {
            pb = pn;
            uxb = K.u_in;
            uyb = T(0);
        }
    } else {
        p1b = p1n;
        mbb = mbn;
        pb = K.p_out;
        uxb = uxn;
        uyb = uyn;
        Sxb = Sxn;
        Syb = Syn;
    }
    const T rn = K.rho0 * p0n + K.rho1 * p1n + K.rho2 * (T(1) - p0n - p1n);
    const T rb = K.rho0 * p0b + K.rho1 * p1b + K.rho2 * (T(1) - p0b - p1b);
    T dh[9], dp[9];
    // CH lattice: h^eq = (phi, phi u, c2 (eta mub - phi) twice, 0, 0, 0, c2^2 (phi - eta mub))
    {
        const T eb = K.eta * mbb, en = K.eta * mbn;
        dh[0] = p1b - p1n;
        dh[1] = p1b * uxb - p1n * uxn;
        dh[2] = p1b * uyb - p1n * uyn;
        dh[3] = c2 * ((eb - p1b) - (en - p1n));
        dh[4] = dh[3];
        dh[5] = dh[6] = dh[7] = T(0);
        dh[8] = c2 * c2 * ((p1b - eb) - (p1n - en));
        from_hermite(dh, dp, c2);
        gptr<T> f = gp<T>(d.f[out]);
#pragma unroll
        for (int q = 0; q < 9; ++q) f[q * N + ib] = f[q * N + in] + dp[q];
    }
    // NS lattice: h^eq = (gauge, rho u, p + Pi_xx - c2 gauge, p + Pi_yy - c2 gauge, Pi_xy, 0, 0,
    // c2^2 gauge - c2 p), Pi = rho uu - (Su + uS)/2; the gauge cancels in the difference
    {
        const T Pxxb = rb * uxb * uxb - Sxb * uxb, Pyyb = rb * uyb * uyb - Syb * uyb;
        const T Pxyb = rb * uxb * uyb - T(0.5) * (Sxb * uyb + uxb * Syb);
        const T Pxxn = rn * uxn * uxn - Sxn * uxn, Pyyn = rn * uyn * uyn - Syn * uyn;
        const T Pxyn = rn * uxn * uyn - T(0.5) * (Sxn * uyn + uxn * Syn);
        dh[0] = T(0);
        dh[1] = rb * uxb - rn * uxn;
        dh[2] = rb * uyb - rn * uyn;
        dh[3] = (pb + Pxxb) - (pn + Pxxn);
        dh[4] = (pb + Pyyb) - (pn + Pyyn);
        dh[5] = Pxyb - Pxyn;
        dh[6] = dh[7] = T(0);
        dh[8] = -c2 * (pb - pn);
        from_hermite(dh, dp, c2);
        gptr<T> g = gp<T>(d.g[out]);
#pragma unroll
        for (int q = 0; q < 9; ++q) g[q * N + ib] = g[q * N + in] + dp[q];
    }
    gptr<T> A = gp<T>(d.lagA);
    A[ib] = p1b * uxb;
    A[N + ib] = p1b * uyb;
    gp<T>(d.lagB)[ib] = (rb * uxb - Sxb) * uxb + (rb * uyb - Syb) * uyb;
    if (d.has_s) {
        gptr<T> Cl = gp<T>(d.lagC);
        Cl[ib] = Sxb * uxb;
        Cl[N + ib] = Syb * uyb;
        Cl[2 * N + ib] = T(0.5) * (Sxb * uyb + Syb * uxb);
        gp<T>(d.psi[out])[ib] = Sxb * uyb - Syb * uxb;
    }
}

// Flow rates of one domain over its pore space (phi0 <= 1/2): sums of u_x,
// phi1 u_x and phi2 u_x (Sec. 4.6), from the moments kernel's output
// mom = [phi1; ux; uy; p] (float64, N each).  partials: [3][2][gridDim.x]
// compensated per block; flow_final folds them in a fixed order.
template <typename T>
__global__ void __launch_bounds__(kRedThreads)
flow_partials(const DomDev* __restrict__ doms, int dom, const double* __restrict__ mom,
              double* __restrict__ partials) {
    const DomDev& d = doms[dom];
    const int N = d.nx * d.ny;                 // mom in the [ny][nx] layout
    gptr<const T> phi0 = gpc<T>(d.phi0);       // rows of pitch elements
    CSum a = {0, 0}, b = {0, 0}, c = {0, 0};
    for (int id = blockIdx.x * kRedThreads + threadIdx.x; id < N; id += gridDim.x * kRedThreads) {
        const int y = id / d.nx, x = id - y * d.nx;
        const double p0 = double(phi0[y * d.pitch + x]);
        if (p0 > 0.5) continue;
        const double ux = mom[N + id], p1 = mom[id];
        csum_add(a, ux);
        csum_add(b, p1 * ux);
        csum_add(c, (1.0 - p0 - p1) * ux);
    }
    __shared__ double sh[6][kRedThreads];
    sh[0][threadIdx.x] = a.s; sh[1][threadIdx.x] = a.c;
    sh[2][threadIdx.x] = b.s; sh[3][threadIdx.x] = b.c;
    sh[4][threadIdx.x] = c.s; sh[5][threadIdx.x] = c.c;
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const int o = threadIdx.x + w;
            for (int j = 0; j < 3; ++j) {
                CSum x = {sh[2 * j][threadIdx.x], sh[2 * j + 1][threadIdx.x]};
                csum_merge(x, CSum{sh[2 * j][o], sh[2 * j + 1][o]});
                sh[2 * j][threadIdx.x] = x.s;
                sh[2 * j + 1][threadIdx.x] = x.c;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) partials[threadIdx.x * gridDim.x + blockIdx.x] = sh[threadIdx.x][0];
}

static __global__ void flow_final(const double* __restrict__ partials, int nblk, double* __restrict__ out) {
    if (threadIdx.x >= 3) return;
    CSum r = {0, 0};
    for (int k = 0; k < nblk; ++k)
        csum_merge(r, CSum{partials[(2 * threadIdx.x) * nblk + k], partials[(2 * threadIdx.x + 1) * nblk + k]});
    out[threadIdx.x] = r.s + r.c;
}

// Copies the post-collision populations of one domain to float64 [2][9][N].
template <typename T>
__global__ void export_populations(const DomDev* __restrict__ doms, int dom, double* __restrict__ out) {
    const DomDev& d = doms[dom];
    const int N = d.nx * d.ny, Np = d.pitch * d.ny;   // out: [2][9][ny][nx]
    gptr<const T> f = gpc<T>(d.f[d.parity]);
    gptr<const T> g = gpc<T>(d.g[d.parity]);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 9 * N; i += gridDim.x * blockDim.x) {
        const int q = i / N, id = i - q * N;
        const int y = id / d.nx, x = id - y * d.nx;
        const int o = q * Np + y * d.pitch + x;
        out[i] = double(f[o]);
        out[9 * N + i] = double(g[o]);
    }
}

}  // namespace tpf
