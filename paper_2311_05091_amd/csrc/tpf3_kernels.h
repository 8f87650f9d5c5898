// Kernels of the three-dimensional coupled step (arXiv 2311.05091, 2f1s model,
// D3Q15, Hermite-moment collision).
//
// step3_kernel: one workgroup of TY wavefronts per (domain, 64 x TY x CZ
// tile).  Lane l of wavefront w owns the column (x0 + l, y0 + w) and the
// workgroup marches the tile's CZ planes in z, plus two halo planes on each
// side.  Iteration r
//   A. pulls the CH populations of plane z0 - 2 + r for the owned columns
//      (kept in a three-deep register ring) and for the xy halo of two
//      columns and rows around the tile, and writes phi0 and phi1 = sum f of
//      the plane into a five-plane LDS ring; it also issues the loads of the
//      NS populations and lagged fields of the plane it will update;
//   B. computes mubar1 (and stages psi = S x u) of the plane below on the
//      tile plus a halo of one (three-plane LDS rings);
//   C. updates the plane two below: stencils from the rings, forces, u, p and
//      the Hermite-space collisions of both lattices from registers.
// Every population of an owned column is read once from memory; the xy halo
// re-reads columns that neighbouring tiles own (through L2).
#pragma once
#include "tpf3_device.h"

namespace tpf3 {

enum { kMode3Step = 0, kMode3Moments = 1 };

template <typename T, int TY, bool HAS_S>
struct Ring3 {
    static constexpr int WX = 68, WY = TY + 4, VX = 66, VY = TY + 2;
    T phi0[5][WY * WX];
    T phi1[5][WY * WX];
    T mub[3][VY * VX];
    T psi[HAS_S ? 3 : 1][HAS_S ? 3 : 1][HAS_S ? VY * VX : 1];   // [slot][component][cell]
};

// Pulled population q at node (x, y, z): f*_q(x - c_q), or across a half-way
// wall the opposite post-collision population of the node itself (Sec. 4).
template <typename T, int q>
__device__ __forceinline__ T pull3(gptr<const T> fin, const DomDev3& d, int x, int y, int z, int64_t N) {
    int xs = x - cx3(q), ys = y - cy3(q), zs = z - cz3(q);
    bool out = false;
    if (d.px) xs = xs < 0 ? xs + d.nx : (xs >= d.nx ? xs - d.nx : xs);
    else out |= (xs < 0 || xs >= d.nx);
    if (d.py) ys = ys < 0 ? ys + d.ny : (ys >= d.ny ? ys - d.ny : ys);
    else out |= (ys < 0 || ys >= d.ny);
    if (d.pz) zs = zs < 0 ? zs + d.nz : (zs >= d.nz ? zs - d.nz : zs);
    else out |= (zs < 0 || zs >= d.nz);
    const int64_t own = ((int64_t)z * d.ny + y) * d.nx + x;
    if (out) return fin[opp3(q) * N + own];
    return fin[q * N + ((int64_t)zs * d.ny + ys) * d.nx + xs];
}

template <typename T>
__device__ __forceinline__ void pull15(gptr<const T> fin, const DomDev3& d, int x, int y, int z, int64_t N,
                                       T (&o)[15]) {
    o[0] = pull3<T, 0>(fin, d, x, y, z, N);
    o[1] = pull3<T, 1>(fin, d, x, y, z, N);
    o[2] = pull3<T, 2>(fin, d, x, y, z, N);
    o[3] = pull3<T, 3>(fin, d, x, y, z, N);
    o[4] = pull3<T, 4>(fin, d, x, y, z, N);
    o[5] = pull3<T, 5>(fin, d, x, y, z, N);
    o[6] = pull3<T, 6>(fin, d, x, y, z, N);
    o[7] = pull3<T, 7>(fin, d, x, y, z, N);
    o[8] = pull3<T, 8>(fin, d, x, y, z, N);
    o[9] = pull3<T, 9>(fin, d, x, y, z, N);
    o[10] = pull3<T, 10>(fin, d, x, y, z, N);
    o[11] = pull3<T, 11>(fin, d, x, y, z, N);
    o[12] = pull3<T, 12>(fin, d, x, y, z, N);
    o[13] = pull3<T, 13>(fin, d, x, y, z, N);
    o[14] = pull3<T, 14>(fin, d, x, y, z, N);
}

// Pulled populations of a node in a row whose y and z are uniform across the
// wavefront and whose x is periodic: the source columns x - 1, x, x + 1 come
// as byte offsets xb (wrapped once per tile), the row part of every address
// is a uniform (scalar) base, and the bounce-back decision of a wall in y or
// z is uniform too.
template <typename T, int q>
__device__ __forceinline__ T pull3_row(gptr<const T> fin, const DomDev3& d, const uint32_t (&xb)[3], int y, int z,
                                       int64_t N) {
    int ys = y - cy3(q), zs = z - cz3(q);
    bool out = false;
    if (d.py) ys = ys < 0 ? ys + d.ny : (ys >= d.ny ? ys - d.ny : ys);
    else out |= (ys < 0 || ys >= d.ny);
    if (d.pz) zs = zs < 0 ? zs + d.nz : (zs >= d.nz ? zs - d.nz : zs);
    else out |= (zs < 0 || zs >= d.nz);
    if (out) return *tpf::at_bytes(fin + (opp3(q) * N + ((int64_t)z * d.ny + y) * d.nx), xb[1]);
    return *tpf::at_bytes(fin + (q * N + ((int64_t)zs * d.ny + ys) * d.nx), xb[1 - cx3(q)]);
}

template <typename T>
__device__ __forceinline__ void pull15_row(gptr<const T> fin, const DomDev3& d, const uint32_t (&xb)[3], int y, int z,
                                           int64_t N, T (&o)[15]) {
    o[0] = pull3_row<T, 0>(fin, d, xb, y, z, N);
    o[1] = pull3_row<T, 1>(fin, d, xb, y, z, N);
    o[2] = pull3_row<T, 2>(fin, d, xb, y, z, N);
    o[3] = pull3_row<T, 3>(fin, d, xb, y, z, N);
    o[4] = pull3_row<T, 4>(fin, d, xb, y, z, N);
    o[5] = pull3_row<T, 5>(fin, d, xb, y, z, N);
    o[6] = pull3_row<T, 6>(fin, d, xb, y, z, N);
    o[7] = pull3_row<T, 7>(fin, d, xb, y, z, N);
    o[8] = pull3_row<T, 8>(fin, d, xb, y, z, N);
    o[9] = pull3_row<T, 9>(fin, d, xb, y, z, N);
    o[10] = pull3_row<T, 10>(fin, d, xb, y, z, N);
    o[11] = pull3_row<T, 11>(fin, d, xb, y, z, N);
    o[12] = pull3_row<T, 12>(fin, d, xb, y, z, N);
    o[13] = pull3_row<T, 13>(fin, d, xb, y, z, N);
    o[14] = pull3_row<T, 14>(fin, d, xb, y, z, N);
}

template <typename T>
__device__ __forceinline__ T sum15(const T (&p)[15]) {
    T s = p[0];
#pragma unroll
    for (int q = 1; q < 15; ++q) s += p[q];
    return s;
}

// Lagged fields of one node (read before the update).
template <typename T>
struct Lag3 {
    T A[3], B, C[6];
};

// Per-node part of the 3D step: forces, u, p and both collisions (Sec. 3, 4).
// dpsi[b][a] = d_a psi_b (the previous step's S x u).
template <typename T, int MODE>
__device__ __forceinline__ void node_update3(const DomDev3& d, const KConst3<T>& K, bool dS, int64_t id, int64_t N,
                                             T ph0, T ph1, const T (&g0)[3], T lap0, const T (&g1)[3], T lap1, T mub,
                                             const T (&gm)[3], const T (&dpsi)[3][3], const T (&fp)[15],
                                             const T (&gq)[15], const Lag3<T>& L, int cur,
                                             double* __restrict__ mom_out) {
    const T c2 = K.c2;
    T mu0, mu1, mu2;
    (void)mubar1_3<T>(K, ph0, ph1, lap0, lap1, mu0, mu1, mu2);
    const T fdeg = ph1 * (T(1) - ph1) * (T(1) - ph0);
    const T a = K.Mdeg_frac * (T(1) - fdeg);
    const T ph2 = T(1) - ph0 - ph1;
    const T rho = K.rho0 * ph0 + K.rho1 * ph1 + K.rho2 * ph2;
    const T muv = K.muv0 * ph0 + K.muv1 * ph1 + K.muv2 * ph2;
    T dr[3], F[3], S[3] = {T(0), T(0), T(0)};
    const T Fb[3] = {K.Fbx, K.Fby, K.Fbz};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        dr[k] = K.drho0 * g0[k] + K.drho1 * g1[k];
        F[k] = mu0 * g0[k] + mu1 * g1[k] - mu2 * (g0[k] + g1[k]) + Fb[k];
    }
    if (dS) {
        const T Mob = K.Mcst + K.Mdeg * fdeg;
#pragma unroll
        for (int k = 0; k < 3; ++k) S[k] = K.Sfac * Mob * gm[k];
        // F_c = -curl(psi)/2
        F[0] += T(-0.5) * (dpsi[2][1] - dpsi[1][2]);
        F[1] += T(-0.5) * (dpsi[0][2] - dpsi[2][0]);
        F[2] += T(-0.5) * (dpsi[1][0] - dpsi[0][1]);
    }
    T mg[15];
    nat_moments15(gq, mg);
    const T inv_rho = fdiv(T(1), rho);
    const T uw[3] = {K.uwx, K.uwy, K.uwz};
    T u[3], fs[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const T us = (mg[1 + k] + T(0.5) * F[k]) * inv_rho;
        fs[k] = uw[k] - us;
        u[k] = us + T(0.5) * ph0 * fs[k];
    }
    const T om = T(1) - ph0;
    const T s2a = fdiv(om, muv * inv_rho * K.inv_cfa + T(0.5) * om);
    const T s2b = fdiv(om, muv * inv_rho * K.inv_cfb + T(0.5) * om);
    const T Q = u[0] * dr[0] + u[1] * dr[1] + u[2] * dr[2];
    const T Bn = (rho * u[0] - S[0]) * u[0] + (rho * u[1] - S[1]) * u[1] + (rho * u[2] - S[2]) * u[2];
    // the s2a term of H is zero where its coefficient is and at a saturated
    // solid node (phi0 = 1 in the working precision, s2a = 0)
    const T H = K.AH - ((d.bh_zero || s2a == T(0)) ? T(0) : fdiv(K.BH, s2a));
    const T p = K.pfac * ((mg[0] - gq[0]) + (T(0.5) + H) * Q - K.pw * Bn + T(0.5) * K.Kp * (Bn - L.B));

    if constexpr (MODE == kMode3Moments) {
        mom_out[id] = double(ph1);
        mom_out[N + id] = double(u[0]);
        mom_out[2 * N + id] = double(u[1]);
        mom_out[3 * N + id] = double(u[2]);
        mom_out[4 * N + id] = double(p);
        return;
    }
    gptr<T> fout = gp<T>(d.f[cur ^ 1]);
    gptr<T> gout = gp<T>(d.g[cur ^ 1]);

    // ---- CH collision in Hermite space ----
    {
        T m[15], h[15];
        nat_moments15(fp, m);
        to_hermite15(m, h, c2);
        const T e = K.eta * mub;
        const T A[3] = {ph1 * u[0], ph1 * u[1], ph1 * u[2]};
        const T s0 = K.s0, s1 = K.s1, s2 = K.s2, s3 = K.s3, s4 = K.s4;
        h[0] -= s0 * (h[0] - ph1);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const T W = (A[k] - L.A[k]) + a * K.eta * c2 * gm[k];
            h[1 + k] += -s1 * (h[1 + k] - A[k]) + (T(1) - T(0.5) * s1) * W;
        }
        const T e4 = c2 * (e - ph1);
        h[4] -= s2 * (h[4] - e4);
        h[5] -= s2 * (h[5] - e4);
        h[6] -= s2 * (h[6] - e4);
        h[7] -= s2 * h[7];
        h[8] -= s2 * h[8];
        h[9] -= s2 * h[9];
        h[10] -= s3 * h[10];
        h[11] -= s3 * h[11];
        h[12] -= s3 * h[12];
        h[13] -= s3 * h[13];
        h[14] -= s4 * (h[14] - T(2) * c2 * c2 * (ph1 - e));
        T fo[15];
        from_hermite15(h, fo, c2);
#pragma unroll
        for (int q = 0; q < 15; ++q) __builtin_nontemporal_store(fo[q], fout + (q * N + id));
        gptr<T> lA = gp<T>(d.lagA);
#pragma unroll
        for (int k = 0; k < 3; ++k) lA[k * N + id] = A[k];
    }

    // ---- NS collision in Hermite space ----
    {
        T G[3], J[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            G[k] = F[k] + ph0 * rho * fs[k];
            J[k] = rho * u[k];
        }
        // momentum flux of g^eq, rho uu - (Su + uS)/2: xx, yy, zz, xy, yz, xz
        const T Pi[6] = {rho * u[0] * u[0] - S[0] * u[0], rho * u[1] * u[1] - S[1] * u[1],
                         rho * u[2] * u[2] - S[2] * u[2],
                         rho * u[0] * u[1] - T(0.5) * (S[0] * u[1] + u[0] * S[1]),
                         rho * u[1] * u[2] - T(0.5) * (S[1] * u[2] + u[1] * S[2]),
                         rho * u[0] * u[2] - T(0.5) * (S[0] * u[2] + u[0] * S[2])};
        const T Cn[6] = {S[0] * u[0], S[1] * u[1], S[2] * u[2], T(0.5) * (S[0] * u[1] + S[1] * u[0]),
                         T(0.5) * (S[1] * u[2] + S[2] * u[1]), T(0.5) * (S[0] * u[2] + S[2] * u[0])};
        // M2F = uF + Fu - d_t C + c_s^2 (u grad rho + grad rho u) + (1 - 3 c_s^2)(u . grad rho) I
        const T q3 = (T(1) - T(3) * c2) * Q;
        constexpr int a1[6] = {0, 1, 2, 0, 1, 0}, a2[6] = {0, 1, 2, 1, 2, 2};
        T M2[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const int i1 = a1[k], i2 = a2[k];
            M2[k] = u[i1] * F[i2] + F[i1] * u[i2] + c2 * (u[i1] * dr[i2] + dr[i1] * u[i2]) + (k < 3 ? q3 : T(0));
            if (dS) M2[k] -= Cn[k] - L.C[k];
        }
        T h[15];
        to_hermite15(mg, h, c2);
        const T gauge = K.gauge;
        const T sg0 = K.sg0, sg1 = K.sg1, sg3 = K.sg3, sg4 = K.sg4;
        h[0] += -sg0 * (h[0] - gauge) + (T(1) - T(0.5) * sg0) * Q;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            h[1 + k] += -sg1 * (h[1 + k] - J[k]) + (T(1) - T(0.5) * sg1) * G[k];
            h[4 + k] += -s2a * (h[4 + k] - (p + Pi[k] - c2 * gauge)) + (T(1) - T(0.5) * s2a) * M2[k];
            h[7 + k] += -s2b * (h[7 + k] - Pi[3 + k]) + (T(1) - T(0.5) * s2b) * M2[3 + k];
        }
        h[10] -= sg3 * h[10];
        h[11] -= sg3 * h[11];
        h[12] -= sg3 * h[12];
        h[13] -= sg3 * h[13];
        h[14] -= sg4 * (h[14] - T(2) * (c2 * c2 * gauge - c2 * p));
        T go[15];
        from_hermite15(h, go, c2);
#pragma unroll
        for (int q = 0; q < 15; ++q) __builtin_nontemporal_store(go[q], gout + (q * N + id));
        gp<T>(d.lagB)[id] = Bn;
        if (dS) {
            gptr<T> lC = gp<T>(d.lagC);
#pragma unroll
            for (int k = 0; k < 6; ++k) lC[k * N + id] = Cn[k];
            gptr<T> ps = gp<T>(d.psi[cur ^ 1]);
            ps[id] = S[1] * u[2] - S[2] * u[1];
            ps[N + id] = S[2] * u[0] - S[0] * u[2];
            ps[2 * N + id] = S[0] * u[1] - S[1] * u[0];
        }
    }
}

// One iteration r of step3_kernel (see the file comment); FL receives the
// populations pulled now, FU holds those pulled two iterations earlier.
template <typename T, int TY, int CZ, bool HAS_S, int MODE>
__device__ __forceinline__ void step3_iter(const DomDev3& d, const KConst3<T>& K, Ring3<T, TY, HAS_S>& sh, int r,
                                           int x0, int y0, int z0, int cur, bool dS, T (&FL)[15], T (&FU)[15],
                                           double* __restrict__ mom_out) {
    using R = Ring3<T, TY, HAS_S>;
    constexpr int WX = R::WX, VX = R::VX, VY = R::VY;
    constexpr int NT = 64 * TY;
    constexpr int NHALO = 4 * WX + 4 * TY;   // two full rows below and above, two columns each side
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    const int64_t N = (int64_t)nx * ny * nz;
    gptr<const T> fin = gpc<T>(d.f[cur]);
    gptr<const T> gin = gpc<T>(d.g[cur]);
    gptr<const T> phi0g = gpc<T>(d.phi0);
    const int tid = threadIdx.x, lane = tid & 63, wy = tid >> 6;
    const int x = x0 + lane, y = y0 + wy;
    const bool owned = x < nx && y < ny;
    // node whose values fill the owned window cell (wrapped or mirrored)
    const int ox = map3(x, nx, d.px), oy = map3(y, ny, d.py);
    const int zr = z0 - 2 + r;
    const int sz = map3(zr, nz, d.pz);
    const int zu = zr - 2;
    const bool upd = owned && r >= 4 && zu < nz;
    const int slot5 = r % 5;

    // ---- A. CH populations and phi of plane zr ----
    // periodic x: the wavefront's row and plane are uniform, so the owned
    // columns take the scalar-base addressing of pull15_row
    uint32_t xb[3] = {0, 0, 0};
    T p0own;
    // loads at the highest wavefront priority (until the NS prefetch is
    // issued), so that a memory-bound wavefront gets its loads out before the
    // others' arithmetic
    __builtin_amdgcn_s_setprio(3);
    if (d.px) {
#pragma unroll
        for (int k = 0; k < 3; ++k) xb[k] = (uint32_t)map3(x - 1 + k, nx, 1) * (uint32_t)sizeof(T);
        pull15_row<T>(fin, d, xb, oy, sz, N, FL);
        p0own = *tpf::at_bytes(phi0g + ((int64_t)sz * ny + oy) * nx, xb[1]);
    } else {
        pull15<T>(fin, d, ox, oy, sz, N, FL);
        p0own = phi0g[((int64_t)sz * ny + oy) * nx + ox];
    }
    // NS populations and lagged fields of the node to update
    T gq[15];
    Lag3<T> L;
    int64_t idu = 0;
    if (upd) {
        if (d.px) pull15_row<T>(gin, d, xb, y, zu, N, gq);
        else pull15<T>(gin, d, x, y, zu, N, gq);
        idu = ((int64_t)zu * ny + y) * nx + x;
        gptr<const T> lA = gpc<T>(d.lagA);
        L.A[0] = lA[idu];
        L.A[1] = lA[N + idu];
        L.A[2] = lA[2 * N + idu];
        L.B = gpc<T>(d.lagB)[idu];
        if (dS) {
            gptr<const T> lC = gpc<T>(d.lagC);
#pragma unroll
            for (int k = 0; k < 6; ++k) L.C[k] = lC[k * N + idu];
        }
    }
    __builtin_amdgcn_s_setprio(0);
    {
        const int i = (wy + 2) * WX + lane + 2;
        sh.phi1[slot5][i] = sum15(FL);
        sh.phi0[slot5][i] = p0own;
    }
    // xy halo: two columns and rows around the tile (general addressing)
    for (int k = tid; k < NHALO; k += NT) {
        int cx, cy;
        if (k < 4 * WX) {
            const int rr = k / WX;
            cy = rr < 2 ? rr : TY + rr;
            cx = k - rr * WX;
        } else {
            const int kk = k - 4 * WX;
            cy = 2 + kk / 4;
            const int s = kk & 3;
            cx = s < 2 ? s : 64 + s;
        }
        const int hx = map3(x0 - 2 + cx, nx, d.px), hy = map3(y0 - 2 + cy, ny, d.py);
        T hf[15];
        pull15<T>(fin, d, hx, hy, sz, N, hf);
        const int i = cy * WX + cx;
        sh.phi1[slot5][i] = sum15(hf);
        sh.phi0[slot5][i] = phi0g[((int64_t)sz * ny + hy) * nx + hx];
    }
    __syncthreads();

    // ---- B. mubar1 (and psi) of plane zr - 1 on the tile + 1 ----
    const int slot3 = r % 3;
    if (r >= 2) {
        const T* pl = sh.phi1[(r + 3) % 5];
        const T* pm = sh.phi1[(r + 4) % 5];
        const T* ph = sh.phi1[slot5];
        const T* ql = sh.phi0[(r + 3) % 5];
        const T* qm = sh.phi0[(r + 4) % 5];
        const T* qh = sh.phi0[slot5];
        const int zb = map3(zr - 1, nz, d.pz);
        for (int c = tid; c < VX * VY; c += NT) {
            const int vy = c / VX, vx = c - vy * VX;
            const int i = (vy + 1) * WX + vx + 1;
            T mu0, mu1, mu2;
            sh.mub[slot3][c] = mubar1_3<T>(K, qm[i], pm[i], lap15(ql, qm, qh, i, WX), lap15(pl, pm, ph, i, WX), mu0,
                                           mu1, mu2);
            if constexpr (HAS_S) {
                if (dS) {
                    const int px_ = map3(x0 - 1 + vx, nx, d.px), py_ = map3(y0 - 1 + vy, ny, d.py);
                    const int64_t ip = ((int64_t)zb * ny + py_) * nx + px_;
                    gptr<const T> ps = gpc<T>(d.psi[cur]);
                    sh.psi[slot3][0][c] = ps[ip];
                    sh.psi[slot3][1][c] = ps[N + ip];
                    sh.psi[slot3][2][c] = ps[2 * N + ip];
                }
            }
        }
    }
    __syncthreads();

    // ---- C. update plane zu ----
    if (upd) {
        const int i = (wy + 2) * WX + lane + 2;
        const int j = (wy + 1) * VX + lane + 1;
        const T* pl = sh.phi1[(r + 2) % 5];
        const T* pm = sh.phi1[(r + 3) % 5];
        const T* ph = sh.phi1[(r + 4) % 5];
        const T* ql = sh.phi0[(r + 2) % 5];
        const T* qm = sh.phi0[(r + 3) % 5];
        const T* qh = sh.phi0[(r + 4) % 5];
        T g0[3], g1[3], gmv[3], lap0, lap1;
        stencil15(ql, qm, qh, i, WX, g0[0], g0[1], g0[2], lap0);
        stencil15(pl, pm, ph, i, WX, g1[0], g1[1], g1[2], lap1);
        grad15(sh.mub[(r + 1) % 3], sh.mub[(r + 2) % 3], sh.mub[slot3], j, VX, gmv[0], gmv[1], gmv[2]);
        T dpsi[3][3] = {{T(0), T(0), T(0)}, {T(0), T(0), T(0)}, {T(0), T(0), T(0)}};
        if constexpr (HAS_S) {
            if (dS) {
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    grad15(sh.psi[(r + 1) % 3][b], sh.psi[(r + 2) % 3][b], sh.psi[slot3][b], j, VX, dpsi[b][0],
                           dpsi[b][1], dpsi[b][2]);
            }
        }
        node_update3<T, MODE>(d, K, dS, idu, N, qm[i], pm[i], g0, lap0, g1, lap1, sh.mub[(r + 2) % 3][j], gmv, dpsi,
                              FU, gq, L, cur, mom_out);
    }
}

template <typename T, int TY, int CZ, bool HAS_S, int MODE>
__global__ void __launch_bounds__(64 * TY)
step3_kernel(const DomDev3* __restrict__ doms, const int4* __restrict__ tiles, int ntiles, int step_offset,
             double* __restrict__ mom_out) {
    __shared__ Ring3<T, TY, HAS_S> sh;
    const int t = tpf::xcd_tile(blockIdx.x, gridDim.x);
    if (t >= ntiles) return;
    const int4 tile = tiles[t];
    const DomDev3& d = doms[tile.x];
    if (!d.live && MODE == kMode3Step) return;
    const KConst3<T> K = kconst3<T>(d);
    const int cur = (d.parity + step_offset) & 1;
    const bool dS = HAS_S && d.has_s;
    T F0[15], F1[15], F2[15];
    // register ring: iteration r pulls into F[r % 3] and updates with F[(r + 1) % 3]
    constexpr int RR = CZ + 4;
    for (int r = 0; r < RR; r += 3) {
        step3_iter<T, TY, CZ, HAS_S, MODE>(d, K, sh, r, tile.y, tile.z, tile.w, cur, dS, F0, F1, mom_out);
        if (r + 1 < RR)
            step3_iter<T, TY, CZ, HAS_S, MODE>(d, K, sh, r + 1, tile.y, tile.z, tile.w, cur, dS, F1, F2, mom_out);
        if (r + 2 < RR)
            step3_iter<T, TY, CZ, HAS_S, MODE>(d, K, sh, r + 2, tile.y, tile.z, tile.w, cur, dS, F2, F0, mom_out);
    }
}

// Initial state: f = f^eq(phi1, eta mubar1, u = 0), g = gauge at rest, lagged 0.
template <typename T>
__global__ void init3_kernel(const DomDev3* __restrict__ doms, int dom, const double* __restrict__ phi1_in) {
    const DomDev3& d = doms[dom];
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    const int64_t N = (int64_t)nx * ny * nz;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= N) return;
    const int x = (int)(id % nx), y = (int)((id / nx) % ny), z = (int)(id / ((int64_t)nx * ny));
    gptr<const T> phi0 = gpc<T>(d.phi0);
    // 3 x 3 x 3 neighbourhoods of phi0 and phi1 (pitch 3, planes of 9)
    T v0[27], v1[27];
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int k = (dz + 1) * 9 + (dy + 1) * 3 + dx + 1;
                const int sx = map3(x + dx, nx, d.px), sy = map3(y + dy, ny, d.py), sz = map3(z + dz, nz, d.pz);
                const int64_t s = ((int64_t)sz * ny + sy) * nx + sx;
                v0[k] = phi0[s];
                v1[k] = T(phi1_in[s]);
            }
    const T lap0 = lap15(v0, v0 + 9, v0 + 18, 4, 3), lap1 = lap15(v1, v1 + 9, v1 + 18, 4, 3);
    const KConst3<T> K = kconst3<T>(d);
    T mu0, mu1, mu2;
    const T e = K.eta * mubar1_3<T>(K, v0[13], v1[13], lap0, lap1, mu0, mu1, mu2);
    const T c2 = K.c2;
    const T w1 = (c2 - c2 * c2) * T(0.5), w7 = c2 * c2 * T(0.125);
    gptr<T> f = gp<T>(d.f[d.parity]);
    gptr<T> g = gp<T>(d.g[d.parity]);
    f[id] = v1[13] + (K.w0 - T(1)) * e;
    for (int q = 1; q <= 6; ++q) f[q * N + id] = w1 * e;
    for (int q = 7; q < 15; ++q) f[q * N + id] = w7 * e;
    g[id] = K.gauge;
    for (int q = 1; q < 15; ++q) g[q * N + id] = T(0);
    for (int k = 0; k < 3; ++k) gp<T>(d.lagA)[k * N + id] = T(0);
    gp<T>(d.lagB)[id] = T(0);
    if (d.has_s) {
        for (int k = 0; k < 6; ++k) gp<T>(d.lagC)[k * N + id] = T(0);
        for (int k = 0; k < 3; ++k) {
            gp<T>(d.psi[0])[k * N + id] = T(0);
            gp<T>(d.psi[1])[k * N + id] = T(0);
        }
    }
}

// Phase mass sum_x phi1 = sum of all post-collision CH populations (streaming
// only permutes them), FP64 with compensated accumulation: per-block partial
// sums, then one block folds them in a fixed order.
template <typename T>
__global__ void __launch_bounds__(256) mass3_partials(const DomDev3* __restrict__ doms, int dom,
                                                      double* __restrict__ part) {
    const DomDev3& d = doms[dom];
    const int64_t n = 15 * (int64_t)d.nx * d.ny * d.nz;
    gptr<const T> f = gpc<T>(d.f[d.parity]);
    double s = 0.0, c = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double v = double(f[i]);
        const double t = s + v;
        c += (fabs(s) >= fabs(v)) ? (s - t) + v : (v - t) + s;
        s = t;
    }
    __shared__ double sh[2][256];
    sh[0][threadIdx.x] = s;
    sh[1][threadIdx.x] = c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const double a = sh[0][threadIdx.x], b = sh[0][threadIdx.x + w];
            const double t = a + b;
            const double e = (fabs(a) >= fabs(b)) ? (a - t) + b : (b - t) + a;
            sh[0][threadIdx.x] = t;
            sh[1][threadIdx.x] += sh[1][threadIdx.x + w] + e;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sh[0][0];
        part[2 * blockIdx.x + 1] = sh[1][0];
    }
}

static __global__ void mass3_final(const double* __restrict__ part, int nblk, double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0, c = 0.0;
    for (int b = 0; b < nblk; ++b) {
        const double v = part[2 * b];
        const double t = s + v;
        c += ((fabs(s) >= fabs(v)) ? (s - t) + v : (v - t) + s) + part[2 * b + 1];
        s = t;
    }
    out[0] = s + c;
}

template <typename T>
__global__ void export3_populations(const DomDev3* __restrict__ doms, int dom, double* __restrict__ out) {
    const DomDev3& d = doms[dom];
    const int64_t n = 15 * (int64_t)d.nx * d.ny * d.nz;
    gptr<const T> f = gpc<T>(d.f[d.parity]);
    gptr<const T> g = gpc<T>(d.g[d.parity]);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        out[i] = double(f[i]);
        out[n + i] = double(g[i]);
    }
}

}  // namespace tpf3
