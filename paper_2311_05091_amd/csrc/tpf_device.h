// Device-side building blocks of the coupled ternary phase-field LB step
// (arXiv 2311.05091): per-domain descriptor, index maps, LDS stencils, the
// D2Q9 natural/Hermite moment transforms and the per-node physics.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tpf {

// Pointers into the arena are stored generically in the descriptor; casting
// them to the global address space lets the compiler emit global (not flat)
// memory instructions, whose completion is tracked apart from LDS traffic.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;

template <typename T>
__device__ __forceinline__ gptr<T> gp(void* p) {
    return (gptr<T>)p;
}

template <typename T>
__device__ __forceinline__ gptr<const T> gpc(const void* p) {
    return (gptr<const T>)p;
}

// Element at a byte offset from a uniform base: with a 32-bit unsigned offset
// the compiler uses the scalar-base + vector-offset addressing form, so
// per-lane addresses cost no 64-bit vector arithmetic.
// The empty asm statement only re-defines the offset register where it is
// used (no instruction), so that the zero extension is formed next to the
// access instead of being hoisted out of the loop, where instruction
// selection could no longer fold it into the addressing mode.
template <typename T>
__device__ __forceinline__ gptr<const T> at_bytes(gptr<const T> base, uint32_t off) {
    asm volatile("" : "+v"(off));
    return (gptr<const T>)((__attribute__((address_space(1))) const char*)base + off);
}

template <typename T>
__device__ __forceinline__ gptr<T> at_bytes(gptr<T> base, uint32_t off) {
    asm volatile("" : "+v"(off));
    return (gptr<T>)((__attribute__((address_space(1))) char*)base + off);
}

// a / b; in FP32 through the hardware reciprocal (about 1 ulp), in FP64 exact.
__device__ __forceinline__ float fdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double fdiv(double a, double b) { return a / b; }

// D2Q9 velocities in the order of the rows of M0 (App. A):
// 0 (0,0) 1 (1,0) 2 (0,1) 3 (-1,0) 4 (0,-1) 5 (1,1) 6 (-1,1) 7 (-1,-1) 8 (1,-1)
__device__ __constant__ const int kCx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ __constant__ const int kCy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ __constant__ const int kOpp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
// the same tables as compile-time functions (for unrolled address arithmetic)
constexpr int cx_of(int q) { return q == 1 || q == 5 || q == 8 ? 1 : (q == 3 || q == 6 || q == 7 ? -1 : 0); }
constexpr int cy_of(int q) { return q == 2 || q == 5 || q == 6 ? 1 : (q == 4 || q == 7 || q == 8 ? -1 : 0); }
constexpr int opp_of(int q) { return q == 0 ? 0 : (q <= 4 ? (q + 1) % 4 + 1 : (q + 1) % 4 + 5); }
static_assert(opp_of(1) == 3 && opp_of(2) == 4 && opp_of(3) == 1 && opp_of(4) == 2, "opp");
static_assert(opp_of(5) == 7 && opp_of(6) == 8 && opp_of(7) == 5 && opp_of(8) == 6, "opp");

// Per-domain constants of the step in one precision (derived on the host in
// FP64, stored once as double and once as float so that kernels read them
// in their own precision without conversions).
template <typename T>
struct KConst {
    T c2, w0;                    // c_s^2 = d0, omega_0
    T gam0, gam1, gam2, gT3;     // gamma_p, gamma^T/3 (Sec. 2.1)
    T inv_gam0, inv_gam2;
    T c12D, c3D4;                // 12/D, 3D/4
    T eta, Mcst, Mdeg, Mdeg_frac;  // Mdeg_frac = M_deg/(M_cst + M_deg)
    T s0, s1, s2, s3, s4;        // CH rates
    T rho0, rho1, rho2, muv0, muv1, muv2;
    T drho0, drho1;              // rho0 - rho2, rho1 - rho2
    T Sfac;                      // (rho1 - rho2)/gamma1
    T sg0, sg1, sg3, sg4;        // NS rates (s2a, s2b per node)
    T inv_cfa, inv_cfb;          // 2/(1 - c_s^2) and 1/c_s^2
    T Fbx, Fby, uwx, uwy, gauge;
    T om, xc, yc;                // solid rotation rate and centre: u_w = (uwx - om (y - yc),
                                 //                                       uwy + om (x - xc))
    T pfac, pw, Kp, AH, BH;      // p = pfac [ sum_{i>0} g_i + (1/2 + H) Q - pw B + Kp/2 dB ],
                                 // H = Kp (AH - BH/s2a)
    T p_in, u_in, p_out, phi1_in;  // open-boundary values (inlet x = 0, outlet x = nx - 1)
};

// Fields an open domain's step stores for the columns x = 1 and x = nx - 2
// (the inner neighbours of the inlet and outlet), for the boundary kernel:
// bnd[side][field][y], side 0 = inlet, 1 = outlet.
enum { kBndPhi1, kBndMub, kBndUx, kBndUy, kBndP, kBndSx, kBndSy, kBndFields };

// Per-domain descriptor in device memory.  Pointers are element pointers of
// the storage precision.
struct DomDev {
    int32_t nx, ny, px, py;      // size and periodicity (1) / walls (0)
    int32_t parity;              // buffer holding the current post-collision state
    int32_t live;                // 1 while the domain is being advanced
    int32_t has_s;               // rho1 != rho2: extra flux S, F_c and C are active
    int32_t bh_zero;             // BH == 0 (d0 = 1/2): H does not depend on s2a
    int32_t open_x, inlet_type;  // open ends in x (inlet 0 pressure / 1 velocity)
    int32_t pitch;               // row stride of every field in elements: nx rounded up to 64,
                                 // so that each strip row starts on a cache-line boundary
    void* f[2];                  // [9][ny][pitch] CH populations (ping-pong)
    void* g[2];                  // [9][ny][nx] NS populations (ping-pong)
    void* phi0;                  // [ny][nx] solid field
    void* lagA;                  // [2][ny][nx] phi1 u of the previous step
    void* lagB;                  // [ny][nx]    (rho u - S).u of the previous step
    void* lagC;                  // [3][ny][nx] sym(S u) of the previous step (has_s)
    void* psi[2];                // [ny][nx]    S_x u_y - S_y u_x (has_s, ping-pong)
    double* snap;                // [ny][nx]    phi1 at the last residual check
    void* bnd;                   // [2][kBndFields][ny] inner-neighbour fields (open_x)
    KConst<double> kd;
    KConst<float> kf;
};

// Control block and per-domain state of a persistent launch.
//   ctl[0] next item, ctl[1] failure flag, ctl[2] domains still live.
//   done[dom]: finished items of dom; retired[dom]: call-relative step at
//   which dom left (-1 while live); last_check[dom]: call-relative step of
//   its last residual check; stats[dom][4]: residual, mass, non-finite count,
//   1 when it left because of non-finite values.
struct PersistArgs {
    const int4* tiles;
    int ntiles;
    const int* live_doms;   // domains of the tile table, in table order
    int nlive;
    int nsteps;             // steps of this launch
    int step_base;          // steps of the call done by earlier launches
    int call_steps;         // steps of the whole call (a check also falls on the last)
    int check_every;        // 0: no residual checks in the launch
    double tol;
    const int* dom_tiles;
    int* ctl;
    int* done;
    int* retired;
    int* last_check;
    double* stats;
    int spin_limit;
};

template <typename T>
__device__ __forceinline__ const KConst<T>& kconst(const DomDev& d);
template <>
__device__ __forceinline__ const KConst<double>& kconst<double>(const DomDev& d) { return d.kd; }
template <>
__device__ __forceinline__ const KConst<float>& kconst<float>(const DomDev& d) { return d.kf; }

// Maps blockIdx.x to a logical tile so that each XCD (blocks are dealt to
// the 8 XCDs round-robin) processes one contiguous band of tiles, whose
// halos then hit in that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int G) {
    int q = G >> 3, r = G & 7;
    int x = b & 7;
    int start = x * q + (x < r ? x : r);
    return start + (b >> 3);
}

// Window cell -> node index.  Periodic axes wrap; across a half-way wall the
// node is the even mirror (-1 -> 0, -2 -> 1, n -> n-1, n+1 -> n-2).  Cells
// farther out only occur in the unused part of a ragged tile's window and
// are clamped so that every access stays inside the domain.
__device__ __forceinline__ int map_index(int j, int n, int periodic) {
    if (periodic) {
        if ((unsigned)j >= (unsigned)n) {
            j %= n;
            if (j < 0) j += n;
        }
        return j;
    }
    if (j < 0) j = -1 - j;
    else if (j >= n) j = 2 * n - 1 - j;
    return j < 0 ? 0 : (j >= n ? n - 1 : j);
}

// Pull-streamed population q at node (x, y): f*_q(x - c_q), or the opposite
// post-collision population of the node itself across a wall (half-way
// bounce-back, Sec. 4).
template <typename T>
__device__ __forceinline__ T pull(gptr<const T> fin, int q, int x, int y, int nx, int ny,
                                  int px, int py, int N, int ld) {
    int xs = x - kCx[q], ys = y - kCy[q];
    bool out = false;
    if (px) { xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs); }
    else if (xs < 0 || xs >= nx) out = true;
    if (py) { ys = ys < 0 ? ys + ny : (ys >= ny ? ys - ny : ys); }
    else if (ys < 0 || ys >= ny) out = true;
    if (out) return fin[kOpp[q] * N + y * ld + x];
    return fin[q * N + ys * ld + xs];
}

// Isotropic 9-point central gradient and Laplacian on a row-major LDS tile.
template <typename T>
__device__ __forceinline__ void stencil9(const T* s, int i, int W, T& gx, T& gy, T& lap) {
    T C = s[i], E = s[i + 1], Wv = s[i - 1], Nn = s[i + W], Ss = s[i - W];
    T NE = s[i + W + 1], NW = s[i + W - 1], SE = s[i - W + 1], SW = s[i - W - 1];
    gx = (T(4) * (E - Wv) + (NE - NW + SE - SW)) * T(1.0 / 12.0);
    gy = (T(4) * (Nn - Ss) + (NE - SE + NW - SW)) * T(1.0 / 12.0);
    lap = (T(4) * (E + Wv + Nn + Ss) + (NE + NW + SE + SW) - T(20) * C) * T(1.0 / 6.0);
}

template <typename T>
__device__ __forceinline__ void grad9(const T* s, int i, int W, T& gx, T& gy) {
    T E = s[i + 1], Wv = s[i - 1], Nn = s[i + W], Ss = s[i - W];
    T NE = s[i + W + 1], NW = s[i + W - 1], SE = s[i - W + 1], SW = s[i - W - 1];
    gx = (T(4) * (E - Wv) + (NE - NW + SE - SW)) * T(1.0 / 12.0);
    gy = (T(4) * (Nn - Ss) + (NE - SE + NW - SW)) * T(1.0 / 12.0);
}

template <typename T>
__device__ __forceinline__ T lap9(const T* s, int i, int W) {
    T C = s[i], E = s[i + 1], Wv = s[i - 1], Nn = s[i + W], Ss = s[i - W];
    T NE = s[i + W + 1], NW = s[i + W - 1], SE = s[i - W + 1], SW = s[i - W - 1];
    return (T(4) * (E + Wv + Nn + Ss) + (NE + NW + SE + SW) - T(20) * C) * T(1.0 / 6.0);
}

// mu_p = gamma_p [ (12/D) phi (1-phi)(1-2phi) - (3D/4) lap(phi) ]   (Sec. 2.1)
template <typename T>
__device__ __forceinline__ T chem(T gam, T c12D, T c3D4, T phi, T lap) {
    return gam * (c12D * phi * (T(1) - phi) * (T(1) - T(2) * phi) - c3D4 * lap);
}

// mubar_1 = (gamma^T/3) [ (mu1 - mu0)/gamma0 + (mu1 - mu2)/gamma2 ]  (Eq. eq-CHmodel)
template <typename T>
__device__ __forceinline__ T mubar1(const KConst<T>& K, T phi0, T phi1, T lap0, T lap1, T& mu0,
                                    T& mu1, T& mu2) {
    T phi2 = T(1) - phi0 - phi1;
    mu0 = chem(K.gam0, K.c12D, K.c3D4, phi0, lap0);
    mu1 = chem(K.gam1, K.c12D, K.c3D4, phi1, lap1);
    mu2 = chem(K.gam2, K.c12D, K.c3D4, phi2, -lap0 - lap1);
    return K.gT3 * ((mu1 - mu0) * K.inv_gam0 + (mu1 - mu2) * K.inv_gam2);
}

// Natural moments m = M0 p (rows 1, cx, cy, cx^2, cy^2, cxcy, cxcy^2, cx^2cy, cx^2cy^2).
template <typename T>
__device__ __forceinline__ void nat_moments(const T p[9], T m[9]) {
    T a = p[5] + p[7], b = p[6] + p[8];
    T c = p[5] - p[7], e = p[6] - p[8];
    m[8] = a + b;
    m[0] = p[0] + p[1] + p[2] + p[3] + p[4] + m[8];
    m[1] = p[1] - p[3] + c - e;
    m[2] = p[2] - p[4] + c + e;
    m[3] = p[1] + p[3] + m[8];
    m[4] = p[2] + p[4] + m[8];
    m[5] = a - b;
    m[6] = c - e;
    m[7] = c + e;
}

// Hermite moments h = N m (App. A, c = 1).
template <typename T>
__device__ __forceinline__ void to_hermite(const T m[9], T h[9], T c2) {
    h[0] = m[0];
    h[1] = m[1];
    h[2] = m[2];
    h[3] = m[3] - c2 * m[0];
    h[4] = m[4] - c2 * m[0];
    h[5] = m[5];
    h[6] = m[6] - c2 * m[1];
    h[7] = m[7] - c2 * m[2];
    h[8] = m[8] - c2 * (m[3] + m[4]) + c2 * c2 * m[0];
}

// Populations from Hermite moments: p = M0^-1 N^-1 h.
template <typename T>
__device__ __forceinline__ void from_hermite(const T h[9], T p[9], T c2) {
    T m0 = h[0], m1 = h[1], m2 = h[2];
    T m3 = h[3] + c2 * h[0];
    T m4 = h[4] + c2 * h[0];
    T m5 = h[5];
    T m6 = h[6] + c2 * h[1];
    T m7 = h[7] + c2 * h[2];
    T m8 = h[8] + c2 * (m3 + m4) - c2 * c2 * m0;
    p[0] = m0 - m3 - m4 + m8;
    T a = m3 - m8, b = m1 - m6;
    p[1] = T(0.5) * (a + b);
    p[3] = T(0.5) * (a - b);
    T c = m4 - m8, e = m2 - m7;
    p[2] = T(0.5) * (c + e);
    p[4] = T(0.5) * (c - e);
    p[5] = T(0.25) * (m8 + m5 + m6 + m7);
    p[6] = T(0.25) * (m8 - m5 - m6 + m7);
    p[7] = T(0.25) * (m8 + m5 - m6 - m7);
    p[8] = T(0.25) * (m8 - m5 + m6 - m7);
}

}  // namespace tpf
