// Device building blocks of the three-dimensional coupled step (arXiv
// 2311.05091, 2f1s model on the D3Q15 lattice of Appendix A): per-domain
// descriptor, the natural and Hermite moment transforms written out for the
// fifteen velocities, and the isotropic 15-point stencils.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tpf_device.h"

namespace tpf3 {

using tpf::gptr;
using tpf::gp;
using tpf::gpc;
using tpf::fdiv;

// D3Q15 velocities in the order of the columns of M0 (App. A): 0 rest, 1-6
// the axes (+x, -x, +y, -y, +z, -z), 7-14 the cube diagonals with the signs of
// (x, y, z) given by bits 0, 1, 2 of (i - 7) (bit set = negative):
// 7 (+,+,+) 8 (-,+,+) 9 (+,-,+) 10 (-,-,+) 11 (+,+,-) 12 (-,+,-) 13 (+,-,-) 14 (-,-,-).
constexpr int cx3(int q) { return q == 1 ? 1 : q == 2 ? -1 : (q >= 7 ? (((q - 7) & 1) ? -1 : 1) : 0); }
constexpr int cy3(int q) { return q == 3 ? 1 : q == 4 ? -1 : (q >= 7 ? (((q - 7) & 2) ? -1 : 1) : 0); }
constexpr int cz3(int q) { return q == 5 ? 1 : q == 6 ? -1 : (q >= 7 ? (((q - 7) & 4) ? -1 : 1) : 0); }
constexpr int opp3(int q) { return q == 0 ? 0 : (q <= 6 ? (q & 1 ? q + 1 : q - 1) : 7 + (7 ^ (q - 7))); }
static_assert(opp3(1) == 2 && opp3(4) == 3 && opp3(5) == 6 && opp3(7) == 14 && opp3(10) == 11, "opp3");

// Per-domain constants in one precision (derived on the host in FP64).
template <typename T>
struct KConst3 {
    T c2, w0;                     // c_s^2 = d0, omega_0 = 1 - 3 d0 + 2 d0^2
    T gam0, gam1, gam2, gT3, inv_gam0, inv_gam2;
    T c12D, c3D4;
    T eta, Mcst, Mdeg, Mdeg_frac;
    T s0, s1, s2, s3, s4;         // CH rates
    T rho0, rho1, rho2, muv0, muv1, muv2, drho0, drho1, Sfac;
    T sg0, sg1, sg3, sg4;         // NS rates (s2a, s2b per node)
    T inv_cfa, inv_cfb;           // 2/(1 - c_s^2), 1/c_s^2
    T Fbx, Fby, Fbz, uwx, uwy, uwz, gauge;
    T pfac, pw, Kp, AH, BH;       // p = pfac [ sum_{i>0} g_i + (1/2 + H) Q - pw B + Kp/2 dB ],
                                  // H = AH - BH/s2a (3D: AH = K ((1-d0)/s0 + 1 - 3 d0), BH = K (3 - 7 d0))
};

struct DomDev3 {
    int32_t nx, ny, nz, px, py, pz;
    int32_t parity, live, has_s, bh_zero;
    void* f[2];                   // [15][nz][ny][nx]
    void* g[2];
    void* phi0;                   // [nz][ny][nx]
    void* lagA;                   // [3][...] phi1 u
    void* lagB;                   // (rho u - S).u
    void* lagC;                   // [6][...] sym(S u): xx, yy, zz, xy, yz, xz (has_s)
    void* psi[2];                 // [3][...] S x u (has_s, ping-pong)
    KConst3<double> kd;
    KConst3<float> kf;
};

template <typename T>
__device__ __forceinline__ const KConst3<T>& kconst3(const DomDev3& d);
template <>
__device__ __forceinline__ const KConst3<double>& kconst3<double>(const DomDev3& d) { return d.kd; }
template <>
__device__ __forceinline__ const KConst3<float>& kconst3<float>(const DomDev3& d) { return d.kf; }

// Periodic wrap or even mirror across a half-way wall (clamped beyond).
__device__ __forceinline__ int map3(int j, int n, int periodic) { return tpf::map_index(j, n, periodic); }

// Walsh transform of the eight diagonal populations p[7..14]:
// w = (sum, sum sx, sum sy, sum sz, sum sx sy, sum sy sz, sum sx sz, sum sx sy sz)
template <typename T>
__device__ __forceinline__ void walsh8(const T* p, T (&w)[8]) {
    // stage x (bit 0): + for even, - for odd
    T a0 = p[0] + p[1], b0 = p[0] - p[1];
    T a1 = p[2] + p[3], b1 = p[2] - p[3];
    T a2 = p[4] + p[5], b2 = p[4] - p[5];
    T a3 = p[6] + p[7], b3 = p[6] - p[7];
    // stage y (bit 1)
    T c0 = a0 + a1, d0 = a0 - a1, e0 = b0 + b1, f0 = b0 - b1;
    T c1 = a2 + a3, d1 = a2 - a3, e1 = b2 + b3, f1 = b2 - b3;
    // stage z (bit 2)
    w[0] = c0 + c1;   // sum
    w[1] = e0 + e1;   // sx
    w[2] = d0 + d1;   // sy
    w[3] = c0 - c1;   // sz
    w[4] = f0 + f1;   // sx sy
    w[5] = d0 - d1;   // sy sz
    w[6] = e0 - e1;   // sx sz
    w[7] = f0 - f1;   // sx sy sz
}

// Natural moments m = M0 p, rows 1, cx, cy, cz, cx^2, cy^2, cz^2, cx cy,
// cy cz, cx cz, cx cy^2, cy cz^2, cz cx^2, cx cy cz, cx^2 cy^2 cz^2.
template <typename T>
__device__ __forceinline__ void nat_moments15(const T (&p)[15], T (&m)[15]) {
    T w[8];
    walsh8<T>(p + 7, w);
    const T a1 = p[1] + p[2], b1 = p[1] - p[2];
    const T a2 = p[3] + p[4], b2 = p[3] - p[4];
    const T a3 = p[5] + p[6], b3 = p[5] - p[6];
    m[14] = w[0];
    m[10] = w[1];
    m[11] = w[2];
    m[12] = w[3];
    m[7] = w[4];
    m[8] = w[5];
    m[9] = w[6];
    m[13] = w[7];
    m[0] = p[0] + a1 + a2 + a3 + w[0];
    m[1] = b1 + w[1];
    m[2] = b2 + w[2];
    m[3] = b3 + w[3];
    m[4] = a1 + w[0];
    m[5] = a2 + w[0];
    m[6] = a3 + w[0];
}

// h = N_H m (App. A, c = 1).
template <typename T>
__device__ __forceinline__ void to_hermite15(const T (&m)[15], T (&h)[15], T c2) {
#pragma unroll
    for (int k = 0; k < 15; ++k) h[k] = m[k];
    h[4] = m[4] - c2 * m[0];
    h[5] = m[5] - c2 * m[0];
    h[6] = m[6] - c2 * m[0];
    h[10] = m[10] - c2 * m[1];
    h[11] = m[11] - c2 * m[2];
    h[12] = m[12] - c2 * m[3];
    h[14] = m[14] - c2 * (m[4] + m[5] + m[6]) + T(2) * c2 * c2 * m[0];
}

// p = M0^-1 N_H^-1 h.
template <typename T>
__device__ __forceinline__ void from_hermite15(const T (&h)[15], T (&p)[15], T c2) {
    const T m0 = h[0], m1 = h[1], m2 = h[2], m3 = h[3];
    const T m4 = h[4] + c2 * m0, m5 = h[5] + c2 * m0, m6 = h[6] + c2 * m0;
    const T m10 = h[10] + c2 * m1, m11 = h[11] + c2 * m2, m12 = h[12] + c2 * m3;
    const T m14 = h[14] + c2 * (m4 + m5 + m6) - T(2) * c2 * c2 * m0;
    const T m7 = h[7], m8 = h[8], m9 = h[9], m13 = h[13];
    p[0] = m0 - m4 - m5 - m6 + T(2) * m14;
    const T a1 = m4 - m14, b1 = m1 - m10;
    const T a2 = m5 - m14, b2 = m2 - m11;
    const T a3 = m6 - m14, b3 = m3 - m12;
    p[1] = T(0.5) * (a1 + b1);
    p[2] = T(0.5) * (a1 - b1);
    p[3] = T(0.5) * (a2 + b2);
    p[4] = T(0.5) * (a2 - b2);
    p[5] = T(0.5) * (a3 + b3);
    p[6] = T(0.5) * (a3 - b3);
    // inverse Walsh transform of (m14, m10, m11, m12, m7, m8, m9, m13) / 8
    T w[8] = {m14, m10, m11, m12, m7, m8, m9, m13};
    // diagonal d: p = (w0 + sx w1 + sy w2 + sz w3 + sx sy w4 + sy sz w5 + sx sz w6 + sx sy sz w7)/8
    // done as the same three butterfly stages (the transform is its own inverse up to 1/8)
    T q[8];
    // reorder to the natural bit order of walsh8's output: index (bz by bx) -> coefficient
    // coefficient for subset s (bit0 x, bit1 y, bit2 z): s=0 w0, 1 w1, 2 w2, 3 w4, 4 w3, 5 w6, 6 w5, 7 w7
    q[0] = w[0]; q[1] = w[1]; q[2] = w[2]; q[3] = w[4];
    q[4] = w[3]; q[5] = w[6]; q[6] = w[5]; q[7] = w[7];
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        T s = T(0);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            // sign of subset k at diagonal d: product over bits b in k of (-1)^(bit b of d)
            const int par = __builtin_popcount(k & d) & 1;
            s += par ? -q[k] : q[k];
        }
        p[7 + d] = T(0.125) * s;
    }
}

// mu_p (Sec. 2.1) and mubar_1 (Eq. eq-CHmodel)
template <typename T>
__device__ __forceinline__ T chem3(T gam, T c12D, T c3D4, T phi, T lap) {
    return gam * (c12D * phi * (T(1) - phi) * (T(1) - T(2) * phi) - c3D4 * lap);
}

template <typename T>
__device__ __forceinline__ T mubar1_3(const KConst3<T>& K, T phi0, T phi1, T lap0, T lap1, T& mu0, T& mu1,
                                      T& mu2) {
    const T phi2 = T(1) - phi0 - phi1;
    mu0 = chem3(K.gam0, K.c12D, K.c3D4, phi0, lap0);
    mu1 = chem3(K.gam1, K.c12D, K.c3D4, phi1, lap1);
    mu2 = chem3(K.gam2, K.c12D, K.c3D4, phi2, -lap0 - lap1);
    return K.gT3 * ((mu1 - mu0) * K.inv_gam0 + (mu1 - mu2) * K.inv_gam2);
}

// Isotropic 15-point stencils built on the D3Q15 weights at d0 = 1/3
// (1/9 on the axes, 1/72 on the diagonals, c_s^2 = 1/3):
//   grad a = (a_{+a} - a_{-a})/3 + (1/24) sum_diag s_a a_d,
//   lap a  = (2/3) sum_axes a + (1/12) sum_diag a - (14/3) a_0.
// Values come from three planes of a row-major LDS window of pitch W: lo
// (z - 1), mid (z), hi (z + 1) at cell index i.
template <typename T>
__device__ __forceinline__ void stencil15(const T* lo, const T* mid, const T* hi, int i, int W, T& gx, T& gy,
                                          T& gz, T& lap) {
    const T c = mid[i];
    const T xp = mid[i + 1], xm = mid[i - 1], yp = mid[i + W], ym = mid[i - W], zp = hi[i], zm = lo[i];
    // diagonals: z = +1 plane (hi) and z = -1 plane (lo) at (x +- 1, y +- 1)
    const T hpp = hi[i + W + 1], hmp = hi[i + W - 1], hpm = hi[i - W + 1], hmm = hi[i - W - 1];
    const T lpp = lo[i + W + 1], lmp = lo[i + W - 1], lpm = lo[i - W + 1], lmm = lo[i - W - 1];
    const T sx = (hpp - hmp + hpm - hmm) + (lpp - lmp + lpm - lmm);
    const T sy = (hpp + hmp - hpm - hmm) + (lpp + lmp - lpm - lmm);
    const T sz = (hpp + hmp + hpm + hmm) - (lpp + lmp + lpm + lmm);
    const T third = T(1.0 / 3.0), d24 = T(1.0 / 24.0);
    gx = (xp - xm) * third + sx * d24;
    gy = (yp - ym) * third + sy * d24;
    gz = (zp - zm) * third + sz * d24;
    const T axes = xp + xm + yp + ym + zp + zm;
    const T diag = (hpp + hmp + hpm + hmm) + (lpp + lmp + lpm + lmm);
    lap = T(2.0 / 3.0) * axes + T(1.0 / 12.0) * diag - T(14.0 / 3.0) * c;
}

template <typename T>
__device__ __forceinline__ T lap15(const T* lo, const T* mid, const T* hi, int i, int W) {
    const T axes = mid[i + 1] + mid[i - 1] + mid[i + W] + mid[i - W] + hi[i] + lo[i];
    const T diag = (hi[i + W + 1] + hi[i + W - 1] + hi[i - W + 1] + hi[i - W - 1]) +
                   (lo[i + W + 1] + lo[i + W - 1] + lo[i - W + 1] + lo[i - W - 1]);
    return T(2.0 / 3.0) * axes + T(1.0 / 12.0) * diag - T(14.0 / 3.0) * mid[i];
}

template <typename T>
__device__ __forceinline__ void grad15(const T* lo, const T* mid, const T* hi, int i, int W, T& gx, T& gy, T& gz) {
    const T hpp = hi[i + W + 1], hmp = hi[i + W - 1], hpm = hi[i - W + 1], hmm = hi[i - W - 1];
    const T lpp = lo[i + W + 1], lmp = lo[i + W - 1], lpm = lo[i - W + 1], lmm = lo[i - W - 1];
    const T sx = (hpp - hmp + hpm - hmm) + (lpp - lmp + lpm - lmm);
    const T sy = (hpp + hmp - hpm - hmm) + (lpp + lmp - lpm - lmm);
    const T sz = (hpp + hmp + hpm + hmm) - (lpp + lmp + lpm + lmm);
    const T third = T(1.0 / 3.0), d24 = T(1.0 / 24.0);
    gx = (mid[i + 1] - mid[i - 1]) * third + sx * d24;
    gy = (mid[i + W] - mid[i - W]) * third + sy * d24;
    gz = (hi[i] - lo[i]) * third + sz * d24;
}

}  // namespace tpf3
