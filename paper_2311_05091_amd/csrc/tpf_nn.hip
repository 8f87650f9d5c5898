// Kernels of the learned warm start (see include/tpf_nn.h): implicit-GEMM
// 3x3 convolutions on the gfx950 BF16 matrix cores (v_mfma_f32_16x16x32_bf16,
// FP32 accumulation), their weight and input gradients, and the elementwise
// pieces of a small encoder-decoder (pooling, upsampling, concatenation,
// output head with the cross-entropy loss, Adam).
//
// Matrix-core operand layout (one wavefront, 16x16x32): lane l holds
//   A: row l%16, k = 8*(l/16) .. 8*(l/16)+7      (8 bf16)
//   B: col l%16, k = 8*(l/16) .. 8*(l/16)+7      (8 bf16)
//   D: col l%16, rows 4*(l/16) .. 4*(l/16)+3      (4 fp32)
// tpfnn_mfma_selftest checks it against a host product.
#include <hip/hip_runtime.h>

#include <cmath>

#include <cstddef>
#include <cstdint>
#include <mutex>

#include "tpf_nn.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kOk = 0, kEinval = -1, kEdevice = -2;

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
    u += 0x7fffu + ((u >> 16) & 1u);                      // round to nearest even
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

inline int launch_status() { return hipGetLastError() == hipSuccess ? kOk : kEdevice; }

// ---------------------------------------------------------------------------
// matrix-core layout self-test
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) mfma_selftest_k(const uint16_t* A, const uint16_t* B, float* D) {
    const int l = threadIdx.x;
    uint16_t a[8], b[8];
    for (int e = 0; e < 8; ++e) {
        a[e] = A[(l % 16) * 32 + 8 * (l / 16) + e];   // A[row][k], 16 x 32 row-major
        b[e] = B[(8 * (l / 16) + e) * 16 + (l % 16)];  // B[k][col], 32 x 16 row-major
    }
    bf16x8 av = as_bf16x8(*(uint4*)a), bv = as_bf16x8(*(uint4*)b);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
    for (int i = 0; i < 4; ++i) D[(4 * (l / 16) + i) * 16 + (l % 16)] = acc[i];
}

// ---------------------------------------------------------------------------
// 3x3 convolution, forward (also the input gradient with flipped weights)
// GEMM: M = pixels (64 per block), N = output channels (BN per block),
// K = 9 * Cin in chunks of 32 channels of one tap.
// ---------------------------------------------------------------------------
template <int BN, int KC>
__global__ void __launch_bounds__(256)
conv3x3_fwd_k(const uint16_t* __restrict__ x, int H, int W, int Cin, const uint16_t* __restrict__ w,
              const float* __restrict__ bias, int Cout, int relu, uint16_t* __restrict__ y) {
    // KC input channels staged per barrier pair (32 or 64; Cin a multiple of
    // KC), row pitch KC + 8 halfwords so that the 16 rows an MFMA operand
    // reads fall in distinct LDS banks
    static_assert(KC == 32 || KC == 64, "KC is 32 or 64");
    constexpr int KP = KC + 8;
    constexpr int SEGS = KC / 32;   // 16-byte loads per thread and row quarter
    __shared__ __attribute__((aligned(16))) uint16_t As[64][KP];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[BN][KP];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int p0 = blockIdx.x * 64;
    const int co0 = blockIdx.y * BN;
    const int HW = H * W;
    // loader roles: thread tid stages row tid / 4 at channel offsets
    // (tid % 4) * 8 + 32 k, k < SEGS
    const int ar = tid >> 2, aseg = (tid & 3) * 8;
    const int p = p0 + ar;
    const int n = p / HW, rem = p - n * HW;
    const int py = rem / W, px = rem - py * W;
    const bool bload = tid < BN * 4;
    const int bco = co0 + (tid >> 2), bseg = (tid & 3) * 8;

    f32x4 acc[BN / 16];
#pragma unroll
    for (int j = 0; j < BN / 16; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int kk = 0; kk < 9; ++kk) {
        const int sy = py + kk / 3 - 1, sx = px + kk % 3 - 1;
        const bool inb = (sy >= 0) && (sy < H) && (sx >= 0) && (sx < W);
        const uint16_t* xr = x + ((size_t)(n * H + (inb ? sy : 0)) * W + (inb ? sx : 0)) * Cin;
        const uint16_t* wr = w + ((size_t)bco * 9 + kk) * Cin;
        for (int ci0 = 0; ci0 < Cin; ci0 += KC) {
            uint4 av[SEGS], bv[SEGS];
#pragma unroll
            for (int k = 0; k < SEGS; ++k) {
                av[k] = inb ? *(const uint4*)(xr + ci0 + aseg + 32 * k) : make_uint4(0, 0, 0, 0);
                bv[k] = bload ? *(const uint4*)(wr + ci0 + bseg + 32 * k) : make_uint4(0, 0, 0, 0);
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < SEGS; ++k) {
                *(uint4*)&As[ar][aseg + 32 * k] = av[k];
                if (bload) *(uint4*)&Bs[tid >> 2][bseg + 32 * k] = bv[k];
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < SEGS; ++k) {
                const bf16x8 a = as_bf16x8(*(const uint4*)&As[16 * wave + (lane & 15)][32 * k + (lane >> 4) * 8]);
#pragma unroll
                for (int j = 0; j < BN / 16; ++j) {
                    const bf16x8 b = as_bf16x8(*(const uint4*)&Bs[16 * j + (lane & 15)][32 * k + (lane >> 4) * 8]);
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[j], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < BN / 16; ++j) {
        const int co = co0 + 16 * j + (lane & 15);
        const float bb = bias ? bias[co] : 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = 16 * wave + 4 * (lane >> 4) + i;
            float v = acc[j][i] + bb;
            if (relu) v = v > 0.f ? v : 0.f;
            y[(size_t)(p0 + row) * Cout + co] = f2bf(v);
        }
    }
}

// ---------------------------------------------------------------------------
// 3x3 convolution, forward, for wide layers (Cout a multiple of 128, Cin of
// 32).  A block computes BM pixels x 128 output channels with 2 x 2
// wavefronts of (BM / 2) x 64 outputs each (BM / 32 x 4 MFMA tiles of
// 16 x 16).  The K loop runs over 9 taps x Cin / 32 channel chunks; each step
// stages 32 channels of BM pixels and of 128 output channels in one of two
// LDS buffers: the next step's global loads are issued before the current
// step's MFMAs and stored into the other buffer after them, so a step needs
// one barrier.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// 3x3 convolution, forward, staging input patches (Cout a multiple of 64, Cin
// of 32; W a multiple of 128 or a divisor of 128 of at least 16).  A block
// of 2 PXB threads computes PXB output pixels (R = PXB / WB image rows of
// WB = min(W, 128) columns) x 64 output channels; its PXB / 64 x 2
// wavefronts compute 64 x 32 outputs each.  For each chunk of 32 input
// channels it stages in LDS the input patch of those pixels (R + 2 rows of
// WB + 2 columns, zero outside the image) and the 64 x 9 weights, and then
// runs all nine taps on them: each tap's A operand is the patch shifted by
// (ky, kx).  The next chunk's global loads are in flight (in registers) while
// the current chunk is computed.  With one LDS buffer (NB = 1) a chunk costs
// two barriers; 256-pixel blocks whose two buffers fit in the 160 KB of a
// compute unit (NB = 2) store the next chunk into the other buffer and need
// one.
// ---------------------------------------------------------------------------
constexpr int kPatchCo = 64;
constexpr int kPatchKP = 40;   // LDS row pitch in halfwords (32 channels + padding): the 16 rows of an operand in distinct banks

template <int WB, int PXB>
struct PatchCfg {
    static constexpr int NTH = 2 * PXB;                  // threads per block
    static constexpr int R = PXB / WB;                   // image rows per block
    static constexpr int PC = WB + 2;                    // patch columns
    static constexpr int PIX = (R + 2) * PC;             // patch pixels
    static constexpr int PL = (PIX * 4 + NTH - 1) / NTH;             // 16-byte patch loads per thread
    static constexpr int WROWS = kPatchCo * 9;                        // (tap, co) weight rows
    static constexpr int WL = (WROWS * 4 + NTH - 1) / NTH;           // 16-byte weight loads per thread
};

// One input-channel chunk of the patch kernel in registers: PL patch pixels
// and WL weight rows of 16 bytes per thread.
template <int PL, int WL>
struct PatchRegs {
    uint4 p[PL];
    uint4 w[WL];
};

// Global loads of the chunk ci0 .. ci0 + 31 (patch pixels read as zero where
// pval is false).  Weight row i = (tap, co) with co fastest, so that the LDS
// store spreads consecutive rows over distinct banks; rows past the last
// (when the thread count does not divide them) read row 0 and are not stored.
template <typename C>
__device__ __forceinline__ PatchRegs<C::PL, C::WL> patch_load(const uint16_t* __restrict__ x,
                                                              const uint16_t* __restrict__ w, int Cin, int co0, int tid,
                                                              int seg, const int (&poff)[C::PL],
                                                              const bool (&pval)[C::PL], int ci0) {
    PatchRegs<C::PL, C::WL> g;
#pragma unroll
    for (int k = 0; k < C::PL; ++k) {
        const uint4 v = *(const uint4*)(x + (size_t)poff[k] * Cin + ci0 + seg);
        g.p[k] = pval[k] ? v : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int k = 0; k < C::WL; ++k) {
        int i = (tid + C::NTH * k) >> 2;
        if (i >= C::WROWS) i = 0;
        const int kk = i / kPatchCo, co = i - kk * kPatchCo;
        g.w[k] = *(const uint4*)(w + ((size_t)(co0 + co) * 9 + kk) * Cin + ci0 + seg);
    }
    return g;
}

template <typename C>
__device__ __forceinline__ void patch_store(uint16_t (*Ps)[kPatchKP], uint16_t (*Ws)[kPatchCo][kPatchKP], int tid,
                                            int seg, const PatchRegs<C::PL, C::WL>& g) {
#pragma unroll
    for (int k = 0; k < C::PL; ++k) {
        const int i = (tid + C::NTH * k) >> 2;
        if (i < C::PIX) *(uint4*)&Ps[i][seg] = g.p[k];
    }
#pragma unroll
    for (int k = 0; k < C::WL; ++k) {
        const int i = (tid + C::NTH * k) >> 2;
        const int kk = i / kPatchCo, co = i - kk * kPatchCo;
        if (i < C::WROWS) *(uint4*)&Ws[kk][co][seg] = g.w[k];
    }
}

template <int WB, int PXB, int NB>
__global__ void __launch_bounds__(2 * PXB)
conv3x3_fwd_patch_k(const uint16_t* __restrict__ x, int H, int W, int Cin, const uint16_t* __restrict__ w,
                    const float* __restrict__ bias, int Cout, int relu, uint16_t* __restrict__ y) {
    using C = PatchCfg<WB, PXB>;
    // NB = 2: two LDS buffers (a chunk's operands are stored into the other
    // buffer while the current one is read; one barrier per chunk)
    __shared__ __attribute__((aligned(16))) uint16_t Ps[NB][C::PIX][kPatchKP];
    __shared__ __attribute__((aligned(16))) uint16_t Ws[NB][9][kPatchCo][kPatchKP];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wm = wave >> 1, wn = wave & 1;
    // block -> (image, first row, first column) of its R x WB output pixels
    const int segs = W / WB, bands = H / C::R;
    int t = blockIdx.x;
    const int n = t / (bands * segs);
    t -= n * bands * segs;
    const int y0 = (t / segs) * C::R, x0 = (t % segs) * WB;
    const int co0 = blockIdx.y * kPatchCo;
    const int seg = (tid & 3) * 8;
    // patch loads: item i = tid + NTH k -> patch pixel i >> 2, segment seg;
    // items past the patch or pixels outside the image load the first pixel
    // and are replaced by zero
    int poff[C::PL];
    bool pval[C::PL];
#pragma unroll
    for (int k = 0; k < C::PL; ++k) {
        const int i = (tid + C::NTH * k) >> 2;
        const int pr = i / C::PC, pc = i - pr * C::PC;
        const int sy = y0 - 1 + pr, sx = x0 - 1 + pc;
        pval[k] = i < C::PIX && sy >= 0 && sy < H && sx >= 0 && sx < W;
        poff[k] = pval[k] ? ((n * H + sy) * W + sx) : 0;
    }
    PatchRegs<C::PL, C::WL> g;
    const int nchunk = Cin / 32;
    // a wavefront's 4 pixel fragments of 16 (rows of the output region) and
    // their patch positions
    int frag_base[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const int q = wm * 64 + 16 * f + (lane & 15);
        const int rr = q / WB, cc = q - rr * WB;
        frag_base[f] = rr * C::PC + cc;
    }
    f32x4 acc[4][2];
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[f][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#define PATCH_COMPUTE(B_)                                                                    \
    _Pragma("unroll") for (int kk = 0; kk < 9; ++kk) {                                       \
        const int sh = (kk / 3) * C::PC + (kk % 3);                                          \
        bf16x8 a[4], b[2];                                                                   \
        _Pragma("unroll") for (int f = 0; f < 4; ++f)                                        \
            a[f] = as_bf16x8(*(const uint4*)&Ps[B_][frag_base[f] + sh][(lane >> 4) * 8]);    \
        _Pragma("unroll") for (int j = 0; j < 2; ++j)                                        \
            b[j] = as_bf16x8(*(const uint4*)&Ws[B_][kk][wn * 32 + 16 * j + (lane & 15)][(lane >> 4) * 8]); \
        _Pragma("unroll") for (int f = 0; f < 4; ++f)                                        \
            _Pragma("unroll") for (int j = 0; j < 2; ++j)                                    \
                acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[f], b[j], acc[f][j], 0, 0, 0); \
    }
    g = patch_load<C>(x, w, Cin, co0, tid, seg, poff, pval, 0);
    patch_store<C>(Ps[0], Ws[0], tid, seg, g);
    __syncthreads();
    for (int c = 0; c < nchunk - 1; ++c) {
        g = patch_load<C>(x, w, Cin, co0, tid, seg, poff, pval, (c + 1) * 32);   // in flight during the nine taps
        if constexpr (NB == 2) {
            PATCH_COMPUTE(c & 1)
            // the other buffer was last read in chunk c - 1, before the
            // barrier that ended it
            patch_store<C>(Ps[(c + 1) & 1], Ws[(c + 1) & 1], tid, seg, g);
            __syncthreads();
        } else {
            PATCH_COMPUTE(0)
            __syncthreads();    // every wavefront is done with the chunk in LDS
            patch_store<C>(Ps[0], Ws[0], tid, seg, g);
            __syncthreads();
        }
    }
    PATCH_COMPUTE(NB == 2 ? ((nchunk - 1) & 1) : 0)
#undef PATCH_COMPUTE
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int co = co0 + wn * 32 + 16 * j + (lane & 15);
        const float bb = bias ? bias[co] : 0.f;
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int q = wm * 64 + 16 * f + 4 * (lane >> 4) + e;
                const int rr = q / WB, cc = q - rr * WB;
                float v = acc[f][j][e] + bb;
                if (relu) v = v > 0.f ? v : 0.f;
                y[((size_t)(n * H + y0 + rr) * W + x0 + cc) * Cout + co] = f2bf(v);
            }
    }
}

__global__ void weight_flip_k(const uint16_t* __restrict__ w, int Cout, int Cin, uint16_t* __restrict__ wt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)Cout * 9 * Cin;
    if (i >= total) return;
    // wt[ci][ky][kx][co] = w[co][2-ky][2-kx][ci]
    const int co = (int)(i % Cout);
    const int64_t r = i / Cout;
    const int kk = (int)(r % 9);
    const int ci = (int)(r / 9);
    wt[i] = w[((int64_t)co * 9 + (8 - kk)) * Cin + ci];
}

// ---------------------------------------------------------------------------
// 3x3 convolution, weight gradient (split over pixels, fixed-order reduction)
// GEMM per tap: M = output channels (BM per block), N = 32 input channels,
// K = pixels in chunks of 32.
// ---------------------------------------------------------------------------
template <int BM>
__global__ void __launch_bounds__(256)
conv3x3_wgrad_k(const uint16_t* __restrict__ x, const uint16_t* __restrict__ dy, int H, int W, int Cin,
                int Cout, int P, int chunk, float* __restrict__ part) {
    __shared__ __attribute__((aligned(16))) uint16_t As[BM][40];  // [co][pixel]
    __shared__ __attribute__((aligned(16))) uint16_t Bs[32][40];  // [ci][pixel]
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int co0 = blockIdx.x * BM;
    const int ncb = Cin / 32;
    const int kk = blockIdx.y / ncb, ci0 = (blockIdx.y % ncb) * 32;
    const int dyk = kk / 3 - 1, dxk = kk % 3 - 1;
    const int HW = H * W;
    const int pbeg = blockIdx.z * chunk;
    const int pend = min(P, pbeg + chunk);
    // tiles: (BM/16) row groups of 16 channels x 2 column groups of 16 ci,
    // spread over the 4 waves (each wave owns NCW column groups of one row group)
    constexpr int RG = BM / 16, WPR = 4 / RG, NCW = 2 / WPR;
    const int tr = wave % RG;
    f32x4 acc[NCW];
#pragma unroll
    for (int k = 0; k < NCW; ++k) acc[k] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int pc = pbeg; pc < pend; pc += 32) {
        // dy[p][co0 .. co0+BM) for 32 pixels: BM*32*2 bytes, 16 B per thread
        uint4 av = make_uint4(0, 0, 0, 0);
        const int apix = tid / (BM / 8), aseg = (tid % (BM / 8)) * 8;
        const bool aload = tid < 32 * (BM / 8);
        if (aload && pc + apix < pend) av = *(const uint4*)(dy + (size_t)(pc + apix) * Cout + co0 + aseg);
        // x[p + tap][ci0 .. ci0+32) for 32 pixels
        uint4 bv = make_uint4(0, 0, 0, 0);
        const int bpix = tid >> 2, bseg = (tid & 3) * 8;
        if (tid < 128 && pc + bpix < pend) {
            const int p = pc + bpix;
            const int n = p / HW, rem = p - n * HW;
            const int sy = rem / W + dyk, sx = rem % W + dxk;
            if (sy >= 0 && sy < H && sx >= 0 && sx < W)
                bv = *(const uint4*)(x + ((size_t)(n * H + sy) * W + sx) * Cin + ci0 + bseg);
        }
        __syncthreads();
        if (aload) {
            const uint16_t* e = (const uint16_t*)&av;
#pragma unroll
            for (int j = 0; j < 8; ++j) As[aseg + j][apix] = e[j];
        }
        if (tid < 128) {
            const uint16_t* e = (const uint16_t*)&bv;
#pragma unroll
            for (int j = 0; j < 8; ++j) Bs[bseg + j][bpix] = e[j];
        }
        __syncthreads();
        const bf16x8 a = as_bf16x8(*(const uint4*)&As[16 * tr + (lane & 15)][(lane >> 4) * 8]);
#pragma unroll
        for (int k = 0; k < NCW; ++k) {
            const int tc = wave / RG + k * WPR;
            const bf16x8 b = as_bf16x8(*(const uint4*)&Bs[16 * tc + (lane & 15)][(lane >> 4) * 8]);
            acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[k], 0, 0, 0);
        }
    }
    float* out = part + (size_t)blockIdx.z * Cout * 9 * Cin;
#pragma unroll
    for (int k = 0; k < NCW; ++k) {
        const int tc = wave / RG + k * WPR;
        const int ci = ci0 + 16 * tc + (lane & 15);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int co = co0 + 16 * tr + 4 * (lane >> 4) + i;
            out[((size_t)co * 9 + kk) * Cin + ci] = acc[k][i];
        }
    }
}

// ---------------------------------------------------------------------------
// 3x3 convolution, weight gradient with all nine taps per block.
// The pixels are walked in segments of 32 consecutive pixels of one image
// row.  Per segment a block stages dy (32 pixels x BM output channels) and
// the input patch around it (3 rows x 34 pixels x 32 input channels) in LDS,
// both transposed to pixel-fastest order; the patch is stored three times,
// shifted by one column each, so that every tap's operand is an aligned
// 16-byte LDS read.  Each dy fragment then feeds 9 (taps) x 2 (ci groups)
// MFMA tiles.  Splits over segments give partial sums, added later in a
// fixed order.  Requires W % 32 == 0.
// ---------------------------------------------------------------------------
template <int BM>
__global__ void __launch_bounds__(256)
conv3x3_wgrad9_k(const uint16_t* __restrict__ x, const uint16_t* __restrict__ dy, int H, int W, int Cin,
                 int Cout, int nseg, int segs_per_split, float* __restrict__ part) {
    __shared__ __attribute__((aligned(16))) uint16_t As[BM][40];        // [co][px]
    __shared__ __attribute__((aligned(16))) uint16_t Bs[3][32][3][40];  // [column shift][ci][row][px]
    constexpr int CG = BM / 16;          // output-channel groups of 16
    constexpr int TPW = CG * 2 * 9 / 4;  // MFMA tiles per wave: 18 (BM = 64) or 9 (BM = 32)
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int co0 = blockIdx.x * BM, ci0 = blockIdx.y * 32;
    const int s0 = blockIdx.z * segs_per_split, s1 = min(nseg, s0 + segs_per_split);
    const int segs_row = W / 32;
    // wave -> (output-channel group, first ci group)
    const int cg = BM == 64 ? wave : (wave & 1);
    const int gg = BM == 64 ? 0 : (wave >> 1);
    f32x4 acc[TPW];
#pragma unroll
    for (int k = 0; k < TPW; ++k) acc[k] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int sg = s0; sg < s1; ++sg) {
        const int n = sg / (H * segs_row);
        const int rr = sg - n * H * segs_row;
        const int yy = rr / segs_row, xs0 = (rr - yy * segs_row) * 32;
        // dy tile: thread -> (pixel, 8 output channels)
        constexpr int TPP = BM / 8;
        const bool aload = tid < 32 * TPP;
        const int apx = tid / TPP, aseg = (tid % TPP) * 8;
        uint4 av = make_uint4(0, 0, 0, 0);
        if (aload)
            av = *(const uint4*)(dy + ((size_t)(n * H + yy) * W + xs0 + apx) * Cout + co0 + aseg);
        // input patch: 3 rows x 34 columns x 4 groups of 8 channels = 408 items
        uint4 bv[2];
        int bit[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int it = tid + 256 * k;
            bit[k] = it;
            bv[k] = make_uint4(0, 0, 0, 0);
            if (it < 408) {
                const int r = it / 136, rem = it - r * 136;
                const int c = rem >> 2, q = rem & 3;
                const int sy = yy - 1 + r, sx = xs0 - 1 + c;
                if (sy >= 0 && sy < H && sx >= 0 && sx < W)
                    bv[k] = *(const uint4*)(x + ((size_t)(n * H + sy) * W + sx) * Cin + ci0 + 8 * q);
            }
        }
        __syncthreads();
        if (aload) {
            const uint16_t* e = (const uint16_t*)&av;
#pragma unroll
            for (int j = 0; j < 8; ++j) As[aseg + j][apx] = e[j];
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int it = bit[k];
            if (it < 408) {
                const int r = it / 136, rem = it - r * 136;
                const int c = rem >> 2, q = rem & 3;
                const uint16_t* e = (const uint16_t*)&bv[k];
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    const int px = c - dx;
                    if (px >= 0 && px < 32) {
#pragma unroll
                        for (int j = 0; j < 8; ++j) Bs[dx][8 * q + j][r][px] = e[j];
                    }
                }
            }
        }
        __syncthreads();
        const bf16x8 a = as_bf16x8(*(const uint4*)&As[16 * cg + (lane & 15)][(lane >> 4) * 8]);
#pragma unroll
        for (int k = 0; k < TPW; ++k) {
            // tile k -> (tap, ci group)
            const int g = BM == 64 ? (k / 9) : gg;
            const int tap = BM == 64 ? (k % 9) : k;
            const int ky = tap / 3, kx = tap % 3;
            const bf16x8 b = as_bf16x8(*(const uint4*)&Bs[kx][16 * g + (lane & 15)][ky][(lane >> 4) * 8]);
            acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[k], 0, 0, 0);
        }
    }
    float* out = part + (size_t)blockIdx.z * Cout * 9 * Cin;
#pragma unroll
    for (int k = 0; k < TPW; ++k) {
        const int g = BM == 64 ? (k / 9) : gg;
        const int tap = BM == 64 ? (k % 9) : k;
        const int ci = ci0 + 16 * g + (lane & 15);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int co = co0 + 16 * cg + 4 * (lane >> 4) + i;
            out[((size_t)co * 9 + tap) * Cin + ci] = acc[k][i];
        }
    }
}

// out[i] = sum over k of part[k][i].  A block covers 64 outputs with four
// waves, wave g adding splits g, g + 4, g + 8, ...; the four partial sums
// are then added in order g = 0..3 (fixed order, deterministic).
__global__ void __launch_bounds__(256)
sum_splits_k(const float* __restrict__ part, int splits, int64_t n, float* __restrict__ out) {
    __shared__ float red[4][64];
    const int o = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * 64 + o;
    float s = 0.f;
    if (i < n) {
#pragma unroll 8
        for (int k = g; k < splits; k += 4) s += part[(size_t)k * n + i];
    }
    red[g][o] = s;
    __syncthreads();
    if (g == 0 && i < n) out[i] = ((red[0][o] + red[1][o]) + red[2][o]) + red[3][o];
}

// db partials: block b sums pixels [b*kBiasPix, (b+1)*kBiasPix) for every
// channel.  A thread reads 8 consecutive channels (16 bytes) of every
// G-th pixel, G = 256/(C/8), so a wave reads whole pixel rows (coalesced);
// the G partial sums of a channel are then added in a fixed order.
// C is a multiple of 8 that divides 256.
constexpr int kBiasPix = 1024;

__global__ void __launch_bounds__(256)
bias_grad_part_k(const uint16_t* __restrict__ dy, int P, int C, float* __restrict__ part) {
    __shared__ float red[256][8];
    const int tpp = C / 8, G = 256 / tpp;
    const int c8 = threadIdx.x % tpp, pl = threadIdx.x / tpp;
    const int pbeg = blockIdx.x * kBiasPix, pend = min(P, pbeg + kBiasPix);
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int p = pbeg + pl; p < pend; p += G) {
        const uint4 v = *(const uint4*)(dy + (size_t)p * C + 8 * c8);
        const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            s[2 * j] += bf2f((uint16_t)(u[j] & 0xffffu));
            s[2 * j + 1] += bf2f((uint16_t)(u[j] >> 16));
        }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) red[threadIdx.x][j] = s[j];
    __syncthreads();
    if (threadIdx.x < C) {
        const int cc = threadIdx.x / 8, j = threadIdx.x % 8;
        float t = 0.f;
        for (int g = 0; g < G; ++g) t += red[g * tpp + cc][j];
        part[(size_t)blockIdx.x * C + threadIdx.x] = t;
    }
}

// ---------------------------------------------------------------------------
// elementwise kernels
// ---------------------------------------------------------------------------
__global__ void relu_bwd_k(const uint16_t* __restrict__ y, uint16_t* __restrict__ dy, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !(bf2f(y[i]) > 0.f)) dy[i] = 0;
}

__global__ void avgpool2_fwd_k(const uint16_t* __restrict__ x, int N, int H, int W, int C,
                               uint16_t* __restrict__ y) {
    const int Ho = H / 2, Wo = W / 2;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)N * Ho * Wo * C) return;
    const int c = (int)(i % C);
    int64_t r = i / C;
    const int xo = (int)(r % Wo);
    r /= Wo;
    const int yo = (int)(r % Ho);
    const int n = (int)(r / Ho);
    const size_t b = ((size_t)(n * H + 2 * yo) * W + 2 * xo) * C + c;
    const float s = bf2f(x[b]) + bf2f(x[b + C]) + bf2f(x[b + (size_t)W * C]) + bf2f(x[b + (size_t)W * C + C]);
    y[i] = f2bf(0.25f * s);
}

__global__ void avgpool2_bwd_k(const uint16_t* __restrict__ dy, int N, int H, int W, int C,
                               uint16_t* __restrict__ dx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)N * H * W * C) return;
    const int c = (int)(i % C);
    int64_t r = i / C;
    const int xx = (int)(r % W);
    r /= W;
    const int yy = (int)(r % H);
    const int n = (int)(r / H);
    const int Ho = H / 2, Wo = W / 2;
    dx[i] = f2bf(0.25f * bf2f(dy[((size_t)(n * Ho + yy / 2) * Wo + xx / 2) * C + c]));
}

__global__ void upsample2_fwd_k(const uint16_t* __restrict__ x, int N, int H, int W, int C,
                                uint16_t* __restrict__ y) {
    const int Ho = 2 * H, Wo = 2 * W;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)N * Ho * Wo * C) return;
    const int c = (int)(i % C);
    int64_t r = i / C;
    const int xo = (int)(r % Wo);
    r /= Wo;
    const int yo = (int)(r % Ho);
    const int n = (int)(r / Ho);
    y[i] = x[((size_t)(n * H + yo / 2) * W + xo / 2) * C + c];
}

__global__ void upsample2_bwd_k(const uint16_t* __restrict__ dy, int N, int H, int W, int C,
                                uint16_t* __restrict__ dx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)N * H * W * C) return;
    const int c = (int)(i % C);
    int64_t r = i / C;
    const int xx = (int)(r % W);
    r /= W;
    const int yy = (int)(r % H);
    const int n = (int)(r / H);
    const int Wo = 2 * W;
    const size_t b = ((size_t)(n * 2 * H + 2 * yy) * Wo + 2 * xx) * C + c;
    const float s = bf2f(dy[b]) + bf2f(dy[b + C]) + bf2f(dy[b + (size_t)Wo * C]) +
                    bf2f(dy[b + (size_t)Wo * C + C]);
    dx[i] = f2bf(s);
}

// 16-byte (8-channel) versions of the copies and masks above, used when the
// channel counts are multiples of 8.
__global__ void relu_bwd_v8_k(const uint4* __restrict__ y, uint4* __restrict__ dy, int64_t n8) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n8) return;
    const uint4 yv = y[i];
    uint4 g = dy[i];
    const uint32_t ys[4] = {yv.x, yv.y, yv.z, yv.w};
    uint32_t gs[4] = {g.x, g.y, g.z, g.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (!(bf2f((uint16_t)(ys[j] & 0xffffu)) > 0.f)) gs[j] &= 0xffff0000u;
        if (!(bf2f((uint16_t)(ys[j] >> 16)) > 0.f)) gs[j] &= 0x0000ffffu;
    }
    dy[i] = make_uint4(gs[0], gs[1], gs[2], gs[3]);
}

__global__ void upsample2_fwd_v8_k(const uint4* __restrict__ x, int N, int H, int W, int C8,
                                   uint4* __restrict__ y) {
    const int Ho = 2 * H, Wo = 2 * W;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)N * Ho * Wo * C8) return;
    const int c = (int)(i % C8);
    int64_t r = i / C8;
    const int xo = (int)(r % Wo);
    r /= Wo;
    const int yo = (int)(r % Ho);
    const int n = (int)(r / Ho);
    y[i] = x[((size_t)(n * H + yo / 2) * W + xo / 2) * C8 + c];
}

__global__ void concat_v8_k(const uint4* __restrict__ a, int Ca8, const uint4* __restrict__ b, int Cb8,
                            int64_t npix, uint4* __restrict__ y) {
    const int C8 = Ca8 + Cb8;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npix * C8) return;
    const int64_t p = i / C8;
    const int c = (int)(i % C8);
    y[i] = c < Ca8 ? a[p * Ca8 + c] : b[p * Cb8 + (c - Ca8)];
}

__global__ void split_v8_k(const uint4* __restrict__ dy, int Ca8, int Cb8, int64_t npix, uint4* __restrict__ da,
                           uint4* __restrict__ db) {
    const int C8 = Ca8 + Cb8;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npix * C8) return;
    const int64_t p = i / C8;
    const int c = (int)(i % C8);
    if (c < Ca8) da[p * Ca8 + c] = dy[i];
    else db[p * Cb8 + (c - Ca8)] = dy[i];
}

__global__ void concat_k(const uint16_t* __restrict__ a, int Ca, const uint16_t* __restrict__ b, int Cb,
                         int64_t npix, uint16_t* __restrict__ y) {
    const int C = Ca + Cb;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npix * C) return;
    const int64_t p = i / C;
    const int c = (int)(i % C);
    y[i] = c < Ca ? a[p * Ca + c] : b[p * Cb + (c - Ca)];
}

__global__ void split_k(const uint16_t* __restrict__ dy, int Ca, int Cb, int64_t npix,
                        uint16_t* __restrict__ da, uint16_t* __restrict__ db) {
    const int C = Ca + Cb;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npix * C) return;
    const int64_t p = i / C;
    const int c = (int)(i % C);
    if (c < Ca) da[p * Ca + c] = dy[i];
    else db[p * Cb + (c - Ca)] = dy[i];
}

__global__ void add_inplace_k(uint16_t* __restrict__ a, const uint16_t* __restrict__ b, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = f2bf(bf2f(a[i]) + bf2f(b[i]));
}

// Output head, one thread per pixel; per-block partial sums of dw, db, loss.
constexpr int kHeadThreads = 256;

__global__ void __launch_bounds__(kHeadThreads)
head_k(const uint16_t* __restrict__ x, int64_t npix, int C, const float* __restrict__ w,
       const float* __restrict__ b, float* __restrict__ pred, const float* __restrict__ target,
       uint16_t* __restrict__ dx, double* __restrict__ part) {
    __shared__ double red[kHeadThreads / 64][34];
    const int64_t p = (int64_t)blockIdx.x * kHeadThreads + threadIdx.x;
    const bool ok = p < npix;
    float xv[32];
    float z = b[0];
    for (int c = 0; c < C; ++c) {
        xv[c] = ok ? bf2f(x[p * C + c]) : 0.f;
        z += w[c] * xv[c];
    }
    const float pr = 1.f / (1.f + __expf(-z));
    if (ok) pred[p] = pr;
    if (!target) return;
    const float tg = ok ? target[p] : 0.f;
    const float dz = ok ? (pr - tg) / (float)npix : 0.f;
    // binary cross-entropy with logits: softplus(z) - t z, softplus in the
    // overflow-free form max(z, 0) + log(1 + exp(-|z|))
    const float bce = ok ? fmaxf(z, 0.f) + log1pf(__expf(-fabsf(z))) - tg * z : 0.f;
    if (ok)
        for (int c = 0; c < C; ++c) dx[p * C + c] = f2bf(dz * w[c]);
    // C + 2 block sums (dw[0..C), db, loss): a shuffle tree per wave, then the
    // four wave sums in order (fixed order throughout, so deterministic)
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    for (int k = 0; k < C + 2; ++k) {
        double v = k < C ? (double)(dz * xv[k]) : (k == C ? (double)dz : (double)bce);
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
        if (ln == 0) red[wv][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < C + 2) {
        double t = 0.0;
        for (int i = 0; i < kHeadThreads / 64; ++i) t += red[i][threadIdx.x];
        part[(size_t)blockIdx.x * (C + 2) + threadIdx.x] = t;
    }
}

// One block per output k: strided partial sums per thread, then a tree.
__global__ void __launch_bounds__(256)
head_final_k(const double* __restrict__ part, int nblk, int C, int64_t npix, float* __restrict__ dw,
             float* __restrict__ db, double* __restrict__ loss) {
    __shared__ double red[256];
    const int k = blockIdx.x;
    double s = 0.0;
    for (int i = threadIdx.x; i < nblk; i += 256) s += part[(size_t)i * (C + 2) + k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (k < C) dw[k] = (float)red[0];
        else if (k == C) db[0] = (float)red[0];
        else loss[0] = red[0] / (double)npix;
    }
}

__global__ void adam_k(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, uint16_t* __restrict__ pb, int64_t n, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    if (pb) pb[i] = f2bf(pi);
}

__global__ void to_bf16_k(const float* __restrict__ x, uint16_t* __restrict__ y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

__global__ void from_bf16_k(const uint16_t* __restrict__ x, float* __restrict__ y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = bf2f(x[i]);
}

__global__ void resample_k(const float* __restrict__ src, int N, int sh, int sw, float* __restrict__ dst,
                           int dh, int dw) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)N * dh * dw) return;
    const int x = (int)(i % dw);
    const int64_t r = i / dw;
    const int y = (int)(r % dh);
    const int n = (int)(r / dh);
    const float fy = dh > 1 ? (float)y * (float)(sh - 1) / (float)(dh - 1) : 0.f;
    const float fx = dw > 1 ? (float)x * (float)(sw - 1) / (float)(dw - 1) : 0.f;
    int y0 = (int)fy, x0 = (int)fx;
    y0 = min(max(y0, 0), sh - 1);
    x0 = min(max(x0, 0), sw - 1);
    const int y1 = min(y0 + 1, sh - 1), x1 = min(x0 + 1, sw - 1);
    const float ty = fy - (float)y0, tx = fx - (float)x0;
    const float* s = src + (size_t)n * sh * sw;
    const float v = (1.f - ty) * ((1.f - tx) * s[(size_t)y0 * sw + x0] + tx * s[(size_t)y0 * sw + x1]) +
                    ty * ((1.f - tx) * s[(size_t)y1 * sw + x0] + tx * s[(size_t)y1 * sw + x1]);
    dst[i] = v;
}

// Mass projection of a predicted phase field by a shift of its logit:
// phi1 = sigmoid(logit(p) + c) (1 - phi0), with the c that gives
// sum(phi1) = the target (the sum is increasing in c): Newton steps on the
// sum, kept inside a bisection bracket (a step that would leave it bisects
// instead).  One block; FP32 sigmoid, FP64 sums in a fixed order, so the
// result is deterministic.
constexpr int kProjThreads = 1024;
constexpr float kProjClip = 1e-7f;
constexpr float kProjRange = 40.f;

__device__ __forceinline__ float proj_logit(float p) {
    p = fminf(fmaxf(p, kProjClip), 1.f - kProjClip);
    return logf(p) - log1pf(-p);
}

__device__ double block_sum_1024(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < kProjThreads / 64; ++i) t += red[i];
    return t;
}

// Block b projects field b of a batch of equal-size fields: pred, phi0 and
// out advance by n per field, info by 2; its mass is targets[b] (target0
// when targets is null, a single field).
__global__ void __launch_bounds__(kProjThreads)
mass_project_k(const float* __restrict__ pred_all, const float* __restrict__ phi0_all, int64_t n,
               const double* __restrict__ targets, double target0, double* __restrict__ out_all,
               double* __restrict__ info_all) {
    __shared__ double red[kProjThreads / 64];
    const int64_t b = blockIdx.x;
    const float* __restrict__ pred = pred_all + b * n;
    const float* __restrict__ phi0 = phi0_all + b * n;
    double* __restrict__ out = out_all + b * n;
    double* __restrict__ info = info_all + 2 * b;
    const double target = targets ? targets[b] : target0;
    // sum of phi1 at shift c and its derivative in c
    auto mass = [&](float c, double* dmass) {
        double acc = 0.0, dacc = 0.0;
        for (int64_t i = threadIdx.x; i < n; i += kProjThreads) {
            const float z = proj_logit(pred[i]) + c;
            const float sg = 1.f / (1.f + __expf(-z));
            const float w = 1.f - phi0[i];
            acc += (double)(w * sg);
            if (dmass) dacc += (double)(w * sg * (1.f - sg));
        }
        const double m = block_sum_1024(acc, red);
        if (dmass) *dmass = block_sum_1024(dacc, red);
        return m;
    };
    const double m_lo = mass(-kProjRange, nullptr), m_hi = mass(kProjRange, nullptr);
    if (!(target > m_lo && target < m_hi)) {
        for (int64_t i = threadIdx.x; i < n; i += kProjThreads) out[i] = 0.0;
        if (threadIdx.x == 0) info[0] = info[1] = __builtin_nan("");
        return;
    }
    float lo = -kProjRange, hi = kProjRange, c = 0.f;
    for (int it = 0; it < 48; ++it) {
        double dm = 0.0;
        const double m = mass(c, &dm);
        if (fabs(m - target) <= 1e-9 * target) break;
        if (m < target) lo = c;
        else hi = c;
        float cn = (float)((double)c + (target - m) / dm);
        if (!(dm > 0.0) || !(cn > lo && cn < hi)) cn = 0.5f * (lo + hi);
        if (cn == c || lo >= hi) break;
        c = cn;
    }
    const double m = mass(c, nullptr);
    const double scale = target / m;  // removes the last residue of the root search
    for (int64_t i = threadIdx.x; i < n; i += kProjThreads) {
        // the same FP32 expression as in mass(), so that the FP64 sum of the
        // output is target to rounding
        const float z = proj_logit(pred[i]) + c;
        const float sg = 1.f / (1.f + __expf(-z));
        out[i] = (double)((1.f - phi0[i]) * sg) * scale;
    }
    if (threadIdx.x == 0) {
        info[0] = c;
        info[1] = m;
    }
}

__global__ void pack_input_k(const float* __restrict__ phi0, const float* __restrict__ phi1,
                             const float* __restrict__ theta, const float* __restrict__ vol, int N, int HW,
                             uint16_t* __restrict__ x) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (int64_t)N * HW) return;
    const int n = (int)(p / HW);
    uint16_t* o = x + p * 32;
    o[0] = f2bf(phi0[p]);
    o[1] = f2bf((theta[n] - 90.f) / 60.f);
    o[2] = f2bf(vol[n]);
    o[3] = phi1 ? f2bf(phi1[p]) : (uint16_t)0;
    for (int c = 4; c < 32; ++c) o[c] = 0;
}

inline dim3 grid1(int64_t n, int t = 256) { return dim3((unsigned)((n + t - 1) / t)); }

int wgrad_splits(int64_t P) {
    int64_t s = P / 4096;
    if (s < 1) s = 1;
    if (s > 64) s = 64;
    return (int)s;
}

// Segments (32 pixels of one row) per split of the nine-tap weight gradient:
// about 2048 blocks in all, at least 16 segments per block.
int wgrad9_segs_per_split(int64_t nseg, int Cin, int Cout) {
    const int bm = Cout % 64 == 0 ? 64 : 32;
    const int64_t nxy = (int64_t)(Cout / bm) * (Cin / 32);
    int64_t splits = (2048 + nxy - 1) / nxy;
    if (splits > 512) splits = 512;  // bounds the partial sums the reduction reads
    const int64_t max_splits = nseg / 16 > 0 ? nseg / 16 : 1;
    if (splits > max_splits) splits = max_splits;
    if (splits < 1) splits = 1;
    return (int)((nseg + splits - 1) / splits);
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" int tpfnn_mfma_selftest(const uint16_t* A, const uint16_t* B, float* D, void* stream) {
    if (!A || !B || !D) return kEinval;
    hipLaunchKernelGGL(mfma_selftest_k, dim3(1), dim3(64), 0, (hipStream_t)stream, A, B, D);
    return launch_status();
}

extern "C" int tpfnn_conv3x3_fwd(const uint16_t* x, int32_t N, int32_t H, int32_t W, int32_t Cin,
                                 const uint16_t* w, const float* bias, int32_t Cout, int32_t relu,
                                 uint16_t* y, void* stream) {
    if (!x || !w || !y || N <= 0 || H <= 0 || W <= 0) return kEinval;
    if (Cin % 32 || Cout % 32 || ((int64_t)H * W) % 64) return kEinval;
    const int64_t P = (int64_t)N * H * W;
    if (P / 64 > 0x7fffffff) return kEinval;
    {
        // patch-staging kernel: W a multiple of 128, or a divisor of 128 of
        // at least 16; 256 pixels per block where that still gives a block
        // per compute unit (and H holds the rows), else 128
        const int wb = W % 128 == 0 ? 128 : W;
        const bool shape = (W % 128 == 0 || (128 % W == 0 && W >= 16)) && H % (128 / wb) == 0;
        if (shape && Cout % 64 == 0) {
            const int64_t t256 = H % (256 / wb) == 0 ? (int64_t)N * (H / (256 / wb)) * (W / wb) : 0;
            const bool big = t256 * (Cout / 64) >= 256;
            const int pxb = big ? 256 : 128;
            const dim3 g((unsigned)((int64_t)N * (H / (pxb / wb)) * (W / wb)), Cout / 64);
            hipStream_t st = (hipStream_t)stream;
#define PATCH_LAUNCH(WBV, PXV, NBV)                                                             \
    hipLaunchKernelGGL((conv3x3_fwd_patch_k<WBV, PXV, NBV>), g, dim3(2 * PXV), 0, st, x, H, W, Cin, w, bias, \
                       Cout, relu, y)
            // 256-pixel blocks (one per compute unit) double-buffer their LDS
            // where two buffers fit in 160 KB (not for 128-column rows)
            if (big) {
                switch (wb) {
                    case 128: PATCH_LAUNCH(128, 256, 1); break;
                    case 64: PATCH_LAUNCH(64, 256, 2); break;
                    case 32: PATCH_LAUNCH(32, 256, 2); break;
                    default: PATCH_LAUNCH(16, 256, 2); break;
                }
            } else {
                switch (wb) {
                    case 128: PATCH_LAUNCH(128, 128, 1); break;
                    case 64: PATCH_LAUNCH(64, 128, 1); break;
                    case 32: PATCH_LAUNCH(32, 128, 1); break;
                    default: PATCH_LAUNCH(16, 128, 1); break;
                }
            }
#undef PATCH_LAUNCH
            return launch_status();
        }
    }
    // 64 input channels per barrier pair where Cin allows it, else 32
    const bool k64 = Cin % 64 == 0;
    if (Cout % 64 == 0) {
        dim3 g((unsigned)(P / 64), Cout / 64);
        if (k64)
            hipLaunchKernelGGL((conv3x3_fwd_k<64, 64>), g, dim3(256), 0, (hipStream_t)stream, x, H, W, Cin, w,
                               bias, Cout, relu, y);
        else
            hipLaunchKernelGGL((conv3x3_fwd_k<64, 32>), g, dim3(256), 0, (hipStream_t)stream, x, H, W, Cin, w,
                               bias, Cout, relu, y);
    } else {
        dim3 g((unsigned)(P / 64), Cout / 32);
        if (k64)
            hipLaunchKernelGGL((conv3x3_fwd_k<32, 64>), g, dim3(256), 0, (hipStream_t)stream, x, H, W, Cin, w,
                               bias, Cout, relu, y);
        else
            hipLaunchKernelGGL((conv3x3_fwd_k<32, 32>), g, dim3(256), 0, (hipStream_t)stream, x, H, W, Cin, w,
                               bias, Cout, relu, y);
    }
    return launch_status();
}

extern "C" int tpfnn_weight_flip(const uint16_t* w, int32_t Cout, int32_t Cin, uint16_t* wt, void* stream) {
    if (!w || !wt || Cout <= 0 || Cin <= 0) return kEinval;
    const int64_t n = (int64_t)Cout * 9 * Cin;
    hipLaunchKernelGGL(weight_flip_k, grid1(n), dim3(256), 0, (hipStream_t)stream, w, Cout, Cin, wt);
    return launch_status();
}

extern "C" size_t tpfnn_wgrad_workspace(int32_t N, int32_t H, int32_t W, int32_t Cin, int32_t Cout) {
    const int64_t P = (int64_t)N * H * W;
    size_t nb;
    if (W % 32 == 0 && Cin > 0 && Cout > 0) {
        const int64_t nseg = P / 32;
        const int sps = wgrad9_segs_per_split(nseg, Cin, Cout);
        nb = (size_t)((nseg + sps - 1) / sps);
    } else {
        const int S = wgrad_splits(P);
        const int chunk = (int)((P + S - 1) / S + 31) / 32 * 32;
        nb = (size_t)((P + chunk - 1) / chunk);
    }
    const size_t wpart = nb * Cout * 9 * Cin * sizeof(float);
    const size_t bpart = (size_t)((P + kBiasPix - 1) / kBiasPix) * Cout * sizeof(float);
    return wpart + bpart + 256;
}

extern "C" int tpfnn_conv3x3_wgrad(const uint16_t* x, const uint16_t* dy, int32_t N, int32_t H, int32_t W,
                                   int32_t Cin, int32_t Cout, float* dw, float* db, void* work,
                                   size_t work_bytes, void* stream) {
    if (!x || !dy || !dw || !work || N <= 0 || H <= 0 || W <= 0) return kEinval;
    if (Cin % 32 || Cout % 32 || ((int64_t)H * W) % 64) return kEinval;
    if (work_bytes < tpfnn_wgrad_workspace(N, H, W, Cin, Cout)) return kEinval;
    if (db && 256 % Cout) return kEinval;
    const int64_t P = (int64_t)N * H * W;
    if (P > 0x7fffffff) return kEinval;
    float* wpart = (float*)work;
    hipStream_t st = (hipStream_t)stream;
    const int ncb = Cin / 32;
    int nb;
    if (W % 32 == 0) {
        const int64_t nseg = P / 32;
        const int sps = wgrad9_segs_per_split(nseg, Cin, Cout);
        nb = (int)((nseg + sps - 1) / sps);
        if (Cout % 64 == 0) {
            dim3 g(Cout / 64, ncb, nb);
            hipLaunchKernelGGL(conv3x3_wgrad9_k<64>, g, dim3(256), 0, st, x, dy, H, W, Cin, Cout, (int)nseg, sps,
                               wpart);
        } else {
            dim3 g(Cout / 32, ncb, nb);
            hipLaunchKernelGGL(conv3x3_wgrad9_k<32>, g, dim3(256), 0, st, x, dy, H, W, Cin, Cout, (int)nseg, sps,
                               wpart);
        }
    } else {
        const int S = wgrad_splits(P);
        const int chunk = (int)((P + S - 1) / S + 31) / 32 * 32;
        nb = (int)((P + chunk - 1) / chunk);
        if (Cout % 64 == 0) {
            dim3 g(Cout / 64, 9 * ncb, nb);
            hipLaunchKernelGGL(conv3x3_wgrad_k<64>, g, dim3(256), 0, st, x, dy, H, W, Cin, Cout, (int)P, chunk,
                               wpart);
        } else {
            dim3 g(Cout / 32, 9 * ncb, nb);
            hipLaunchKernelGGL(conv3x3_wgrad_k<32>, g, dim3(256), 0, st, x, dy, H, W, Cin, Cout, (int)P, chunk,
                               wpart);
        }
    }
    float* bpart = wpart + (size_t)nb * Cout * 9 * Cin;
    if (hipGetLastError() != hipSuccess) return kEdevice;
    const int64_t nw = (int64_t)Cout * 9 * Cin;
    hipLaunchKernelGGL(sum_splits_k, dim3((unsigned)((nw + 63) / 64)), dim3(256), 0, st, wpart, nb, nw, dw);
    if (hipGetLastError() != hipSuccess) return kEdevice;
    if (db) {
        const int nbb = (int)((P + kBiasPix - 1) / kBiasPix);
        hipLaunchKernelGGL(bias_grad_part_k, dim3(nbb), dim3(256), 0, st, dy, (int)P, Cout, bpart);
        if (hipGetLastError() != hipSuccess) return kEdevice;
        hipLaunchKernelGGL(sum_splits_k, dim3((unsigned)((Cout + 63) / 64)), dim3(256), 0, st, bpart, nbb,
                           (int64_t)Cout, db);
    }
    return launch_status();
}

extern "C" int tpfnn_relu_bwd(const uint16_t* y, uint16_t* dy, int64_t n, void* stream) {
    if (!y || !dy || n < 0) return kEinval;
    if (n == 0) return kOk;
    if (n % 8 == 0 && ((uintptr_t)y | (uintptr_t)dy) % 16 == 0) {
        hipLaunchKernelGGL(relu_bwd_v8_k, grid1(n / 8), dim3(256), 0, (hipStream_t)stream, (const uint4*)y,
                           (uint4*)dy, n / 8);
        return launch_status();
    }
    hipLaunchKernelGGL(relu_bwd_k, grid1(n), dim3(256), 0, (hipStream_t)stream, y, dy, n);
    return launch_status();
}

extern "C" int tpfnn_avgpool2_fwd(const uint16_t* x, int32_t N, int32_t H, int32_t W, int32_t C, uint16_t* y,
                                  void* stream) {
    if (!x || !y || H % 2 || W % 2 || N <= 0 || C <= 0) return kEinval;
    const int64_t n = (int64_t)N * (H / 2) * (W / 2) * C;
    hipLaunchKernelGGL(avgpool2_fwd_k, grid1(n), dim3(256), 0, (hipStream_t)stream, x, N, H, W, C, y);
    return launch_status();
}

extern "C" int tpfnn_avgpool2_bwd(const uint16_t* dy, int32_t N, int32_t H, int32_t W, int32_t C, uint16_t* dx,
                                  void* stream) {
    if (!dy || !dx || H % 2 || W % 2 || N <= 0 || C <= 0) return kEinval;
    const int64_t n = (int64_t)N * H * W * C;
    hipLaunchKernelGGL(avgpool2_bwd_k, grid1(n), dim3(256), 0, (hipStream_t)stream, dy, N, H, W, C, dx);
    return launch_status();
}

extern "C" int tpfnn_upsample2_fwd(const uint16_t* x, int32_t N, int32_t H, int32_t W, int32_t C, uint16_t* y,
                                   void* stream) {
    if (!x || !y || N <= 0 || H <= 0 || W <= 0 || C <= 0) return kEinval;
    const int64_t n = (int64_t)N * 4 * H * W * C;
    if (C % 8 == 0 && ((uintptr_t)x | (uintptr_t)y) % 16 == 0) {
        hipLaunchKernelGGL(upsample2_fwd_v8_k, grid1(n / 8), dim3(256), 0, (hipStream_t)stream, (const uint4*)x, N,
                           H, W, C / 8, (uint4*)y);
        return launch_status();
    }
    hipLaunchKernelGGL(upsample2_fwd_k, grid1(n), dim3(256), 0, (hipStream_t)stream, x, N, H, W, C, y);
    return launch_status();
}

extern "C" int tpfnn_upsample2_bwd(const uint16_t* dy, int32_t N, int32_t H, int32_t W, int32_t C, uint16_t* dx,
                                   void* stream) {
    if (!dy || !dx || N <= 0 || H <= 0 || W <= 0 || C <= 0) return kEinval;
    const int64_t n = (int64_t)N * H * W * C;
    hipLaunchKernelGGL(upsample2_bwd_k, grid1(n), dim3(256), 0, (hipStream_t)stream, dy, N, H, W, C, dx);
    return launch_status();
}

extern "C" int tpfnn_concat(const uint16_t* a, int32_t Ca, const uint16_t* b, int32_t Cb, int64_t npix,
                            uint16_t* y, void* stream) {
    if (!a || !b || !y || Ca <= 0 || Cb <= 0 || npix <= 0) return kEinval;
    const int64_t n = npix * (Ca + Cb);
    if (Ca % 8 == 0 && Cb % 8 == 0 && ((uintptr_t)a | (uintptr_t)b | (uintptr_t)y) % 16 == 0) {
        hipLaunchKernelGGL(concat_v8_k, grid1(n / 8), dim3(256), 0, (hipStream_t)stream, (const uint4*)a, Ca / 8,
                           (const uint4*)b, Cb / 8, npix, (uint4*)y);
        return launch_status();
    }
    hipLaunchKernelGGL(concat_k, grid1(n), dim3(256), 0, (hipStream_t)stream, a, Ca, b, Cb, npix, y);
    return launch_status();
}

extern "C" int tpfnn_split(const uint16_t* dy, int32_t Ca, int32_t Cb, int64_t npix, uint16_t* da,
                           uint16_t* db, void* stream) {
    if (!dy || !da || !db || Ca <= 0 || Cb <= 0 || npix <= 0) return kEinval;
    const int64_t n = npix * (Ca + Cb);
    if (Ca % 8 == 0 && Cb % 8 == 0 && ((uintptr_t)dy | (uintptr_t)da | (uintptr_t)db) % 16 == 0) {
        hipLaunchKernelGGL(split_v8_k, grid1(n / 8), dim3(256), 0, (hipStream_t)stream, (const uint4*)dy, Ca / 8,
                           Cb / 8, npix, (uint4*)da, (uint4*)db);
        return launch_status();
    }
    hipLaunchKernelGGL(split_k, grid1(n), dim3(256), 0, (hipStream_t)stream, dy, Ca, Cb, npix, da, db);
    return launch_status();
}

extern "C" int tpfnn_add_inplace(uint16_t* a, const uint16_t* b, int64_t n, void* stream) {
    if (!a || !b || n < 0) return kEinval;
    if (n == 0) return kOk;
    hipLaunchKernelGGL(add_inplace_k, grid1(n), dim3(256), 0, (hipStream_t)stream, a, b, n);
    return launch_status();
}

extern "C" size_t tpfnn_head_workspace(int64_t npix, int32_t C) {
    const int64_t nblk = (npix + kHeadThreads - 1) / kHeadThreads;
    return (size_t)nblk * (C + 2) * sizeof(double) + 256;
}

extern "C" int tpfnn_head(const uint16_t* x, int64_t npix, int32_t C, const float* w, const float* b,
                          float* pred, const float* target, uint16_t* dx, float* dw, float* db, double* loss,
                          void* work, size_t work_bytes, void* stream) {
    if (!x || !w || !b || !pred || npix <= 0 || C <= 0 || C > 32) return kEinval;
    if (target && (!dx || !dw || !db || !loss || !work || work_bytes < tpfnn_head_workspace(npix, C)))
        return kEinval;
    const int64_t nblk = (npix + kHeadThreads - 1) / kHeadThreads;
    if (nblk > 0x7fffffff) return kEinval;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(head_k, dim3((unsigned)nblk), dim3(kHeadThreads), 0, st, x, npix, C, w, b, pred, target,
                       dx, (double*)work);
    if (hipGetLastError() != hipSuccess) return kEdevice;
    if (target)
        hipLaunchKernelGGL(head_final_k, dim3(C + 2), dim3(256), 0, st, (const double*)work, (int)nblk, C, npix, dw,
                           db, loss);
    return launch_status();
}

extern "C" int tpfnn_adam(float* p, float* m, float* v, const float* g, uint16_t* p_bf16, int64_t n, float lr,
                          float beta1, float beta2, float eps, int32_t t, void* stream) {
    if (!p || !m || !v || !g || n <= 0 || t <= 0) return kEinval;
    const float c1 = 1.f - powf(beta1, (float)t), c2 = 1.f - powf(beta2, (float)t);
    hipLaunchKernelGGL(adam_k, grid1(n), dim3(256), 0, (hipStream_t)stream, p, m, v, g, p_bf16, n, lr, beta1,
                       beta2, eps, c1, c2);
    return launch_status();
}

extern "C" int tpfnn_to_bf16(const float* x, uint16_t* y, int64_t n, void* stream) {
    if (!x || !y || n < 0) return kEinval;
    if (n == 0) return kOk;
    hipLaunchKernelGGL(to_bf16_k, grid1(n), dim3(256), 0, (hipStream_t)stream, x, y, n);
    return launch_status();
}

extern "C" int tpfnn_from_bf16(const uint16_t* x, float* y, int64_t n, void* stream) {
    if (!x || !y || n < 0) return kEinval;
    if (n == 0) return kOk;
    hipLaunchKernelGGL(from_bf16_k, grid1(n), dim3(256), 0, (hipStream_t)stream, x, y, n);
    return launch_status();
}

extern "C" int tpfnn_resample(const float* src, int32_t N, int32_t sh, int32_t sw, float* dst, int32_t dh,
                              int32_t dw, void* stream) {
    if (!src || !dst || N <= 0 || sh <= 0 || sw <= 0 || dh <= 0 || dw <= 0) return kEinval;
    const int64_t n = (int64_t)N * dh * dw;
    hipLaunchKernelGGL(resample_k, grid1(n), dim3(256), 0, (hipStream_t)stream, src, N, sh, sw, dst, dh, dw);
    return launch_status();
}

extern "C" int tpfnn_mass_project(const float* pred, const float* phi0, int64_t n, double target,
                                  double* phi1_out, double* info, void* stream) {
    if (!pred || !phi0 || !phi1_out || !info || n <= 0 || !(target > 0.0) || !std::isfinite(target))
        return kEinval;
    hipLaunchKernelGGL(mass_project_k, dim3(1), dim3(kProjThreads), 0, (hipStream_t)stream, pred, phi0, n,
                       (const double*)nullptr, target, phi1_out, info);
    return launch_status();
}

extern "C" int tpfnn_mass_project_batch(const float* pred, const float* phi0, int32_t count, int64_t n,
                                        const double* targets, double* phi1_out, double* info, void* stream) {
    if (!pred || !phi0 || !targets || !phi1_out || !info || count <= 0 || n <= 0) return kEinval;
    hipLaunchKernelGGL(mass_project_k, dim3(count), dim3(kProjThreads), 0, (hipStream_t)stream, pred, phi0, n,
                       targets, 0.0, phi1_out, info);
    return launch_status();
}

extern "C" int tpfnn_pack_input(const float* phi0, const float* phi1_init, const float* theta_deg,
                                const float* vol, int32_t N, int32_t H, int32_t W, uint16_t* x, void* stream) {
    if (!phi0 || !theta_deg || !vol || !x || N <= 0 || H <= 0 || W <= 0) return kEinval;
    const int64_t n = (int64_t)N * H * W;
    hipLaunchKernelGGL(pack_input_k, grid1(n), dim3(256), 0, (hipStream_t)stream, phi0, phi1_init, theta_deg,
                       vol, N, H * W, x);
    return launch_status();
}

// ---------------------------------------------------------------------------
// Allocation-free variant of the output head.  Its per-block partial sums live
// in a file-scope device array instead of a caller workspace.  Every device the
// library runs on holds one copy of the array until the process ends; its
// address on a device comes from hipGetSymbolAddress with that device current
// (in host code the array's name is not a device address).
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[TPFNN_HEAD_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
int scratch_on_current_device(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return kEdevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return kEdevice;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return kOk;
}
}  // namespace

extern "C" int tpfnn_head_noalloc(const uint16_t* x, int64_t npix, int32_t C, const float* w, const float* b,
                                  float* pred, const float* target, uint16_t* dx, float* dw, float* db,
                                  double* loss, void* stream) {
    if (!x || !w || !b || !pred || npix <= 0 || C <= 0 || C > 32) return kEinval;
    if (target && (!dx || !dw || !db || !loss)) return kEinval;
    if (tpfnn_head_workspace(npix, C) > (size_t)TPFNN_HEAD_SCRATCH_BYTES) return kEinval;
    void* work = nullptr;
    const int rc = scratch_on_current_device(&work);
    if (rc != kOk) return rc;
    // every block writes its own partial sums before the final kernel reads
    // them, so nothing needs clearing between calls
    return tpfnn_head(x, npix, C, w, b, pred, target, dx, dw, db, loss, work, (size_t)TPFNN_HEAD_SCRATCH_BYTES,
                      stream);
}
