/*
 * tpf_nn.h -- C ABI of the kernels behind the learned warm start: a small
 * convolutional encoder-decoder that predicts the equilibrium phase field
 * phi1 from the solid field phi0, a contact-angle map and the droplet volume,
 * trained on equilibria that the lattice Boltzmann library itself computes.
 * The LB method then relaxes from the prediction (Zhan, Chai & Shi, arXiv
 * 2311.05091, supplies the LB method; the network is not part of the paper).
 *
 * Conventions
 *   - All pointers are device pointers; sizes are element counts.  Tensors
 *     are NHWC (channels fastest).  Activations and gradients flowing through
 *     the network are bfloat16 (stored as uint16_t); weights have an FP32
 *     master copy and a bf16 copy; all products accumulate in FP32 on the
 *     BF16 matrix cores (v_mfma_f32_16x16x32_bf16).
 *   - Convolution weights are [Cout][3][3][Cin]; channel counts of the
 *     matrix-core paths must be multiples of 32; H*W must be a multiple of 64.
 *   - Every function enqueues on `stream` (a hipStream_t, NULL = default) and
 *     returns 0, or TPF_EINVAL (-1) for shapes the kernels do not support,
 *     or TPF_EDEVICE (-2) for a launch failure.  Nothing is allocated.
 */
#ifndef TPF_NN_H
#define TPF_NN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* D = A B for one 16x32 (row-major bf16) by 32x16 (row-major bf16) product
 * on one wavefront's matrix core; D is 16x16 row-major FP32.  Checks the
 * operand layout the convolution kernels rely on. */
int tpfnn_mfma_selftest(const uint16_t* A, const uint16_t* B, float* D, void* stream);

/* y[n,h,w,co] = act(bias[co] + sum_{ky,kx,ci} w[co,ky,kx,ci] x[n,h+ky-1,w+kx-1,ci]),
 * zero padding, act = ReLU when relu != 0.  bias may be NULL.  Cin, Cout
 * multiples of 32, H W a multiple of 64.  Layers with Cout a multiple of 64
 * and W a multiple of 128 (or W = 16, 32, 64 with H holding 128 / W rows)
 * run a kernel that stages each 32-channel input patch and the weights of
 * all nine taps in LDS once per chunk; the others stage one tap at a time. */
int tpfnn_conv3x3_fwd(const uint16_t* x, int32_t N, int32_t H, int32_t W, int32_t Cin,
                      const uint16_t* w, const float* bias, int32_t Cout, int32_t relu,
                      uint16_t* y, void* stream);

/* wt[ci,ky,kx,co] = w[co,2-ky,2-kx,ci] (bf16): the weights of the input-gradient
 * convolution, dx = conv3x3(dy, wt). */
int tpfnn_weight_flip(const uint16_t* w, int32_t Cout, int32_t Cin, uint16_t* wt, void* stream);

/* dw[co,ky,kx,ci] = sum_{n,h,w} dy[n,h,w,co] x[n,h+ky-1,w+kx-1,ci] and, when db is
 * not NULL, db[co] = sum dy[...,co]; both FP32, overwritten.  work must hold
 * tpfnn_wgrad_workspace(...) bytes (split-K partial sums, reduced in a fixed
 * order so that the result is deterministic).  Cin, Cout multiples of 32,
 * H*W a multiple of 64; with db, Cout must divide 256 (TPF_EINVAL otherwise). */
size_t tpfnn_wgrad_workspace(int32_t N, int32_t H, int32_t W, int32_t Cin, int32_t Cout);
int tpfnn_conv3x3_wgrad(const uint16_t* x, const uint16_t* dy, int32_t N, int32_t H, int32_t W,
                        int32_t Cin, int32_t Cout, float* dw, float* db, void* work,
                        size_t work_bytes, void* stream);

/* dy *= (y > 0), in place (backward of ReLU given its output y). */
int tpfnn_relu_bwd(const uint16_t* y, uint16_t* dy, int64_t n, void* stream);

/* 2x2 average pooling and its adjoint (NHWC, H and W even). */
int tpfnn_avgpool2_fwd(const uint16_t* x, int32_t N, int32_t H, int32_t W, int32_t C, uint16_t* y,
                       void* stream);
int tpfnn_avgpool2_bwd(const uint16_t* dy, int32_t N, int32_t H, int32_t W, int32_t C, uint16_t* dx,
                       void* stream);
/* nearest 2x upsampling of an [N,H,W,C] tensor and its adjoint (sum of 4). */
int tpfnn_upsample2_fwd(const uint16_t* x, int32_t N, int32_t H, int32_t W, int32_t C, uint16_t* y,
                        void* stream);
int tpfnn_upsample2_bwd(const uint16_t* dy, int32_t N, int32_t H, int32_t W, int32_t C, uint16_t* dx,
                        void* stream);
/* channel concatenation y = [a | b] and its adjoint (split). */
int tpfnn_concat(const uint16_t* a, int32_t Ca, const uint16_t* b, int32_t Cb, int64_t npix,
                 uint16_t* y, void* stream);
int tpfnn_split(const uint16_t* dy, int32_t Ca, int32_t Cb, int64_t npix, uint16_t* da,
                uint16_t* db, void* stream);
/* a += b elementwise (gradient accumulation of a tensor used twice). */
int tpfnn_add_inplace(uint16_t* a, const uint16_t* b, int64_t n, void* stream);

/* Output head: z = b + sum_c w[c] x[p,c], pred = sigmoid(z) (FP32).  When target
 * (values in [0, 1]) is not NULL also the mean binary cross-entropy
 * loss = mean_p softplus(z) - target z (FP64 sum, deterministic order),
 * dx[p,c] = dz w[c] (bf16), dw[c] = sum_p dz x[p,c], db = sum_p dz (FP32),
 * dz = (pred - target)/npix.  work must hold
 * tpfnn_head_workspace(npix, C) bytes. */
size_t tpfnn_head_workspace(int64_t npix, int32_t C);
int tpfnn_head(const uint16_t* x, int64_t npix, int32_t C, const float* w, const float* b,
               float* pred, const float* target, uint16_t* dx, float* dw, float* db, double* loss,
               void* work, size_t work_bytes, void* stream);

/* Allocation-free variant of tpfnn_head, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same kernels and results, with the partial sums
 * in a fixed device array of TPFNN_HEAD_SCRATCH_BYTES that the library holds
 * on each device it runs on until the process ends.  Calls with
 * tpfnn_head_workspace(npix, C) > TPFNN_HEAD_SCRATCH_BYTES (with C = 32 about
 * 3.9 M pixels) return TPF_EINVAL (-1) without launching anything; -2 if the
 * array's device address cannot be obtained.  The call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine).  The device current
 * on the calling thread must be the one `stream` belongs to.  All calls on a
 * device share its array: calls that overlap in time on one device (other
 * streams, other threads) race and must be serialised by the caller. */
#define TPFNN_HEAD_SCRATCH_BYTES (4u << 20)
int tpfnn_head_noalloc(const uint16_t* x, int64_t npix, int32_t C, const float* w, const float* b,
                       float* pred, const float* target, uint16_t* dx, float* dw, float* db, double* loss,
                       void* stream);

/* Adam with bias correction on FP32 master weights; also writes the bf16 copy
 * (p_bf16 may be NULL).  t is the 1-based step count. */
int tpfnn_adam(float* p, float* m, float* v, const float* g, uint16_t* p_bf16, int64_t n, float lr,
               float beta1, float beta2, float eps, int32_t t, void* stream);

/* FP32 -> bf16 (round to nearest even) and back. */
int tpfnn_to_bf16(const float* x, uint16_t* y, int64_t n, void* stream);
int tpfnn_from_bf16(const uint16_t* x, float* y, int64_t n, void* stream);

/* Bilinear resampling of N single-channel fields [N,sh,sw] -> [N,dh,dw]
 * (FP32, align-corners sampling: the corner nodes map onto each other). */
int tpfnn_resample(const float* src, int32_t N, int32_t sh, int32_t sw, float* dst, int32_t dh,
                   int32_t dw, void* stream);

/* Mass projection of a predicted phase field (the warm start): phi1_out[i] =
 * sigmoid(logit(p_i) + c) (1 - phi0_i) with p_i = pred[i] clipped to
 * [1e-7, 1 - 1e-7] and the shift c in [-40, 40] such that sum(phi1_out) =
 * target (the sum increases with c; Newton steps kept inside a bisection
 * bracket find the root); a last factor target/sum (|factor - 1| ~ 1e-7) makes
 * the sum exact in FP64.  Unlike a multiplicative rescale the field stays in
 * [0, 1 - phi0], so phi2 = 1 - phi0 - phi1 stays non-negative.  pred, phi0:
 * [n] FP32 device; phi1_out: [n] FP64 device; info: 2 FP64 device values
 * (c, sum before the last factor), both NaN (and phi1_out zero) when the
 * target is out of reach.  One block; deterministic. */
int tpfnn_mass_project(const float* pred, const float* phi0, int64_t n, double target, double* phi1_out,
                       double* info, void* stream);
/* The same projection for `count` fields of n nodes each, one block per field,
 * all launched at once: pred, phi0 [count][n] FP32 device; targets [count]
 * FP64 device (each positive and finite, else that field's info is NaN as
 * for an unreachable target); phi1_out [count][n] FP64 device; info
 * [count][2] FP64 device.  Field b's output equals tpfnn_mass_project on
 * field b alone. */
int tpfnn_mass_project_batch(const float* pred, const float* phi0, int32_t count, int64_t n,
                             const double* targets, double* phi1_out, double* info, void* stream);

/* Network input from physical fields: x[n,h,w,:] = (phi0, (theta - 90 deg)/60 deg,
 * volume scale, plain initial phi1, 0, ..., 0) padded to 32 channels (bf16).
 * phi0 and phi1_init are [N,H,W] FP32, theta_deg and vol [N]; phi1_init may be
 * NULL (channel 3 is then zero). */
int tpfnn_pack_input(const float* phi0, const float* phi1_init, const float* theta_deg, const float* vol,
                     int32_t N, int32_t H, int32_t W, uint16_t* x, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* TPF_NN_H */
