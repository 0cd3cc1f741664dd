/*
 * mpm_nn.h -- C ABI of the grid U-Net surrogate kernels (libmpm_hip.so).
 *
 * The paper has no learned component; these kernels serve the surrogate
 * this library adds in front of the MLS-MPM substep (the network stands in
 * for a 25-substep control step, App. E.3 gives 25 physics steps per control
 * step, and the plain MPM stays its fallback).  They are the training and
 * inference primitives the Python driver composes into the U-Net:
 * convolution forward / adjoint (BF16 MFMA, FP32 accumulate), weight and
 * bias gradients, ReLU and resampling backward, masked MSE, Adam.
 *
 * Conventions: all pointers are device pointers on the current device;
 * work is queued on `stream` (a hipStream_t, NULL = default) and the call
 * returns without waiting.  Activations are BF16 (uint16_t bit patterns),
 * channels-last [n][d][h][w][c]; a call reads / writes the channel slice
 * [off, off + count) of a tensor whose channel stride is `c...`.  Channel
 * counts on the MFMA paths are multiples of 16 (<= 128 input channels for
 * weight gradients); a 3^3 convolution may also take exactly 8 input
 * channels (the network's first layer; channel stride and offset of its
 * input multiples of 8).  Weights are FP32 [taps][cin][cout] (taps = 27, 8 or 1,
 * z-major, as [kd][kh][kw]).  Every call returns 0 on success, -1 on an
 * invalid argument (nothing queued), -2 on a HIP error.
 *
 * kind: 0 = 3^3 convolution, zero padding 1; 1 = 3^3 convolution of the
 * nearest x2 upsampled input (output = 2 x input size); 2 = 2^3 stride-2
 * convolution (output = input / 2); 3 = 1^3 convolution.
 */
#ifndef MPM_NN_H
#define MPM_NN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Pack FP32 weights into the BF16 fragment order of mpm_nn_conv (the
 * order depends on kind and cin_eff: 16x16x16 or 16x16x32 fragments, or the
 * first-layer order with the taps in K for kind 0 and cin = 8).
 * transpose = 0: weights of the layer; 1: weights of its adjoint (input
 * gradient) convolution, taps mirrored and channels swapped.  out holds
 * taps * ceil16(cin_eff) * ceil16(cout_eff) BF16 values, where (cin_eff,
 * cout_eff) = (cin, cout), or (cout, cin) when transposed (the first-layer
 * order uses 224 * ceil16(cout) of them). */
int mpm_nn_pack(const float *w, int kind, int cin, int cout, int transpose, uint16_t *out, void *stream);

/* y = act(conv(x) + bias): input [n][id][ih][iw] slice (cx, x_off, cin),
 * output slice (cy, y_off, cout); relu = 1 applies max(0, .); y32 (nullable)
 * additionally receives FP32 outputs [voxel][cy32]. */
int mpm_nn_conv(int kind, const uint16_t *x, int n, int id, int ih, int iw, int cx, int x_off, int cin,
                const uint16_t *wpack, const float *bias, int relu, uint16_t *y, int cy, int y_off, int cout,
                float *y32, int cy32, void *stream);

/* Weight gradient gw[taps][cin][cout] (+= when accumulate) of the layer that
 * maps x to an output whose gradient is g; `partial` is scratch of
 * ceil(voxels / chunk) * taps * cin * cout floats. */
int mpm_nn_wgrad(int kind, const uint16_t *x, int n, int id, int ih, int iw, int cx, int x_off, int cin,
                 const uint16_t *g, int cg, int g_off, int cout, long long chunk, float *partial, float *gw,
                 int accumulate, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * weight gradient as mpm_nn_wgrad with its partial sums kept in a scratch
 * array the library holds on every GPU it runs on (MPM_NN_SCRATCH_BYTES,
 * reserved from the first call on a device until the process ends).  The
 * call allocates nothing.  Returns -3 when the partial sums,
 * ceil(voxels / chunk) * taps * cin * cout floats, exceed the scratch (raise
 * chunk); otherwise as mpm_nn_wgrad.  Every call on one GPU uses the same
 * scratch, which keeps the last call's values (each call writes every
 * partial it reads, so nothing needs clearing): calls that may run
 * concurrently on one GPU (different streams, host threads) race. */
#define MPM_NN_SCRATCH_BYTES (32LL << 20)
int mpm_nn_wgrad_noalloc(int kind, const uint16_t *x, int n, int id, int ih, int iw, int cx, int x_off, int cin,
                         const uint16_t *g, int cg, int g_off, int cout, long long chunk, float *gw, int accumulate,
                         void *stream);

/* gb[co] (+)= sum over voxels of g[voxel][g_off + co] (cout <= 128; the
 * partial sums are added with float atomics, so the summation order -- and
 * the last bit -- may differ between calls). */
int mpm_nn_bias_grad(const uint16_t *g, long long voxels, int cg, int g_off, int cout, float *gb, int accumulate,
                     void *stream);

/* g *= (y > 0) on a channel slice (ReLU backward from the layer output y). */
int mpm_nn_relu_bwd(uint16_t *g, int cg, int g_off, const uint16_t *y, int cy, int y_off, long long voxels, int c,
                    void *stream);

/* coarse[v] = sum of the 8 children of v in `fine` (upsampling backward);
 * (n, d, h, w) are the coarse sizes. */
int mpm_nn_up_bwd(const uint16_t *fine, int cf, int f_off, uint16_t *coarse, int cc, int c_off, int n, int d, int h,
                  int w, int c, void *stream);

/* Input gradient of the 2^3 stride-2 convolution with FP32 weights w
 * [8][cin][cout] (16-byte aligned for the MFMA path), which are rounded to
 * BF16 as in every other adjoint; (n, d, h, wd) are the fine (input) sizes;
 * accumulate = 1 adds to gx (a skip connection's gradient already there). */
int mpm_nn_down_dgrad(const uint16_t *g, int cg, int g_off, const float *w, int cin, int cout, uint16_t *gx, int cx,
                      int x_off, int n, int d, int h, int wd, int accumulate, void *stream);

/* FP32 [voxel][cs] (first c channels) -> BF16 slice, zero-padded to c_pad channels. */
int mpm_nn_to_bf16(const float *x, int cs, long long voxels, int c, uint16_t *y, int cy, int y_off, int c_pad,
                   void *stream);

/* Masked MSE over the first c channels: loss_parts holds nparts + 1 floats;
 * loss_parts[0 .. nparts) receive partial sums of mask (pred - target)^2 and
 * loss_parts[nparts] the number of masked voxels (mask != 0), so the loss is
 * sum(parts) / (count c).  g [voxel][cg] receives 2 (pred - target) / (count c)
 * on masked voxels and 0 elsewhere (all cg channels).  voxels < 2^24. */
int mpm_nn_masked_mse(const float *pred, int cp, const float *target, const float *mask, long long voxels, int c,
                      uint16_t *g, int cg, float *loss_parts, int nparts, void *stream);

/* One bias-corrected Adam step (t >= 1) on n FP32 parameters. */
int mpm_nn_adam(float *p, const float *g, float *m, float *v, long long n, float lr, float beta1, float beta2,
                float eps, int t, void *stream);

/* Crops of dense per-scene grids [n][R][R][R][c] (the surrogate runs on a
 * box around the material instead of the whole grid).
 * mpm_nn_bbox: bbox[g] (device, [n][6] ints) = (lo x, y, z, hi x, y, z) of
 *   the nodes whose channel 0 of field [n][R^3][cf] is positive, hi
 *   exclusive; all zeros for a grid with none.
 * mpm_nn_crop_origin: origin[g] (device, [n][3]) of a (D, H, W) box centred
 *   on bbox[g] and moved inside the grid (D, H, W <= R).
 * mpm_nn_crop: uncrop = 0: dst [n][D][H][W][c] = src [n][R^3][c] at
 *   origin + (z, y, x); uncrop = 1: dst [n][R^3][c] = src [n][D][H][W][c]
 *   inside the box, 0 outside. */
int mpm_nn_bbox(const float *field, int cf, int n, int R, int *bbox, void *stream);
int mpm_nn_crop_origin(const int *bbox, int n, int R, int D, int H, int W, int *origin, void *stream);
int mpm_nn_crop(const float *src, int c, int n, int R, const int *origin, int D, int H, int W, float *dst, int uncrop,
                void *stream);

#ifdef __cplusplus
}
#endif
#endif /* MPM_NN_H */
