// Launch interface of the surrogate's BF16-MFMA kernels (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nn {

enum Kind : int { KIND_C3 = 0, KIND_UP = 1, KIND_DOWN = 2, KIND_C1 = 3 };

struct ConvArgs {
    int kind;
    const uint16_t *x;    // input, BF16 channels-last
    int n, id, ih, iw;    // input batch and spatial sizes
    int cx, x_off, cin;   // channel stride, slice offset, slice count (multiple of 16)
    const uint16_t *w;    // packed weights (k_pack order)
    const float *bias;    // [cout] or null
    int relu;
    uint16_t *y;          // output BF16 (or null)
    int cy, y_off;
    float *y32;           // optional FP32 output [vox][cy32]
    int cy32;
    int od, oh, ow, cout; // output spatial sizes, channel count
};

struct WgradArgs {
    int kind;
    const uint16_t *x;
    int n, id, ih, iw, cx, x_off, cin;
    const uint16_t *g;    // output gradient
    int cg, g_off, cout;
    int od, oh, ow;
    long long chunk;      // voxels per partial
    float *partial;       // [nchunk][ntap][cin][cout]
    float *gw;            // [ntap][cin][cout]
    int accumulate;
};

hipError_t conv(const ConvArgs &a, hipStream_t st);
hipError_t pack(const float *w, int ntap, int cin, int cout, int cin_p, int cout_p, int transpose, uint16_t *out,
                hipStream_t st);
hipError_t wgrad(const WgradArgs &a, hipStream_t st);
hipError_t bias_grad(const uint16_t *g, long long nvox, int cg, int g_off, int cout, float *gb, int accumulate,
                     hipStream_t st);
hipError_t relu_bwd(uint16_t *g, int cg, int g_off, const uint16_t *y, int cy, int y_off, long long nvox, int c,
                    hipStream_t st);
hipError_t up_bwd(const uint16_t *fine, int cf, int f_off, uint16_t *coarse, int cc, int c_off, int n, int d, int h, int w,
                  int c, hipStream_t st);
hipError_t down_dgrad(const uint16_t *g, int cg, int g_off, const float *w, int cin, int cout, uint16_t *gx, int cx,
                      int x_off, int n, int d, int h, int wd, int accumulate, hipStream_t st);
hipError_t to_bf16(const float *x, int cs, long long nvox, int c, uint16_t *y, int cy, int y_off, int c_pad,
                   hipStream_t st);
hipError_t masked_mse(const float *pred, int cp, const float *target, const float *mask, long long nvox, int c,
                      uint16_t *g, int cg, float *loss_parts, int nparts, hipStream_t st);
hipError_t bbox(const float *field, int cf, int n, int R, int *box, hipStream_t st);
hipError_t crop_origin(const int *box, int n, int R, int D, int H, int W, int *origin, hipStream_t st);
hipError_t crop(const float *src, int c, int n, int R, const int *origin, int D, int H, int W, float *dst, int uncrop,
                hipStream_t st);
hipError_t adam(float *p, const float *g, float *m, float *v, long long n, float lr, float b1, float b2, float eps, int t,
                hipStream_t st);

}  // namespace nn
