// C ABI of the surrogate kernels (argument checks + launches).
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/mpm_nn.h"
#include "nn_kernels.hpp"

namespace {

int taps_of(int kind) { return kind == 0 || kind == 1 ? 27 : (kind == 2 ? 8 : 1); }
int ceil16(int c) { return (c + 15) / 16 * 16; }
int st_of(hipError_t e) { return e == hipSuccess ? 0 : -2; }
bool kind_ok(int k) { return k >= 0 && k <= 3; }
bool c16(int c) { return c > 0 && c % 16 == 0; }

void out_size(int kind, int id, int ih, int iw, int &od, int &oh, int &ow)
{
    if (kind == 1) { od = 2 * id; oh = 2 * ih; ow = 2 * iw; }
    else if (kind == 2) { od = id / 2; oh = ih / 2; ow = iw / 2; }
    else { od = id; oh = ih; ow = iw; }
}

// Partial sums of the allocation-free weight gradient (mpm_nn_wgrad_noalloc):
// one array per GPU, held until the process ends.  Host code never passes
// its name to a kernel: the device address comes from hipGetSymbolAddress,
// once per device (scratch_of_device).
constexpr long long NN_SCRATCH_FLOATS = MPM_NN_SCRATCH_BYTES / sizeof(float);
static_assert(MPM_NN_SCRATCH_BYTES % 256 == 0, "scratch size");
__device__ __align__(256) float scratch[NN_SCRATCH_FLOATS];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
float *scratch_dev[MAX_DEVICES] = {};

// Device address of the current device's scratch, looked up on first use.
int scratch_of_device(float **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -2;
    if (dev < 0 || dev >= MAX_DEVICES) return -1;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return -2;
        scratch_dev[dev] = (float *)p;
    }
    *out = scratch_dev[dev];
    return 0;
}

// Weight gradient with its partial sums in `partial` (cap floats, or < 0:
// the caller sized it).  -3 when the partial sums do not fit in cap.
int wgrad_call(int kind, const uint16_t *x, int n, int id, int ih, int iw, int cx, int x_off, int cin,
               const uint16_t *g, int cg, int g_off, int cout, long long chunk, float *partial, long long cap, float *gw,
               int accumulate, void *stream)
{
    if (!kind_ok(kind) || !x || !g || !partial || !gw || n <= 0 || chunk < 16 || chunk % 16) return -1;
    if (!c16(cin) || cin > 128 || cout <= 0 || cout > 128 || x_off + cin > cx || g_off + cout > cg) return -1;
    if (id <= 0 || ih <= 0 || iw <= 0) return -1;
    const int nf = (cout + 15) / 16;
    if (nf != 1 && nf != 2 && nf != 4 && nf != 8) return -1;
    nn::WgradArgs a{};
    a.kind = kind;
    a.x = x; a.n = n; a.id = id; a.ih = ih; a.iw = iw; a.cx = cx; a.x_off = x_off; a.cin = cin;
    a.g = g; a.cg = cg; a.g_off = g_off; a.cout = cout;
    out_size(kind, id, ih, iw, a.od, a.oh, a.ow);
    a.chunk = chunk; a.partial = partial; a.gw = gw; a.accumulate = accumulate;
    if (cap >= 0) {
        const long long nvox = (long long)n * a.od * a.oh * a.ow;
        const long long need = (nvox + chunk - 1) / chunk * taps_of(kind) * cin * cout;
        if (need > cap) return -3;
    }
    return st_of(nn::wgrad(a, (hipStream_t)stream));
}

}  // namespace

extern "C" {

int mpm_nn_pack(const float *w, int kind, int cin, int cout, int transpose, uint16_t *out, void *stream)
{
    if (!w || !out || !kind_ok(kind) || cin <= 0 || cout <= 0) return -1;
    const int ci_e = transpose ? cout : cin, co_e = transpose ? cin : cout;
    return st_of(nn::pack(w, taps_of(kind), cin, cout, ceil16(ci_e), ceil16(co_e), transpose, out,
                          (hipStream_t)stream));
}

int mpm_nn_conv(int kind, const uint16_t *x, int n, int id, int ih, int iw, int cx, int x_off, int cin,
                const uint16_t *wpack, const float *bias, int relu, uint16_t *y, int cy, int y_off, int cout,
                float *y32, int cy32, void *stream)
{
    if (!kind_ok(kind) || !x || !wpack || (!y && !y32) || n <= 0 || id <= 0 || ih <= 0 || iw <= 0) return -1;
    if (!(c16(cin) || (kind == 0 && cin == 8)) || cout <= 0 || cout > 128 || x_off < 0 || x_off + cin > cx ||
        (x_off % 4) || (cx % 4))
        return -1;
    if (cin == 8 && ((x_off % 8) || (cx % 8))) return -1;
    if (y && (y_off < 0 || y_off + cout > cy)) return -1;
    if (y32 && cy32 < cout) return -1;
    if (kind == 2 && (id % 2 || ih % 2 || iw % 2)) return -1;
    nn::ConvArgs a{};
    a.kind = kind;
    a.x = x; a.n = n; a.id = id; a.ih = ih; a.iw = iw; a.cx = cx; a.x_off = x_off; a.cin = cin;
    a.w = wpack; a.bias = bias; a.relu = relu;
    a.y = y; a.cy = cy; a.y_off = y_off; a.y32 = y32; a.cy32 = cy32;
    out_size(kind, id, ih, iw, a.od, a.oh, a.ow);
    a.cout = cout;
    if ((cout + 15) / 16 != 1 && (cout + 15) / 16 != 2 && (cout + 15) / 16 != 4 && (cout + 15) / 16 != 8) return -1;
    return st_of(nn::conv(a, (hipStream_t)stream));
}

int mpm_nn_wgrad(int kind, const uint16_t *x, int n, int id, int ih, int iw, int cx, int x_off, int cin,
                 const uint16_t *g, int cg, int g_off, int cout, long long chunk, float *partial, float *gw,
                 int accumulate, void *stream)
{
    if (!partial) return -1;
    return wgrad_call(kind, x, n, id, ih, iw, cx, x_off, cin, g, cg, g_off, cout, chunk, partial, -1, gw, accumulate,
                      stream);
}

int mpm_nn_wgrad_noalloc(int kind, const uint16_t *x, int n, int id, int ih, int iw, int cx, int x_off, int cin,
                         const uint16_t *g, int cg, int g_off, int cout, long long chunk, float *gw, int accumulate,
                         void *stream)
{
    float *ptr = nullptr;
    const int r = scratch_of_device(&ptr);
    if (r) return r;
    return wgrad_call(kind, x, n, id, ih, iw, cx, x_off, cin, g, cg, g_off, cout, chunk, ptr, NN_SCRATCH_FLOATS, gw,
                      accumulate, stream);
}

int mpm_nn_bias_grad(const uint16_t *g, long long voxels, int cg, int g_off, int cout, float *gb, int accumulate,
                     void *stream)
{
    if (!g || !gb || voxels <= 0 || cout <= 0 || cout > 128 || g_off + cout > cg) return -1;
    return st_of(nn::bias_grad(g, voxels, cg, g_off, cout, gb, accumulate, (hipStream_t)stream));
}

int mpm_nn_relu_bwd(uint16_t *g, int cg, int g_off, const uint16_t *y, int cy, int y_off, long long voxels, int c,
                    void *stream)
{
    if (!g || !y || voxels <= 0 || c <= 0 || g_off + c > cg || y_off + c > cy) return -1;
    return st_of(nn::relu_bwd(g, cg, g_off, y, cy, y_off, voxels, c, (hipStream_t)stream));
}

int mpm_nn_up_bwd(const uint16_t *fine, int cf, int f_off, uint16_t *coarse, int cc, int c_off, int n, int d, int h,
                  int w, int c, void *stream)
{
    if (!fine || !coarse || n <= 0 || d <= 0 || h <= 0 || w <= 0 || c <= 0 || f_off + c > cf || c_off + c > cc) return -1;
    return st_of(nn::up_bwd(fine, cf, f_off, coarse, cc, c_off, n, d, h, w, c, (hipStream_t)stream));
}

int mpm_nn_down_dgrad(const uint16_t *g, int cg, int g_off, const float *w, int cin, int cout, uint16_t *gx, int cx,
                      int x_off, int n, int d, int h, int wd, int accumulate, void *stream)
{
    if (!g || !w || !gx || n <= 0 || d % 2 || h % 2 || wd % 2 || cin <= 0 || cout <= 0) return -1;
    if (g_off + cout > cg || x_off + cin > cx) return -1;
    return st_of(nn::down_dgrad(g, cg, g_off, w, cin, cout, gx, cx, x_off, n, d, h, wd, accumulate, (hipStream_t)stream));
}

int mpm_nn_to_bf16(const float *x, int cs, long long voxels, int c, uint16_t *y, int cy, int y_off, int c_pad,
                   void *stream)
{
    if (!x || !y || voxels <= 0 || c <= 0 || c_pad < c || y_off + c_pad > cy || cs < c) return -1;
    return st_of(nn::to_bf16(x, cs, voxels, c, y, cy, y_off, c_pad, (hipStream_t)stream));
}

int mpm_nn_masked_mse(const float *pred, int cp, const float *target, const float *mask, long long voxels, int c,
                      uint16_t *g, int cg, float *loss_parts, int nparts, void *stream)
{
    if (!pred || !target || !mask || !g || !loss_parts || voxels <= 0 || c <= 0 || cp < c || cg < c || nparts <= 0)
        return -1;
    if (nparts > 65535 || voxels >= (1LL << 24)) return -1;
    return st_of(nn::masked_mse(pred, cp, target, mask, voxels, c, g, cg, loss_parts, nparts, (hipStream_t)stream));
}

int mpm_nn_adam(float *p, const float *g, float *m, float *v, long long n, float lr, float beta1, float beta2,
                float eps, int t, void *stream)
{
    if (!p || !g || !m || !v || n <= 0 || t < 1) return -1;
    return st_of(nn::adam(p, g, m, v, n, lr, beta1, beta2, eps, t, (hipStream_t)stream));
}

int mpm_nn_bbox(const float *field, int cf, int n, int R, int *bbox, void *stream)
{
    if (!field || !bbox || cf <= 0 || n <= 0 || R <= 0) return -1;
    return st_of(nn::bbox(field, cf, n, R, bbox, (hipStream_t)stream));
}

int mpm_nn_crop_origin(const int *bbox, int n, int R, int D, int H, int W, int *origin, void *stream)
{
    if (!bbox || !origin || n <= 0 || D <= 0 || H <= 0 || W <= 0 || D > R || H > R || W > R) return -1;
    return st_of(nn::crop_origin(bbox, n, R, D, H, W, origin, (hipStream_t)stream));
}

int mpm_nn_crop(const float *src, int c, int n, int R, const int *origin, int D, int H, int W, float *dst, int uncrop,
                void *stream)
{
    if (!src || !dst || !origin || c <= 0 || n <= 0 || D <= 0 || H <= 0 || W <= 0 || D > R || H > R || W > R) return -1;
    if (uncrop != 0 && uncrop != 1) return -1;
    return st_of(nn::crop(src, c, n, R, origin, D, H, W, dst, uncrop, (hipStream_t)stream));
}

}  // extern "C"
