// Library-owned grid U-Net of the surrogate control step: weight blob
// parsing, BF16 packing and the forward pass, sequenced on the host over the
// convolution kernels of mpm_nn.h (3 levels, 32/64/128 channels, 3^3
// convolutions, 2^3 stride-2 down, nearest x2 + 3^3 up, concatenation skips,
// 1^3 head).
#include "sur_net.hpp"

#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/mpm_nn.h"

namespace mpm {

namespace {

enum Kind { C3 = 0, UP = 1, DOWN = 2, C1 = 3 };

// The layers in the blob's order; channels at full width (divided by the
// width factor), cin 0 = the network input, cout 0 = the network output.
struct LayerDef {
    int kind, cin, cout, relu;
};
constexpr int NL = 15;
constexpr LayerDef LAYERS[NL] = {
    {C3, 0, 32, 1},     {C3, 32, 32, 1},   {DOWN, 32, 64, 1},  {C3, 64, 64, 1},   {C3, 64, 64, 1},
    {DOWN, 64, 128, 1}, {C3, 128, 128, 1}, {C3, 128, 128, 1},  {UP, 128, 64, 1},  {C3, 128, 64, 1},
    {C3, 64, 64, 1},    {UP, 64, 32, 1},   {C3, 64, 32, 1},    {C3, 32, 32, 1},   {C1, 32, 0, 0},
};
enum { L_E1A, L_E1B, L_D1, L_E2A, L_E2B, L_D2, L_E3A, L_E3B, L_U2, L_C2A, L_C2B, L_U1, L_C1A, L_C1B, L_HEAD };

constexpr int32_t BLOB_MAGIC = 0x554E504D;   // "MPNU" little-endian
constexpr int32_t BLOB_VERSION = 1;

int taps_of(int kind) { return kind == C3 || kind == UP ? 27 : (kind == DOWN ? 8 : 1); }
int ceil16(int c) { return (c + 15) / 16 * 16; }

}  // namespace

struct SurNet {
    int cin = 0, cout = 0, width = 1;
    int ci[NL] = {}, co[NL] = {};
    uint16_t *wpack[NL] = {};
    float *bias[NL] = {};
    // activations (BF16) for the current (n, D, H, W)
    int n = 0, D = 0, H = 0, W = 0;
    uint16_t *arena = nullptr;
    uint16_t *x = nullptr, *a1 = nullptr, *cat1 = nullptr, *a2 = nullptr, *a3 = nullptr, *cat2 = nullptr;
    uint16_t *a4 = nullptr, *a5 = nullptr, *a6 = nullptr, *a7 = nullptr, *a8 = nullptr, *a9 = nullptr,
             *a10 = nullptr;
};

static void free_acts(SurNet *net)
{
    if (net->arena) (void)hipFree(net->arena);
    net->arena = nullptr;
    net->n = net->D = net->H = net->W = 0;
}

void surnet_destroy(SurNet *net)
{
    if (!net) return;
    free_acts(net);
    for (int l = 0; l < NL; l++) {
        if (net->wpack[l]) (void)hipFree(net->wpack[l]);
        if (net->bias[l]) (void)hipFree(net->bias[l]);
    }
    delete net;
}

int surnet_cin(const SurNet *net) { return net->cin; }
int surnet_cout(const SurNet *net) { return net->cout; }

SurNet *surnet_load(const void *blob, size_t bytes, hipStream_t st, std::string *err, int *err_code)
{
    *err_code = -1;
    if (!blob || bytes < 8 * sizeof(int32_t)) {
        *err = "weight blob too short";
        return nullptr;
    }
    int32_t hdr[8];
    std::memcpy(hdr, blob, sizeof hdr);
    if (hdr[0] != BLOB_MAGIC || hdr[1] != BLOB_VERSION) {
        *err = "not a surrogate weight blob (magic / version)";
        return nullptr;
    }
    const int cin = hdr[2], cout = hdr[3], width = hdr[4], nl = hdr[5];
    if (nl != NL || cin < 1 || cin > 16 || cout < 4 || cout > 16 || (width != 1 && width != 2)) {
        *err = "unsupported network shape in the weight blob";
        return nullptr;
    }
    SurNet *net = new SurNet();
    net->cin = cin;
    net->cout = cout;
    net->width = width;
    size_t need = sizeof hdr;
    for (int l = 0; l < NL; l++) {
        net->ci[l] = LAYERS[l].cin ? LAYERS[l].cin / width : ceil16(cin);
        net->co[l] = LAYERS[l].cout ? LAYERS[l].cout / width : cout;
        need += sizeof(float) * ((size_t)taps_of(LAYERS[l].kind) * net->ci[l] * net->co[l] + net->co[l]);
    }
    if (bytes != need) {
        *err = "weight blob size does not match its network shape";
        delete net;
        return nullptr;
    }
    // upload per layer, pack on the device, drop the FP32 copy of the weights
    const char *p = (const char *)blob + sizeof hdr;
    float *wdev = nullptr;
    size_t wmax = 0;
    for (int l = 0; l < NL; l++) wmax = std::max(wmax, (size_t)taps_of(LAYERS[l].kind) * net->ci[l] * net->co[l]);
    hipError_t e = hipMalloc(&wdev, sizeof(float) * wmax);
    for (int l = 0; l < NL && e == hipSuccess; l++) {
        const int kind = LAYERS[l].kind, taps = taps_of(kind), ci = net->ci[l], co = net->co[l];
        const size_t nw = (size_t)taps * ci * co;
        std::vector<float> w(nw);
        std::memcpy(w.data(), p, sizeof(float) * nw);
        p += sizeof(float) * nw;
        int ci_pack = ci;
        if (l == L_E1A && cin == 8) {
            // the first layer reads the 8 real input channels (taps folded into the MFMA K)
            std::vector<float> w8((size_t)taps * 8 * co);
            for (int t = 0; t < taps; t++)
                for (int c = 0; c < 8; c++)
                    for (int o = 0; o < co; o++) w8[((size_t)t * 8 + c) * co + o] = w[((size_t)t * ci + c) * co + o];
            w.swap(w8);
            ci_pack = 8;
        }
        e = hipMemcpyAsync(wdev, w.data(), sizeof(float) * w.size(), hipMemcpyHostToDevice, st);
        if (e != hipSuccess) break;
        e = hipMalloc(&net->wpack[l], sizeof(uint16_t) * (size_t)taps * ceil16(ci) * ceil16(co));
        if (e != hipSuccess) break;
        if (mpm_nn_pack(wdev, kind, ci_pack, co, 0, net->wpack[l], st) != 0) {
            e = hipErrorInvalidValue;
            break;
        }
        e = hipMalloc(&net->bias[l], sizeof(float) * co);
        if (e != hipSuccess) break;
        e = hipMemcpyAsync(net->bias[l], p, sizeof(float) * co, hipMemcpyHostToDevice, st);
        p += sizeof(float) * co;
        if (e == hipSuccess) e = hipStreamSynchronize(st);   // the host copies above are reused
    }
    if (wdev) (void)hipFree(wdev);
    if (e != hipSuccess) {
        *err = std::string("loading the surrogate weights: ") + hipGetErrorString(e);
        *err_code = e == hipErrorOutOfMemory ? -3 : -2;
        surnet_destroy(net);
        return nullptr;
    }
    *err_code = 0;
    return net;
}

static int alloc_acts(SurNet *net, int n, int D, int H, int W, std::string *err)
{
    if (net->arena && net->n == n && net->D == D && net->H == H && net->W == W) return 0;
    free_acts(net);
    const int w = net->width, c1 = 32 / w, c2 = 64 / w, c3 = 128 / w;
    const size_t v1 = (size_t)n * D * H * W, v2 = v1 / 8, v3 = v1 / 64;
    // channel counts per buffer, in carve order
    const size_t sizes[13] = {v1 * 16, v1 * c1, v1 * 2 * c1, v2 * c2, v2 * c2, v2 * 2 * c2, v3 * c3,
                              v3 * c3, v3 * c3, v2 * c2, v2 * c2, v1 * c1, v1 * c1};
    size_t total = 0;
    for (size_t s : sizes) total += (s + 127) / 128 * 128;   // 256-byte aligned pieces
    hipError_t e = hipMalloc(&net->arena, sizeof(uint16_t) * total);
    if (e != hipSuccess) {
        net->arena = nullptr;
        *err = std::string("surrogate activations: ") + hipGetErrorString(e);
        return e == hipErrorOutOfMemory ? -3 : -2;
    }
    uint16_t **dst[13] = {&net->x, &net->a1, &net->cat1, &net->a2, &net->a3, &net->cat2, &net->a4,
                          &net->a5, &net->a6, &net->a7, &net->a8, &net->a9, &net->a10};
    size_t off = 0;
    for (int i = 0; i < 13; i++) {
        *dst[i] = net->arena + off;
        off += (sizes[i] + 127) / 128 * 128;
    }
    net->n = n;
    net->D = D;
    net->H = H;
    net->W = W;
    return 0;
}

int surnet_forward(SurNet *net, const float *feat, int cf, int n, int D, int H, int W, float *pred, hipStream_t st,
                   std::string *err)
{
    if (!net || !feat || !pred || n <= 0 || D % 4 || H % 4 || W % 4 || D <= 0 || H <= 0 || W <= 0 ||
        cf < net->cin) {
        *err = "surrogate forward: bad sizes";
        return -1;
    }
    int r = alloc_acts(net, n, D, H, W, err);
    if (r) return r;
    const int w = net->width, c1 = 32 / w, c2 = 64 / w, c3 = 128 / w;
    const int d2 = D / 2, h2 = H / 2, w2 = W / 2, d3 = D / 4, h3 = H / 4, w3 = W / 4;
    const long long v1 = (long long)n * D * H * W;
    void *s = (void *)st;
    auto conv = [&](int l, const uint16_t *x, int d, int h, int ww, int cx, int x_off, int cin_used, uint16_t *y,
                    int cy, int y_off, float *y32, int cy32) {
        if (r) return;
        if (l < 0 || l >= NL) {
            r = -1;
            *err = "surrogate forward: bad layer index";
            return;
        }
        r = mpm_nn_conv(LAYERS[l].kind, x, n, d, h, ww, cx, x_off, cin_used, net->wpack[l], net->bias[l],
                        LAYERS[l].relu, y, cy, y_off, net->co[l], y32, cy32, s);
        if (r) *err = "surrogate forward: convolution " + std::to_string(l) + " failed";
    };
    r = mpm_nn_to_bf16(feat, cf, v1, net->cin, net->x, 16, 0, 16, s);
    if (r) {
        *err = "surrogate forward: input conversion failed";
        return r;
    }
    conv(L_E1A, net->x, D, H, W, 16, 0, net->cin == 8 ? 8 : 16, net->a1, c1, 0, nullptr, 0);
    conv(L_E1B, net->a1, D, H, W, c1, 0, c1, net->cat1, 2 * c1, c1, nullptr, 0);
    conv(L_D1, net->cat1, D, H, W, 2 * c1, c1, c1, net->a2, c2, 0, nullptr, 0);
    conv(L_E2A, net->a2, d2, h2, w2, c2, 0, c2, net->a3, c2, 0, nullptr, 0);
    conv(L_E2B, net->a3, d2, h2, w2, c2, 0, c2, net->cat2, 2 * c2, c2, nullptr, 0);
    conv(L_D2, net->cat2, d2, h2, w2, 2 * c2, c2, c2, net->a4, c3, 0, nullptr, 0);
    conv(L_E3A, net->a4, d3, h3, w3, c3, 0, c3, net->a5, c3, 0, nullptr, 0);
    conv(L_E3B, net->a5, d3, h3, w3, c3, 0, c3, net->a6, c3, 0, nullptr, 0);
    conv(L_U2, net->a6, d3, h3, w3, c3, 0, c3, net->cat2, 2 * c2, 0, nullptr, 0);
    conv(L_C2A, net->cat2, d2, h2, w2, 2 * c2, 0, 2 * c2, net->a7, c2, 0, nullptr, 0);
    conv(L_C2B, net->a7, d2, h2, w2, c2, 0, c2, net->a8, c2, 0, nullptr, 0);
    conv(L_U1, net->a8, d2, h2, w2, c2, 0, c2, net->cat1, 2 * c1, 0, nullptr, 0);
    conv(L_C1A, net->cat1, D, H, W, 2 * c1, 0, 2 * c1, net->a9, c1, 0, nullptr, 0);
    conv(L_C1B, net->a9, D, H, W, c1, 0, c1, net->a10, c1, 0, nullptr, 0);
    conv(L_HEAD, net->a10, D, H, W, c1, 0, c1, nullptr, 0, 0, pred, net->cout);
    return r;
}

}  // namespace mpm
