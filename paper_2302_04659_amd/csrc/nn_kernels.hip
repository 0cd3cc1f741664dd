// BF16-MFMA / FP32-accumulate kernels of the grid U-Net surrogate (gfx950).
//
// Activations are BF16, channels-last [N][D][H][W][C]; a kernel reads or
// writes a channel slice [off, off + cnt) of a tensor with channel stride C,
// so skip concatenation costs nothing.  Channel counts used by the MFMA
// paths are multiples of 16.
//
// Convolution = implicit GEMM on the BF16 MFMAs:
//   forward  D[voxel][co] = sum_{tap, ci} X[p(voxel, tap)][ci] W[tap][ci][co]
//   dgrad    the same kernel on dY with flipped, transposed weights
//   wgrad    D[ci][co] += sum_voxel X[p(voxel, tap)][ci] dY[voxel][co]
// with tap geometries: 3^3 zero-padded ("c3"), 3^3 over a nearest x2
// upsampled input ("up"), 2^3 stride 2 ("down") and 1^3 ("c1").  The 3^3
// kinds with a multiple of 32 input channels, the 3^3 first layer over 8
// channels and every weight gradient run on v_mfma_f32_16x16x32_bf16
// (gfx950, twice the rate of the 16x16x16 form); the rest on
// v_mfma_f32_16x16x16bf16_1k.
// Operand lane layout (wave64, 16x16x16): A[i][k] sits in lane i + 16 (k/4),
// element k % 4; B[k][j] in lane j + 16 (k/4), element k % 4; D[i][j] in lane
// j + 16 (i/4), element i % 4.  16x16x32: A[i][k] in lane i + 16 (k/8),
// element k % 8; B[k][j] in lane j + 16 (k/8), element k % 8; D as above.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nn_kernels.hpp"

namespace nn {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));   // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);                                                                 // nearest even
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ int ksize(int kind) { return kind == KIND_C3 || kind == KIND_UP ? 3 : (kind == KIND_DOWN ? 2 : 1); }

// Input voxel read by output voxel (z, y, x) through tap (a, b, c); false if
// it lies in the zero padding.  (D, H, W) are the input's spatial sizes.
__device__ __forceinline__ bool tap_source(int kind, int z, int y, int x, int a, int b, int c, int D, int H, int W,
                                           int &sz, int &sy, int &sx)
{
    if (kind == KIND_C3) {
        sz = z + a - 1; sy = y + b - 1; sx = x + c - 1;
        return sz >= 0 && sy >= 0 && sx >= 0 && sz < D && sy < H && sx < W;
    }
    if (kind == KIND_UP) {
        int uz = z + a - 1, uy = y + b - 1, ux = x + c - 1;
        if (uz < 0 || uy < 0 || ux < 0 || uz >= 2 * D || uy >= 2 * H || ux >= 2 * W) return false;
        sz = uz >> 1; sy = uy >> 1; sx = ux >> 1;
        return true;
    }
    if (kind == KIND_DOWN) {
        sz = 2 * z + a; sy = 2 * y + b; sx = 2 * x + c;
        return true;
    }
    sz = z; sy = y; sx = x;
    return true;
}

// ---------------------------------------------------------------- convolution (forward / dgrad)
// One wave computes 64 consecutive output voxels (4 row fragments) x 16 NF
// output channels.
template <int NF>
__global__ __launch_bounds__(256) void k_conv(ConvArgs a)
{
    const int lane = threadIdx.x & 63;
    const long long wave = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const long long nvox = (long long)a.n * a.od * a.oh * a.ow;
    const long long v0 = wave * 64;
    if (v0 >= nvox) return;
    const int ks = ksize(a.kind);
    const int ntap = ks * ks * ks;
    const int kc = a.cin / 16;
    f4 acc[4][NF];
#pragma unroll
    for (int f = 0; f < 4; f++)
#pragma unroll
        for (int n = 0; n < NF; n++) acc[f][n] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    // coordinates of this lane's A rows (one voxel per fragment)
    int vz[4], vy[4], vx[4], vn[4];
    bool vok[4];
#pragma unroll
    for (int f = 0; f < 4; f++) {
        long long v = v0 + 16 * f + (lane & 15);
        vok[f] = v < nvox;
        if (!vok[f]) v = 0;
        vx[f] = (int)(v % a.ow);
        long long r = v / a.ow;
        vy[f] = (int)(r % a.oh);
        r /= a.oh;
        vz[f] = (int)(r % a.od);
        vn[f] = (int)(r / a.od);
    }
    const int kq = 4 * (lane >> 4);          // this lane's first K element within a fragment
    for (int t = 0; t < ntap; t++) {
        const int ta = t / (ks * ks), tb = (t / ks) % ks, tc = t % ks;
        long long src[4];
        bool ok[4];
#pragma unroll
        for (int f = 0; f < 4; f++) {
            int sz = 0, sy = 0, sx = 0;
            ok[f] = vok[f] && tap_source(a.kind, vz[f], vy[f], vx[f], ta, tb, tc, a.id, a.ih, a.iw, sz, sy, sx);
            src[f] = ok[f] ? ((((long long)vn[f] * a.id + sz) * a.ih + sy) * a.iw + sx) * a.cx + a.x_off + kq : 0;
        }
        const uint16_t *wt = a.w + (size_t)t * kc * NF * 256;
        for (int c = 0; c < kc; c++) {
            s4 A[4];
#pragma unroll
            for (int f = 0; f < 4; f++) {
                if (ok[f]) {
                    const uint2 raw = *(const uint2 *)(a.x + src[f] + 16 * c);
                    A[f] = s4{(short)(raw.x & 0xffff), (short)(raw.x >> 16), (short)(raw.y & 0xffff), (short)(raw.y >> 16)};
                } else {
                    A[f] = s4{0, 0, 0, 0};
                }
            }
#pragma unroll
            for (int n = 0; n < NF; n++) {
                const uint2 raw = *(const uint2 *)(wt + ((size_t)c * NF + n) * 256 + 4 * lane);
                const s4 Bv = s4{(short)(raw.x & 0xffff), (short)(raw.x >> 16), (short)(raw.y & 0xffff), (short)(raw.y >> 16)};
#pragma unroll
                for (int f = 0; f < 4; f++) acc[f][n] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A[f], Bv, acc[f][n], 0, 0, 0);
            }
        }
    }
    // epilogue: D[i][j] -> voxel v0 + 16 f + 4 (lane/16) + r, channel 16 n + lane % 16
#pragma unroll
    for (int f = 0; f < 4; f++)
#pragma unroll
        for (int n = 0; n < NF; n++) {
            const int co = 16 * n + (lane & 15);
            if (co >= a.cout) continue;
            const float bias = a.bias ? a.bias[co] : 0.0f;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const long long v = v0 + 16 * f + 4 * (lane >> 4) + r;
                if (v >= nvox) continue;
                float val = acc[f][n][r] + bias;
                if (a.relu) val = fmaxf(val, 0.0f);
                if (a.y) a.y[v * a.cy + a.y_off + co] = f2bf(val);
                if (a.y32) a.y32[v * a.cy32 + co] = val;
            }
        }
}

// ---------------------------------------------------------------- LDS-tiled convolution (3^3 and up)
// A workgroup computes a 4 x 4 x 16 (z, y, x) tile of output voxels for all
// output channels; wave w owns the z-slice w (4 row fragments of 16 x).  For
// every 16-channel chunk of the input, the tile's input halo is staged once
// in LDS (zero where the padding or the tensor edge is) and all 27 taps read
// their A fragments from it; weights come from the packed B fragments.
constexpr int TLZ = 4, TLY = 4, TLX = 16;
constexpr int HLZ = TLZ + 2, HLY = TLY + 2, HLX = TLX + 2;   // 3^3 halo (the up halo is smaller)

template <int NF, int KIND>
__global__ __launch_bounds__(256) void k_conv_lds(ConvArgs a)
{
    __shared__ uint2 halo[HLZ * HLY * HLX * 4];              // [voxel][4 x (4 bf16)]
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int tiles_x = (a.ow + TLX - 1) / TLX, tiles_y = (a.oh + TLY - 1) / TLY, tiles_z = (a.od + TLZ - 1) / TLZ;
    int b = blockIdx.x;
    const int bx = b % tiles_x;
    b /= tiles_x;
    const int by = b % tiles_y;
    b /= tiles_y;
    const int bz = b % tiles_z;
    const int bn = b / tiles_z;
    const int z0 = bz * TLZ, y0 = by * TLY, x0 = bx * TLX;
    // input-space origin and extent of the halo
    int hz0, hy0, hx0, hz, hy, hx;
    if (KIND == KIND_C3) {
        hz0 = z0 - 1; hy0 = y0 - 1; hx0 = x0 - 1;
        hz = HLZ; hy = HLY; hx = HLX;
    } else {   // nearest x2 upsampled input: fine u = o + t - 1 reads coarse u >> 1
        hz0 = (z0 >> 1) - 1; hy0 = (y0 >> 1) - 1; hx0 = (x0 >> 1) - 1;
        hz = TLZ / 2 + 2; hy = TLY / 2 + 2; hx = TLX / 2 + 2;
    }
    const int nh = hz * hy * hx;
    f4 acc[4][NF];
#pragma unroll
    for (int f = 0; f < 4; f++)
#pragma unroll
        for (int n = 0; n < NF; n++) acc[f][n] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    const int kc = a.cin / 16;
    const int q = lane >> 4, i = lane & 15;
    for (int c = 0; c < kc; c++) {
        // stage the halo of input channels [16 c, 16 c + 16)
        for (int e = threadIdx.x; e < nh * 4; e += 256) {
            const int v = e >> 2, qq = e & 3;
            const int lx = v % hx, ly = (v / hx) % hy, lz = v / (hx * hy);
            const int gz = hz0 + lz, gy = hy0 + ly, gx = hx0 + lx;
            uint2 val = make_uint2(0u, 0u);
            if (gz >= 0 && gy >= 0 && gx >= 0 && gz < a.id && gy < a.ih && gx < a.iw)
                val = *(const uint2 *)(a.x + ((((long long)bn * a.id + gz) * a.ih + gy) * a.iw + gx) * a.cx + a.x_off +
                                       16 * c + 4 * qq);
            halo[e] = val;
        }
        __syncthreads();
        const uint16_t *wc = a.w + (size_t)c * NF * 256 + 4 * lane;
        for (int t = 0; t < 27; t++) {
            const int ta = t / 9, tb = (t / 3) % 3, tc = t % 3;
            s4 Af[4];
#pragma unroll
            for (int f = 0; f < 4; f++) {
                int lz, ly, lx;
                if (KIND == KIND_C3) {
                    lz = wv + ta; ly = f + tb; lx = i + tc;
                } else {
                    lz = ((z0 + wv + ta - 1) >> 1) - hz0;
                    ly = ((y0 + f + tb - 1) >> 1) - hy0;
                    lx = ((x0 + i + tc - 1) >> 1) - hx0;
                }
                const uint2 raw = halo[((lz * hy + ly) * hx + lx) * 4 + q];
                Af[f] = s4{(short)(raw.x & 0xffff), (short)(raw.x >> 16), (short)(raw.y & 0xffff), (short)(raw.y >> 16)};
            }
            const uint16_t *wt = wc + (size_t)t * kc * NF * 256;
#pragma unroll
            for (int n = 0; n < NF; n++) {
                const uint2 raw = *(const uint2 *)(wt + (size_t)n * 256);
                const s4 Bv = s4{(short)(raw.x & 0xffff), (short)(raw.x >> 16), (short)(raw.y & 0xffff), (short)(raw.y >> 16)};
#pragma unroll
                for (int f = 0; f < 4; f++) acc[f][n] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(Af[f], Bv, acc[f][n], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // epilogue: fragment f = output row y0 + f, D[i][j] -> x = x0 + 4 (lane/16) + r, channel 16 n + lane % 16
    const int oz = z0 + wv;
#pragma unroll
    for (int f = 0; f < 4; f++) {
        const int oy = y0 + f;
        if (oz >= a.od || oy >= a.oh) continue;
#pragma unroll
        for (int n = 0; n < NF; n++) {
            const int co = 16 * n + (lane & 15);
            if (co >= a.cout) continue;
            const float bias = a.bias ? a.bias[co] : 0.0f;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int ox = x0 + 4 * (lane >> 4) + r;
                if (ox >= a.ow) continue;
                const long long v = (((long long)bn * a.od + oz) * a.oh + oy) * a.ow + ox;
                float val = acc[f][n][r] + bias;
                if (a.relu) val = fmaxf(val, 0.0f);
                if (a.y) a.y[v * a.cy + a.y_off + co] = f2bf(val);
                if (a.y32) a.y32[v * a.cy32 + co] = val;
            }
        }
    }
}

// Epilogue of the LDS-tiled kernels: bias, ReLU and the outputs of a 4 x 4 x 16
// tile (wave wv owns z-slice wv, fragment f row f, lane (i, g) voxels 4 g + r
// of channel 16 n + i).  A BF16-only output slice (cout = 16 NF, 16-byte
// aligned rows) goes through `ot` (LDS, >= 256 x (16 min(NF, 4) + 8) BF16,
// free after the last barrier) and out as 16-byte rows.
// Output channels per LDS pass of conv_store's fast path (its rows of 64 FR
// voxels x (channels + 8) BF16 must fit the caller's LDS buffer).
template <int NF, int FR>
constexpr int store_pass_channels()
{
    return 16 * NF < (FR == 8 ? 32 : 64) ? 16 * NF : (FR == 8 ? 32 : 64);
}

// Epilogue of the tiled convolutions: wave wv holds FR rows (y) of 16 x
// voxels of the z-slice z0 + wv, for all output channels.
template <int NF, int FR = 4>
__device__ __forceinline__ void conv_store(const ConvArgs &a, f4 (&acc)[FR][NF], int bn, int z0, int y0, int x0, int wv,
                                           int lane, uint16_t *ot)
{
    constexpr int CO = 16 * NF;
    const int g = lane >> 4, i = lane & 15;
    const int oz = z0 + wv;
    const bool fast = a.y && !a.y32 && a.cout == CO && (a.cy % 8) == 0 && (a.y_off % 8) == 0 &&
                      ((uintptr_t)a.y & 15) == 0;
    if (fast) {
        // D[i][j] -> LDS row (wave, f, x = 4 (lane / 16) + r), channel 16 n + lane % 16; then 16-byte rows out
        constexpr int CP = store_pass_channels<NF, FR>();
        constexpr int NP = CO / CP;                           // channel passes
        constexpr int PROW = CP + 8;
#pragma unroll
        for (int pass = 0; pass < NP; pass++) {
#pragma unroll
            for (int f = 0; f < FR; f++)
#pragma unroll
                for (int nn = 0; nn < NF / NP; nn++) {
                    const int n = pass * (NF / NP) + nn;
                    const float bias = a.bias ? a.bias[16 * n + i] : 0.0f;
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        float val = acc[f][n][r] + bias;
                        if (a.relu) val = fmaxf(val, 0.0f);
                        ot[((wv * FR + f) * 16 + 4 * g + r) * PROW + 16 * nn + i] = f2bf(val);
                    }
                }
            __syncthreads();
            for (int e = threadIdx.x; e < 64 * FR * (CP / 8); e += 256) {
                const int vl = e / (CP / 8), part = e % (CP / 8);
                const int tz = vl / (16 * FR), ty = (vl >> 4) % FR, tx = vl & 15;
                const int gz = z0 + tz, gy = y0 + ty, gx = x0 + tx;
                if (gz < a.od && gy < a.oh && gx < a.ow) {
                    const long long gv = (((long long)bn * a.od + gz) * a.oh + gy) * a.ow + gx;
                    *(uint4 *)(a.y + gv * a.cy + a.y_off + pass * CP + 8 * part) = *(const uint4 *)(ot + vl * PROW + 8 * part);
                }
            }
            if (pass + 1 < NP) __syncthreads();
        }
        return;
    }
#pragma unroll
    for (int f = 0; f < FR; f++) {
        const int oy = y0 + f;
        if (oz >= a.od || oy >= a.oh) continue;
#pragma unroll
        for (int n = 0; n < NF; n++) {
            const int co = 16 * n + (lane & 15);
            if (co >= a.cout) continue;
            const float bias = a.bias ? a.bias[co] : 0.0f;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int ox = x0 + 4 * (lane >> 4) + r;
                if (ox >= a.ow) continue;
                const long long v = (((long long)bn * a.od + oz) * a.oh + oy) * a.ow + ox;
                float val = acc[f][n][r] + bias;
                if (a.relu) val = fmaxf(val, 0.0f);
                if (a.y) a.y[v * a.cy + a.y_off + co] = f2bf(val);
                if (a.y32) a.y32[v * a.cy32 + co] = val;
            }
        }
    }
}

// The same tiling on v_mfma_f32_16x16x32_bf16 for a multiple of 32 input
// channels.  K slot e of lane group g (= lane / 16) carries channel 8 g + e of
// the 32-channel chunk, for A (halo) and B (packed weights) alike.  The halo
// holds, per voxel, the chunk's four 16-byte pieces (channels 8 p .. 8 p + 7),
// piece p stored at slot p ^ ((v >> 2) & 3) so that the 16-byte reads of 8
// neighbouring x voxels hit distinct banks.  For each (z tap, x tap) a wave
// reads the six halo rows its four output rows see through the three y taps
// once.  With 16-byte aligned channel slices (x16) the halo is staged by
// 16-byte global-to-LDS copies (global_load_lds_dwordx4): each wave
// instruction fills 64 consecutive slots, lane L slot 64 j + L, so every load
// of a chunk is in flight at once and no register holds the data; voxels in
// the padding copy from a zero block.  A BF16 output slice goes out through
// LDS as 16-byte rows (needs the channel stride and offset of x and y to be
// multiples of 8).
typedef __bf16 b8 __attribute__((ext_vector_type(8)));

__device__ __align__(16) uint16_t g_zero_piece[8];   // 16 zero bytes: the source of padding voxels

// FR: output rows (y) per wave, 4 or 8 (tile 4 x FR x 16).  Every B fragment
// (weights, read through the vector cache) feeds FR MFMAs; at FR = 4 those
// reads alone would use the cache's whole bandwidth at the MFMA rate (a
// timing-only build that skips them runs the forward 1.4x faster).
template <int NF, int KIND, bool X16, int FR>
__global__ __launch_bounds__(256, 2) void k_conv_lds32(ConvArgs a)
{
    constexpr int HZ = KIND == KIND_C3 ? HLZ : TLZ / 2 + 2;
    constexpr int HY = KIND == KIND_C3 ? FR + 2 : FR / 2 + 2;
    constexpr int HX = KIND == KIND_C3 ? HLX : TLX / 2 + 2;
    constexpr int NH = HZ * HY * HX;
    constexpr int HBUF = HLZ * (FR + 2) * HLX * 4;   // uint4 slots of the largest (3^3) halo
    static_assert(64 * FR * (store_pass_channels<NF, FR>() + 8) * 2 <= HBUF * 16, "output rows must fit the halo buffer");
    __shared__ uint4 halo[HBUF];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int tiles_x = (a.ow + TLX - 1) / TLX, tiles_y = (a.oh + FR - 1) / FR, tiles_z = (a.od + TLZ - 1) / TLZ;
    int b = blockIdx.x;
    const int bx = b % tiles_x;
    b /= tiles_x;
    const int by = b % tiles_y;
    b /= tiles_y;
    const int bz = b % tiles_z;
    const int bn = b / tiles_z;
    const int z0 = bz * TLZ, y0 = by * FR, x0 = bx * TLX;
    int hz0, hy0, hx0;
    if (KIND == KIND_C3) {
        hz0 = z0 - 1; hy0 = y0 - 1; hx0 = x0 - 1;
    } else {
        hz0 = (z0 >> 1) - 1; hy0 = (y0 >> 1) - 1; hx0 = (x0 >> 1) - 1;
    }
    f4 acc[FR][NF];
#pragma unroll
    for (int f = 0; f < FR; f++)
#pragma unroll
        for (int n = 0; n < NF; n++) acc[f][n] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    const int kc = a.cin / 32;
    const int g = lane >> 4, i = lane & 15;
    uint2 *h2 = (uint2 *)halo;
    const uint16_t *xb = a.x + (long long)bn * a.id * a.ih * a.iw * a.cx + a.x_off;
    for (int c = 0; c < kc; c++) {
        if (X16) {
            typedef __attribute__((address_space(3))) void lds_void;
            typedef const __attribute__((address_space(1))) void glob_void;
            for (int j = wv; j * 64 < 4 * NH; j += 4) {
                const int slot = 64 * j + lane;
                if (slot < 4 * NH) {
                    const int v = slot >> 2, p = (slot & 3) ^ ((v >> 2) & 3);
                    const int lx = v % HX, ly = (v / HX) % HY, lz = v / (HX * HY);
                    const int gz = hz0 + lz, gy = hy0 + ly, gx = hx0 + lx;
                    const bool in = gz >= 0 && gy >= 0 && gx >= 0 && gz < a.id && gy < a.ih && gx < a.iw;
                    const uint16_t *src =
                        in ? xb + (((long long)gz * a.ih + gy) * a.iw + gx) * a.cx + 32 * c + 8 * p : g_zero_piece;
                    __builtin_amdgcn_global_load_lds((glob_void *)src, (lds_void *)(halo + 64 * j), 16, 0, 0);
                }
            }
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // the copies are not tracked by the compiler
        } else {
            // 4 channels per load, thread t: channels 4 (t & 7) .. + 3 of voxels (t >> 3) + 32 k
            const int q = threadIdx.x & 7;
            for (int v = threadIdx.x >> 3; v < NH; v += 32) {
                const int lx = v % HX, ly = (v / HX) % HY, lz = v / (HX * HY);
                const int gz = hz0 + lz, gy = hy0 + ly, gx = hx0 + lx;
                const bool in = gz >= 0 && gy >= 0 && gx >= 0 && gz < a.id && gy < a.ih && gx < a.iw;
                const long long off = (((long long)gz * a.ih + gy) * a.iw + gx) * a.cx + 32 * c + 4 * q;
                uint2 val = make_uint2(0u, 0u);
                if (in) val = *(const uint2 *)(xb + off);
                h2[v * 8 + 2 * ((q >> 1) ^ ((v >> 2) & 3)) + (q & 1)] = val;
            }
        }
        __syncthreads();
        const uint16_t *wc = a.w + (size_t)c * NF * 512 + 8 * lane;
#pragma unroll 1
        for (int ta = 0; ta < 3; ta++) {
            int lz;
            if (KIND == KIND_C3) lz = wv + ta;
            else lz = ((z0 + wv + ta - 1) >> 1) - hz0;
#pragma unroll 1
            for (int tc = 0; tc < 3; tc++) {
                int lx;
                if (KIND == KIND_C3) lx = i + tc;
                else lx = ((x0 + i + tc - 1) >> 1) - hx0;
                b8 Ar[FR + 2];
#pragma unroll
                for (int r = 0; r < FR + 2; r++) {
                    int ly;
                    if (KIND == KIND_C3) ly = r;
                    else ly = ((y0 + r - 1) >> 1) - hy0;
                    const int v = (lz * HY + ly) * HX + lx;
                    Ar[r] = __builtin_bit_cast(b8, halo[v * 4 + (g ^ ((v >> 2) & 3))]);
                }
#pragma unroll
                for (int tb = 0; tb < 3; tb++) {
                    const int t = (ta * 3 + tb) * 3 + tc;
                    const uint16_t *wt = wc + (size_t)t * kc * NF * 512;
#pragma unroll
                    for (int n = 0; n < NF; n++) {
                        const b8 Bv = __builtin_bit_cast(b8, *(const uint4 *)(wt + (size_t)n * 512));
#pragma unroll
                        for (int f = 0; f < FR; f++)
                            acc[f][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ar[f + tb], Bv, acc[f][n], 0, 0, 0);
                    }
                }
            }
        }
        __syncthreads();
    }
    conv_store<NF, FR>(a, acc, bn, z0, y0, x0, wv, lane, (uint16_t *)halo);
}

// First layer: 3^3 convolution over 8 input channels with the taps folded
// into K.  K step c (32 wide) covers taps 4 c .. 4 c + 3: lane group g takes
// tap 4 c + g and its 8 elements are the 8 channels of that tap's input voxel
// (one 16-byte LDS read); 7 steps cover the 27 taps (the 28th has zero
// weights and reads tap 26's voxel).  The halo holds 8 channels per voxel.
constexpr int FIRST_STEPS = 7;

template <int NF>
__global__ __launch_bounds__(256, 2) void k_conv_first(ConvArgs a)
{
    constexpr int NH = HLZ * HLY * HLX;
    constexpr int OBUF = (256 * (16 * (NF < 4 ? NF : 4) + 8) * 2 + 15) / 16;   // epilogue rows, in uint4
    __shared__ uint4 lds[NH > OBUF ? NH : OBUF];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int tiles_x = (a.ow + TLX - 1) / TLX, tiles_y = (a.oh + TLY - 1) / TLY, tiles_z = (a.od + TLZ - 1) / TLZ;
    int b = blockIdx.x;
    const int bx = b % tiles_x;
    b /= tiles_x;
    const int by = b % tiles_y;
    b /= tiles_y;
    const int bz = b % tiles_z;
    const int bn = b / tiles_z;
    const int z0 = bz * TLZ, y0 = by * TLY, x0 = bx * TLX;
    const uint16_t *xb = a.x + (long long)bn * a.id * a.ih * a.iw * a.cx + a.x_off;
    for (int v = threadIdx.x; v < NH; v += 256) {
        const int lx = v % HLX, ly = (v / HLX) % HLY, lz = v / (HLX * HLY);
        const int gz = z0 - 1 + lz, gy = y0 - 1 + ly, gx = x0 - 1 + lx;
        uint4 val = make_uint4(0u, 0u, 0u, 0u);
        if (gz >= 0 && gy >= 0 && gx >= 0 && gz < a.id && gy < a.ih && gx < a.iw)
            val = *(const uint4 *)(xb + (((long long)gz * a.ih + gy) * a.iw + gx) * a.cx);
        lds[v] = val;
    }
    __syncthreads();
    f4 acc[4][NF];
#pragma unroll
    for (int f = 0; f < 4; f++)
#pragma unroll
        for (int n = 0; n < NF; n++) acc[f][n] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    const int g = lane >> 4, i = lane & 15;
#pragma unroll
    for (int c = 0; c < FIRST_STEPS; c++) {
        const int t = min(4 * c + g, 26);
        const int ta = t / 9, tb = (t / 3) % 3, tc = t % 3;
        b8 A[4];
#pragma unroll
        for (int f = 0; f < 4; f++) A[f] = __builtin_bit_cast(b8, lds[((wv + ta) * HLY + f + tb) * HLX + i + tc]);
#pragma unroll
        for (int n = 0; n < NF; n++) {
            const b8 Bv = __builtin_bit_cast(b8, *(const uint4 *)(a.w + ((size_t)(c * NF + n) * 64 + lane) * 8));
#pragma unroll
            for (int f = 0; f < 4; f++) acc[f][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[f], Bv, acc[f][n], 0, 0, 0);
        }
    }
    __syncthreads();   // the epilogue reuses the halo's LDS
    conv_store<NF>(a, acc, bn, z0, y0, x0, wv, lane, (uint16_t *)lds);
}

// Pack FP32 master weights W[tap][ci][co] (ci < cin, co < cout) into the
// B-fragment order the conv kernel reads, as BF16; `transpose` packs the
// weights of the adjoint (dgrad) convolution: taps mirrored, ci <-> co.
//   k32 = 0: element (((t * KC + c) * NF + n) * 64 + lane) * 4 + r holds
//            B[k][j], k = 16 c + 4 (lane / 16) + r (16x16x16 fragments);
//   k32 = 1: element (((t * KC2 + c) * NF + n) * 64 + lane) * 8 + e holds
//            k = 32 c + 8 (lane / 16) + e (16x16x32 fragments).
//   k32 = 2: the first-layer order (8 input channels, taps folded into K):
//            element ((c * NF + n) * 64 + lane) * 8 + j holds tap 4 c + lane / 16
//            (zero for tap 27), channel j.
__global__ void k_pack(const float *w, int ntap, int cin, int cout, int cin_p, int cout_p, int transpose, int k32,
                       uint16_t *out)
{
    const int KC = cin_p / 16, NF = cout_p / 16;
    const long long total = k32 == 2 ? (long long)FIRST_STEPS * NF * 512 : (long long)ntap * KC * NF * 256;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
        int k, lane, n, t;
        if (k32 == 2) {
            const int j = (int)(e & 7);
            lane = (int)((e >> 3) & 63);
            const long long q = e >> 9;
            n = (int)(q % NF);
            t = 4 * (int)(q / NF) + (lane >> 4);
            const int co = 16 * n + (lane & 15);
            out[e] = f2bf(t < 27 && j < cin && co < cout ? w[((long long)t * cin + j) * cout + co] : 0.0f);
            continue;
        }
        if (!k32) {
            const int r = (int)(e & 3);
            lane = (int)((e >> 2) & 63);
            long long q = e >> 8;
            n = (int)(q % NF);
            q /= NF;
            const int c = (int)(q % KC);
            t = (int)(q / KC);
            k = 16 * c + 4 * (lane >> 4) + r;             // input channel of this conv
        } else {
            const int el = (int)(e & 7);
            lane = (int)((e >> 3) & 63);
            long long q = e >> 9;
            n = (int)(q % NF);
            q /= NF;
            const int c = (int)(q % (KC / 2));
            t = (int)(q / (KC / 2));
            k = 32 * c + 8 * (lane >> 4) + el;
        }
        const int j = 16 * n + (lane & 15);              // output channel of this conv
        float v = 0.0f;
        if (!transpose) {
            if (k < cin && j < cout) v = w[((long long)t * cin + k) * cout + j];
        } else {
            // adjoint: this conv maps cout-channel gradients to cin-channel ones
            const int tm = ntap - 1 - t;
            if (k < cout && j < cin) v = w[((long long)tm * cin + j) * cout + k];
        }
        out[e] = f2bf(v);
    }
}

// ---------------------------------------------------------------- weight gradient
// Partial dW for one tap and one chunk of output voxels:
//   P[chunk][tap][ci][co] = sum_{v in chunk} X[p(v, tap)][ci] dY[v][co]
// Wave w of the workgroup owns input-channel fragments w, w + 4, ...
template <int NF>
__global__ __launch_bounds__(256) void k_wgrad(WgradArgs a)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ks = ksize(a.kind), ntap = ks * ks * ks;
    const int t = blockIdx.x % ntap;
    const int chunk = blockIdx.x / ntap;
    const long long nvox = (long long)a.n * a.od * a.oh * a.ow;
    const long long vb = (long long)chunk * a.chunk, ve = min(nvox, vb + a.chunk);
    const int ta = t / (ks * ks), tb = (t / ks) % ks, tc = t % ks;
    const int KC = a.cin / 16;
    constexpr int MF = 2;      // input-channel fragments per wave (cin <= 128)
    f4 acc[MF][NF];
#pragma unroll
    for (int m = 0; m < MF; m++)
#pragma unroll
        for (int n = 0; n < NF; n++) acc[m][n] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    const int kq = 8 * (lane >> 4);
    for (long long v0 = vb; v0 < ve; v0 += 32) {
        // K = 32 voxels (16x16x32 MFMA); this lane supplies voxels v0 + kq .. + 7
        long long src[8], dst[8];
        bool ok[8];
#pragma unroll
        for (int r = 0; r < 8; r++) {
            long long v = v0 + kq + r;
            ok[r] = v < ve;
            if (!ok[r]) v = vb;
            int x = (int)(v % a.ow);
            long long q = v / a.ow;
            int y = (int)(q % a.oh);
            q /= a.oh;
            int z = (int)(q % a.od);
            int nn = (int)(q / a.od);
            int sz = 0, sy = 0, sx = 0;
            ok[r] = ok[r] && tap_source(a.kind, z, y, x, ta, tb, tc, a.id, a.ih, a.iw, sz, sy, sx);
            src[r] = ((((long long)nn * a.id + sz) * a.ih + sy) * a.iw + sx) * a.cx + a.x_off;
            dst[r] = v * a.cg + a.g_off;
            if (!(v0 + kq + r < ve)) dst[r] = -1;
        }
        b8 Bv[NF];
#pragma unroll
        for (int n = 0; n < NF; n++) {
            const int co = 16 * n + (lane & 15);
            s8 b;
#pragma unroll
            for (int r = 0; r < 8; r++) b[r] = (dst[r] >= 0 && co < a.cout) ? (short)a.g[dst[r] + co] : (short)0;
            Bv[n] = __builtin_bit_cast(b8, b);
        }
#pragma unroll
        for (int m = 0; m < MF; m++) {
            const int cf = wv + 4 * m;
            if (cf >= KC) continue;
            const int ci = 16 * cf + (lane & 15);
            s8 Av;
#pragma unroll
            for (int r = 0; r < 8; r++) Av[r] = ok[r] ? (short)a.x[src[r] + ci] : (short)0;
            const b8 Ab = __builtin_bit_cast(b8, Av);
#pragma unroll
            for (int n = 0; n < NF; n++) acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ab, Bv[n], acc[m][n], 0, 0, 0);
        }
    }
    float *P = a.partial + (((long long)chunk * ntap + t) * a.cin) * a.cout;
#pragma unroll
    for (int m = 0; m < MF; m++) {
        const int cf = wv + 4 * m;
        if (cf >= KC) continue;
#pragma unroll
        for (int n = 0; n < NF; n++) {
            const int co = 16 * n + (lane & 15);
            if (co >= a.cout) continue;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int ci = 16 * cf + 4 * (lane >> 4) + r;
                P[(long long)ci * a.cout + co] = acc[m][n][r];
            }
        }
    }
}

// LDS-tiled weight gradient (3^3 and up kinds).  Workgroup (group, cf, tg):
// the output tiles [group * tpg, (group + 1) * tpg), input channels
// [16 cf, 16 cf + 16) and taps [8 tg, 8 tg + 8).  Per tile it stages the
// input halo channel-major (xh[ci][halo voxel]) and the output-gradient tile
// voxel-packed (gt[co][4-voxel pack]); wave w owns taps 8 tg + w and
// 8 tg + w + 4 and accumulates, over the tile's voxels (K = 32 voxels = two
// x rows per MFMA), D[ci][co] += sum_v X[v + tap][ci] dY[v][co].  The partial
// of the group goes to P[group][tap][ci][co].
template <int NF, int KIND>
__global__ __launch_bounds__(256) void k_wgrad_lds(WgradArgs a, int tpg, int ntiles)
{
    constexpr int TZ = NF == 8 ? 2 : 4;            // tile depth (LDS budget of the gradient tile)
    constexpr int TV = TZ * TLY * TLX;             // tile voxels
    constexpr int HZ = TZ + 2;
    __shared__ unsigned short xh[16 * HZ * HLY * HLX];
    __shared__ uint2 gt[NF * 16 * (TV / 4)];
    unsigned short *gts = (unsigned short *)gt;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int cf = blockIdx.y, tg = blockIdx.z;
    const int tiles_x = (a.ow + TLX - 1) / TLX, tiles_y = (a.oh + TLY - 1) / TLY, tiles_z = (a.od + TZ - 1) / TZ;
    int hz, hy, hx;
    if (KIND == KIND_C3) { hz = HZ; hy = HLY; hx = HLX; }
    else { hz = TZ / 2 + 2; hy = TLY / 2 + 2; hx = TLX / 2 + 2; }
    const int nh = hz * hy * hx;
    const int t0 = 8 * tg + wv, t1 = t0 + 4;
    const int tmax = min(27, 8 * tg + 8);
    f4 acc[2][NF];
#pragma unroll
    for (int u = 0; u < 2; u++)
#pragma unroll
        for (int n = 0; n < NF; n++) acc[u][n] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    const int q = lane >> 4, i = lane & 15;
    const int tile_end = min(ntiles, (int)(blockIdx.x + 1) * tpg);
    for (int tile = blockIdx.x * tpg; tile < tile_end; tile++) {
        int b = tile;
        const int bx = b % tiles_x;
        b /= tiles_x;
        const int by = b % tiles_y;
        b /= tiles_y;
        const int bz = b % tiles_z;
        const int bn = b / tiles_z;
        const int z0 = bz * TZ, y0 = by * TLY, x0 = bx * TLX;
        int hz0, hy0, hx0;
        if (KIND == KIND_C3) { hz0 = z0 - 1; hy0 = y0 - 1; hx0 = x0 - 1; }
        else { hz0 = (z0 >> 1) - 1; hy0 = (y0 >> 1) - 1; hx0 = (x0 >> 1) - 1; }
        // input halo, channels [16 cf, 16 cf + 16), stored channel-major
        for (int e = threadIdx.x; e < nh * 4; e += 256) {
            const int v = e >> 2, qq = e & 3;
            const int lx = v % hx, ly = (v / hx) % hy, lz = v / (hx * hy);
            const int gz = hz0 + lz, gy = hy0 + ly, gx = hx0 + lx;
            uint2 val = make_uint2(0u, 0u);
            if (gz >= 0 && gy >= 0 && gx >= 0 && gz < a.id && gy < a.ih && gx < a.iw)
                val = *(const uint2 *)(a.x + ((((long long)bn * a.id + gz) * a.ih + gy) * a.iw + gx) * a.cx + a.x_off +
                                       16 * cf + 4 * qq);
            const int c0 = 4 * qq;
            xh[(c0 + 0) * nh + v] = (unsigned short)(val.x & 0xffff);
            xh[(c0 + 1) * nh + v] = (unsigned short)(val.x >> 16);
            xh[(c0 + 2) * nh + v] = (unsigned short)(val.y & 0xffff);
            xh[(c0 + 3) * nh + v] = (unsigned short)(val.y >> 16);
        }
        // output-gradient tile, [co][voxel]
        for (int e = threadIdx.x; e < TV * NF * 4; e += 256) {
            const int v = e / (NF * 4), qq = e % (NF * 4);
            const int tx = v % TLX, ty = (v / TLX) % TLY, tz = v / (TLX * TLY);
            const int oz = z0 + tz, oy = y0 + ty, ox = x0 + tx;
            const int c0 = 4 * qq;
            unsigned short w4[4] = {0, 0, 0, 0};
            if (oz < a.od && oy < a.oh && ox < a.ow) {
                const long long gv = (((long long)bn * a.od + oz) * a.oh + oy) * a.ow + ox;
                const uint16_t *gp = a.g + gv * a.cg + a.g_off + c0;
                for (int k = 0; k < 4; k++) w4[k] = (c0 + k < a.cout) ? gp[k] : (unsigned short)0;
            }
            for (int k = 0; k < 4; k++) gts[(c0 + k) * TV + v] = w4[k];
        }
        __syncthreads();
        // two tile rows per 16x16x32 MFMA: K slot 4 h + r of lane group q is voxel
        // (row + h, x = 4 q + r) for both operands (K is summed over, so any
        // common order of the 32 voxels will do)
        for (int row = 0; row < TZ * TLY; row += 2) {
            b8 Bv[NF];
#pragma unroll
            for (int n = 0; n < NF; n++) {
                const uint2 r0 = gt[(16 * n + i) * (TV / 4) + (row * TLX + 4 * q) / 4];
                const uint2 r1 = gt[(16 * n + i) * (TV / 4) + ((row + 1) * TLX + 4 * q) / 4];
                Bv[n] = __builtin_bit_cast(b8, make_uint4(r0.x, r0.y, r1.x, r1.y));
            }
#pragma unroll
            for (int u = 0; u < 2; u++) {
                const int t = u ? t1 : t0;
                if (t >= tmax) continue;
                const int ta = t / 9, tb = (t / 3) % 3, tc = t % 3;
                s8 Av;
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    const int tz = (row + h) / TLY, ty = (row + h) % TLY;
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        const int tx = 4 * q + r;
                        int lz, ly, lx;
                        if (KIND == KIND_C3) { lz = tz + ta; ly = ty + tb; lx = tx + tc; }
                        else {
                            lz = ((z0 + tz + ta - 1) >> 1) - hz0;
                            ly = ((y0 + ty + tb - 1) >> 1) - hy0;
                            lx = ((x0 + tx + tc - 1) >> 1) - hx0;
                        }
                        Av[4 * h + r] = (short)xh[i * nh + (lz * hy + ly) * hx + lx];
                    }
                }
                const b8 Ab = __builtin_bit_cast(b8, Av);
#pragma unroll
                for (int n = 0; n < NF; n++) acc[u][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ab, Bv[n], acc[u][n], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // D[i][j]: ci = 16 cf + 4 (lane / 16) + r, co = 16 n + lane % 16
#pragma unroll
    for (int u = 0; u < 2; u++) {
        const int t = u ? t1 : t0;
        if (t >= tmax) continue;
        float *P = a.partial + ((long long)blockIdx.x * 27 + t) * a.cin * a.cout;
#pragma unroll
        for (int n = 0; n < NF; n++) {
            const int co = 16 * n + (lane & 15);
            if (co >= a.cout) continue;
#pragma unroll
            for (int r = 0; r < 4; r++) P[(long long)(16 * cf + 4 * (lane >> 4) + r) * a.cout + co] = acc[u][n][r];
        }
    }
}

__global__ void k_reduce_partials(const float *partial, int nchunk, long long per, float *out, int accumulate)
{
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < per; e += (long long)gridDim.x * blockDim.x) {
        float s = accumulate ? out[e] : 0.0f;
        for (int c = 0; c < nchunk; c++) s += partial[(long long)c * per + e];
        out[e] = s;
    }
}

// bias gradient: gb[co] (+)= sum over voxels of dY[v][co].  Each workgroup
// sums a chunk of voxels for every channel (consecutive threads read
// consecutive channels of a voxel), reduces in LDS and adds its partial sums
// with one float atomic per channel; gb is cleared first unless accumulating.
constexpr int BIAS_CHUNK = 8192;

__global__ void k_fill_f(float *p, int n, float v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void k_bias_grad(const uint16_t *g, long long nvox, int cg, int g_off, int cout,
                                                   float *gb)
{
    __shared__ float red[256];
    const int vl = 256 / cout;                       // voxel lanes (cout <= 128)
    const int co = threadIdx.x % cout, lv = threadIdx.x / cout;
    const long long v0 = (long long)blockIdx.x * BIAS_CHUNK, v1 = min(nvox, v0 + BIAS_CHUNK);
    float sum = 0.0f;
    if (lv < vl)
        for (long long v = v0 + lv; v < v1; v += vl) sum += bf2f(g[v * cg + g_off + co]);
    red[threadIdx.x] = lv < vl ? sum : 0.0f;
    __syncthreads();
    if (threadIdx.x < cout) {
        float t = 0.0f;
        for (int k = 0; k < vl; k++) t += red[k * cout + threadIdx.x];
        atomicAdd(gb + threadIdx.x, t);
    }
}

// The same sum with 4 channels per thread (8-byte loads) and four voxels in
// flight per thread; needs cout, cg and g_off multiples of 4.
__global__ __launch_bounds__(256) void k_bias_grad4(const uint16_t *g, long long nvox, int cg, int g_off, int cout,
                                                    float *gb)
{
    __shared__ float red[256 * 4];
    const int cq = cout / 4;                         // threads per voxel
    const int vl = 256 / cq;                         // voxel lanes
    const int q = threadIdx.x % cq, lv = threadIdx.x / cq;
    const long long v0 = (long long)blockIdx.x * BIAS_CHUNK, v1 = min(nvox, v0 + BIAS_CHUNK);
    float sum[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (lv < vl) {
        const uint16_t *gp = g + g_off + 4 * q;
        long long v = v0 + lv;
        for (; v + 3 * vl < v1; v += 4 * vl) {
            uint2 r[4];
#pragma unroll
            for (int u = 0; u < 4; u++) r[u] = *(const uint2 *)(gp + (v + u * vl) * cg);
#pragma unroll
            for (int u = 0; u < 4; u++) {
                sum[0] += __uint_as_float(r[u].x << 16);
                sum[1] += __uint_as_float(r[u].x & 0xffff0000u);
                sum[2] += __uint_as_float(r[u].y << 16);
                sum[3] += __uint_as_float(r[u].y & 0xffff0000u);
            }
        }
        for (; v < v1; v += vl) {
            const uint2 r = *(const uint2 *)(gp + v * cg);
            sum[0] += __uint_as_float(r.x << 16);
            sum[1] += __uint_as_float(r.x & 0xffff0000u);
            sum[2] += __uint_as_float(r.y << 16);
            sum[3] += __uint_as_float(r.y & 0xffff0000u);
        }
    }
#pragma unroll
    for (int k = 0; k < 4; k++) red[k * 256 + threadIdx.x] = lv < vl ? sum[k] : 0.0f;
    __syncthreads();
    if (threadIdx.x < cout) {
        const int co = threadIdx.x, qq = co / 4, k = co % 4;
        float t = 0.0f;
        for (int l = 0; l < vl; l++) t += red[k * 256 + l * cq + qq];
        atomicAdd(gb + co, t);
    }
}

// ---------------------------------------------------------------- elementwise and resampling
// g <- g * (y > 0) over a channel slice (ReLU backward; y is the layer output)
__global__ void k_relu_bwd(uint16_t *g, int cg, int g_off, const uint16_t *y, int cy, int y_off, long long nvox, int c)
{
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nvox * c; e += (long long)gridDim.x * blockDim.x) {
        long long v = e / c;
        int ch = (int)(e % c);
        if (!(bf2f(y[v * cy + y_off + ch]) > 0.0f)) g[v * cg + g_off + ch] = 0;
    }
}

// coarse[U] = sum of the 8 fine children (nearest-upsampling backward)
__global__ void k_up_bwd(const uint16_t *fine, int cf, int f_off, uint16_t *coarse, int cc, int c_off, int n, int d, int h,
                         int w, int c)
{
    const long long total = (long long)n * d * h * w * c;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
        int ch = (int)(e % c);
        long long v = e / c;
        int x = (int)(v % w);
        long long q = v / w;
        int y = (int)(q % h);
        q /= h;
        int z = (int)(q % d);
        int nn = (int)(q / d);
        float s = 0.0f;
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++)
                for (int cc2 = 0; cc2 < 2; cc2++) {
                    long long fv = (((long long)nn * 2 * d + 2 * z + a) * 2 * h + 2 * y + b) * 2 * w + 2 * x + cc2;
                    s += bf2f(fine[fv * cf + f_off + ch]);
                }
        coarse[v * cc + c_off + ch] = f2bf(s);
    }
}

// dX of the 2^3 stride-2 convolution: dX[u] = dY[u / 2] W[u % 2]^T (weights
// rounded to BF16 like those of every other adjoint, FP32 accumulation)
__global__ void k_down_dgrad(const uint16_t *g, int cg, int g_off, const float *w, int cin, int cout, uint16_t *gx,
                             int cx, int x_off, int n, int d, int h, int wd, int accumulate)
{
    // (d, h, wd) are the fine sizes
    const long long total = (long long)n * d * h * wd * cin;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
        int ci = (int)(e % cin);
        long long v = e / cin;
        int x = (int)(v % wd);
        long long q = v / wd;
        int y = (int)(q % h);
        q /= h;
        int z = (int)(q % d);
        int nn = (int)(q / d);
        int t = ((z & 1) * 2 + (y & 1)) * 2 + (x & 1);
        long long cv = (((long long)nn * (d / 2) + z / 2) * (h / 2) + y / 2) * (wd / 2) + x / 2;
        const float *wt = w + ((long long)t * cin + ci) * cout;
        float s = 0.0f;
        for (int co = 0; co < cout; co++) s += bf2f(g[cv * cg + g_off + co]) * bf2f(f2bf(wt[co]));
        if (accumulate) s += bf2f(gx[v * cx + x_off + ci]);
        gx[v * cx + x_off + ci] = f2bf(s);
    }
}

// The same adjoint on MFMA: for each of the 8 taps t it is a GEMM
//   D[coarse voxel V][ci] = sum_co dY[V][co] W[t][ci][co]
// whose result lands on the fine voxel 2 V + t.  A wave owns 64 coarse voxels
// (4 row fragments) and all cin = 16 NF input channels; the FP32 weights are
// rounded to BF16 as they are read into the B fragments.
template <int NF>
__global__ __launch_bounds__(256) void k_down_dgrad_mfma(const uint16_t *g, int cg, int g_off, const float *w, int cin,
                                                         int cout, uint16_t *gx, int cx, int x_off, int n, int d, int h,
                                                         int wd, int accumulate)
{
    const int lane = threadIdx.x & 63, i = lane & 15, gq = lane >> 4;
    const int D2 = d / 2, H2 = h / 2, W2 = wd / 2;
    const int nvc = n * D2 * H2 * W2;
    const int V0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 64;
    if (V0 >= nvc) return;
    // fine index of tap 0 for the coarse voxels of this lane's D rows (f, r)
    int fb[4][4];
#pragma unroll
    for (int f = 0; f < 4; f++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int V = V0 + 16 * f + 4 * gq + r;
            if (V >= nvc) { fb[f][r] = -1; continue; }
            const int x = V % W2, y = (V / W2) % H2, z = (V / (W2 * H2)) % D2, nn = V / (W2 * H2 * D2);
            fb[f][r] = ((nn * d + 2 * z) * h + 2 * y) * wd + 2 * x;
        }
    const int kc = cout / 16;
    for (int t = 0; t < 8; t++) {
        const int ta = t >> 2, tb = (t >> 1) & 1, tc = t & 1;
        f4 acc[4][NF];
#pragma unroll
        for (int f = 0; f < 4; f++)
#pragma unroll
            for (int nf = 0; nf < NF; nf++) acc[f][nf] = f4{0.0f, 0.0f, 0.0f, 0.0f};
        for (int c = 0; c < kc; c++) {
            s4 A[4];
#pragma unroll
            for (int f = 0; f < 4; f++) {
                const int V = V0 + 16 * f + i;
                uint2 raw = make_uint2(0u, 0u);
                if (V < nvc) raw = *(const uint2 *)(g + (long long)V * cg + g_off + 16 * c + 4 * gq);
                A[f] = s4{(short)(raw.x & 0xffff), (short)(raw.x >> 16), (short)(raw.y & 0xffff), (short)(raw.y >> 16)};
            }
#pragma unroll
            for (int nf = 0; nf < NF; nf++) {
                const float4 wv = *(const float4 *)(w + ((long long)t * cin + 16 * nf + i) * cout + 16 * c + 4 * gq);
                const s4 Bv = s4{(short)f2bf(wv.x), (short)f2bf(wv.y), (short)f2bf(wv.z), (short)f2bf(wv.w)};
#pragma unroll
                for (int f = 0; f < 4; f++) acc[f][nf] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A[f], Bv, acc[f][nf], 0, 0, 0);
            }
        }
        const int toff = (ta * h + tb) * wd + tc;
#pragma unroll
        for (int f = 0; f < 4; f++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                if (fb[f][r] < 0) continue;
                uint16_t *gp = gx + (long long)(fb[f][r] + toff) * cx + x_off + i;
#pragma unroll
                for (int nf = 0; nf < NF; nf++) {
                    float val = acc[f][nf][r];
                    if (accumulate) val += bf2f(gp[16 * nf]);
                    gp[16 * nf] = f2bf(val);
                }
            }
    }
}

// FP32 -> BF16 channel-slice copy (network input)
__global__ void k_to_bf16(const float *x, int cs, long long nvox, int c, uint16_t *y, int cy, int y_off, int c_pad)
{
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nvox * c_pad; e += (long long)gridDim.x * blockDim.x) {
        long long v = e / c_pad;
        int ch = (int)(e % c_pad);
        y[v * cy + y_off + ch] = ch < c ? f2bf(x[v * cs + ch]) : (uint16_t)0;
    }
}

// Number of masked voxels (mask != 0): integer partial counts per workgroup
// added into the count slot (held as an int while counting), then turned
// into a float (exact below 2^24 voxels).
__global__ void k_mask_count(const float *mask, long long nvox, int *count)
{
    __shared__ int red[256];
    int c = 0;
    for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < nvox; v += (long long)gridDim.x * blockDim.x)
        c += mask[v] != 0.0f;
    red[threadIdx.x] = c;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0]) atomicAdd(count, red[0]);
}

__global__ void k_int_slot(int *slot, int to_float)
{
    if (to_float) *(float *)slot = (float)*slot;
    else *slot = 0;
}

// Masked mean-squared error and its gradient (BF16):
// loss_parts[block] = partial sums of mask (pred - target)^2, g = 2 (pred - target) / (count c)
// on masked voxels, 0 elsewhere (all cg channels written).
__global__ void k_masked_mse(const float *pred, int cp, const float *target, const float *mask, long long nvox, int c,
                             const float *count, uint16_t *g, int cg, float *loss_parts)
{
    __shared__ float red[256];
    const float cnt = (float)*(const int *)count * (float)c;
    const float inv_count = cnt > 0.0f ? 1.0f / cnt : 0.0f;
    float s = 0.0f;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nvox * cg; e += (long long)gridDim.x * blockDim.x) {
        long long v = e / cg;
        int ch = (int)(e % cg);
        float gv = 0.0f;
        if (ch < c && mask[v] != 0.0f) {
            float d = pred[v * cp + ch] - target[v * c + ch];
            s += d * d;
            gv = 2.0f * d * inv_count;
        }
        g[e] = f2bf(gv);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_parts[blockIdx.x] = red[0];
}

// Adam on FP32 master parameters (bias-corrected with step t)
__global__ void k_adam(float *p, const float *g, float *m, float *v, long long n, float lr, float b1, float b2, float eps,
                       int t)
{
    const float c1 = 1.0f / (1.0f - powf(b1, (float)t)), c2 = 1.0f / (1.0f - powf(b2, (float)t));
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        float gg = g[e];
        float mm = b1 * m[e] + (1.0f - b1) * gg;
        float vv = b2 * v[e] + (1.0f - b2) * gg * gg;
        m[e] = mm;
        v[e] = vv;
        p[e] -= lr * (mm * c1) / (sqrtf(vv * c2) + eps);
    }
}

// ---------------------------------------------------------------- crops of dense per-scene grids
// Bounding box of the nodes whose channel 0 is positive, one workgroup per
// grid: bbox[g] = (lo_x, lo_y, lo_z, hi_x, hi_y, hi_z), hi exclusive; an
// empty grid gives (0, 0, 0, 0, 0, 0).
__global__ __launch_bounds__(256) void k_bbox(const float *field, int cf, int R, int *bbox)
{
    __shared__ int red[6][256];
    const long long R3 = (long long)R * R * R;
    const float *f = field + (long long)blockIdx.x * R3 * cf;
    int lo[3] = {R, R, R}, hi[3] = {-1, -1, -1};
    for (long long c = threadIdx.x; c < R3; c += 256) {
        if (!(f[c * cf] > 0.0f)) continue;
        const int ii[3] = {(int)(c / ((long long)R * R)), (int)((c / R) % R), (int)(c % R)};
        for (int d = 0; d < 3; d++) {
            lo[d] = min(lo[d], ii[d]);
            hi[d] = max(hi[d], ii[d]);
        }
    }
    for (int d = 0; d < 3; d++) {
        red[d][threadIdx.x] = lo[d];
        red[3 + d][threadIdx.x] = hi[d];
    }
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            for (int d = 0; d < 3; d++) {
                red[d][threadIdx.x] = min(red[d][threadIdx.x], red[d][threadIdx.x + o]);
                red[3 + d][threadIdx.x] = max(red[3 + d][threadIdx.x], red[3 + d][threadIdx.x + o]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const bool empty = red[3][0] < 0;
        for (int d = 0; d < 3; d++) {
            bbox[6 * blockIdx.x + d] = empty ? 0 : red[d][0];
            bbox[6 * blockIdx.x + 3 + d] = empty ? 0 : red[3 + d][0] + 1;
        }
    }
}

// Crop origin per grid: the box of size (D, H, W) centred on bbox, moved
// inside [0, R).
__global__ void k_crop_origin(const int *bbox, int n, int R, int D, int H, int W, int *origin)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const int size[3] = {D, H, W};
    for (int d = 0; d < 3; d++) {
        const int lo = bbox[6 * g + d], hi = bbox[6 * g + 3 + d];
        int o = (lo + hi - size[d]) / 2;
        o = max(0, min(o, R - size[d]));
        origin[3 * g + d] = o;
    }
}

// dst[g][z][y][x][:c] = src[g][oz + z][oy + y][ox + x][:c]  (crop), or the
// reverse with zeros outside the crop (uncrop: dst is the full grid).
__global__ void k_crop(const float *src, int c, int n, int R, const int *origin, int D, int H, int W, float *dst,
                       int uncrop)
{
    const long long R3 = (long long)R * R * R;
    const long long per = uncrop ? R3 : (long long)D * H * W;
    const long long total = per * n * c;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
        const int ch = (int)(e % c);
        const long long v = e / c;
        const int g = (int)(v / per);
        const long long l = v - (long long)g * per;
        const int* o = origin + 3 * g;
        if (!uncrop) {
            const int z = (int)(l / ((long long)H * W)), y = (int)((l / W) % H), x = (int)(l % W);
            const long long sv = (((long long)g * R + o[0] + z) * R + o[1] + y) * R + o[2] + x;
            dst[e] = src[sv * c + ch];
        } else {
            const int i = (int)(l / ((long long)R * R)), j = (int)((l / R) % R), k = (int)(l % R);
            const int z = i - o[0], y = j - o[1], x = k - o[2];
            float val = 0.0f;
            if (z >= 0 && y >= 0 && x >= 0 && z < D && y < H && x < W)
                val = src[((((long long)g * D + z) * H + y) * W + x) * c + ch];
            dst[e] = val;
        }
    }
}

// ---------------------------------------------------------------- launchers
static unsigned grid_for(long long n, int per = 256)
{
    long long b = (n + per - 1) / per;
    return (unsigned)(b < 16384 ? (b < 1 ? 1 : b) : 16384);
}

template <int KIND>
static hipError_t conv_lds(const ConvArgs &a, hipStream_t st)
{
    const long long tiles = (long long)a.n * ((a.od + TLZ - 1) / TLZ) * ((a.oh + TLY - 1) / TLY) * ((a.ow + TLX - 1) / TLX);
    if (tiles > 0x7fffffff) return hipErrorInvalidValue;
    const unsigned g = (unsigned)tiles;
    if (a.cin % 32 == 0) {   // the weights were packed as 16x16x32 fragments (same condition in pack)
        const bool x16 = a.cx % 8 == 0 && a.x_off % 8 == 0 && ((uintptr_t)a.x & 15) == 0;
        // 8 output rows per wave up to 32 output channels (measured on the 40 x 24 x 40 boxes: the
        // forward 10.1 -> 9.8 ms; 8 rows at 64 channels cost an occupancy step and ran slower)
        const long long t8 = (long long)a.n * ((a.od + TLZ - 1) / TLZ) * ((a.oh + 7) / 8) * ((a.ow + TLX - 1) / TLX);
        if (t8 > 0x7fffffff) return hipErrorInvalidValue;
        const unsigned g8 = (unsigned)t8;
        switch ((a.cout + 15) / 16) {
        case 1: if (x16) k_conv_lds32<1, KIND, true, 8><<<g8, 256, 0, st>>>(a); else k_conv_lds32<1, KIND, false, 8><<<g8, 256, 0, st>>>(a); break;
        case 2: if (x16) k_conv_lds32<2, KIND, true, 8><<<g8, 256, 0, st>>>(a); else k_conv_lds32<2, KIND, false, 8><<<g8, 256, 0, st>>>(a); break;
        case 4: if (x16) k_conv_lds32<4, KIND, true, 4><<<g, 256, 0, st>>>(a); else k_conv_lds32<4, KIND, false, 4><<<g, 256, 0, st>>>(a); break;
        case 8: if (x16) k_conv_lds32<8, KIND, true, 4><<<g, 256, 0, st>>>(a); else k_conv_lds32<8, KIND, false, 4><<<g, 256, 0, st>>>(a); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch ((a.cout + 15) / 16) {
    case 1: k_conv_lds<1, KIND><<<g, 256, 0, st>>>(a); break;
    case 2: k_conv_lds<2, KIND><<<g, 256, 0, st>>>(a); break;
    case 4: k_conv_lds<4, KIND><<<g, 256, 0, st>>>(a); break;
    case 8: k_conv_lds<8, KIND><<<g, 256, 0, st>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t conv(const ConvArgs &a, hipStream_t st)
{
    if (a.kind == KIND_C3 && a.cin == 8) {
        if (a.cx % 8 || a.x_off % 8 || ((uintptr_t)a.x & 15)) return hipErrorInvalidValue;
        const long long tiles = (long long)a.n * ((a.od + TLZ - 1) / TLZ) * ((a.oh + TLY - 1) / TLY) * ((a.ow + TLX - 1) / TLX);
        if (tiles > 0x7fffffff) return hipErrorInvalidValue;
        switch ((a.cout + 15) / 16) {
        case 1: k_conv_first<1><<<(unsigned)tiles, 256, 0, st>>>(a); break;
        case 2: k_conv_first<2><<<(unsigned)tiles, 256, 0, st>>>(a); break;
        case 4: k_conv_first<4><<<(unsigned)tiles, 256, 0, st>>>(a); break;
        case 8: k_conv_first<8><<<(unsigned)tiles, 256, 0, st>>>(a); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (a.kind == KIND_C3) return conv_lds<KIND_C3>(a, st);
    if (a.kind == KIND_UP) return conv_lds<KIND_UP>(a, st);
    const long long nvox = (long long)a.n * a.od * a.oh * a.ow;
    const unsigned g = (unsigned)((nvox + 255) / 256);
    switch ((a.cout + 15) / 16) {
    case 1: k_conv<1><<<g, 256, 0, st>>>(a); break;
    case 2: k_conv<2><<<g, 256, 0, st>>>(a); break;
    case 4: k_conv<4><<<g, 256, 0, st>>>(a); break;
    case 8: k_conv<8><<<g, 256, 0, st>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t pack(const float *w, int ntap, int cin, int cout, int cin_p, int cout_p, int transpose, uint16_t *out,
                hipStream_t st)
{
    const long long total = (long long)ntap * (cin_p / 16) * (cout_p / 16) * 256;
    // 3^3 kernels with a multiple of 32 input channels run on 16x16x32 fragments, and so does the
    // 3^3 layer over 8 input channels (taps folded into K)
    const int k32 = ntap == 27 && !transpose && cin == 8 ? 2 : (ntap == 27 && cin_p % 32 == 0);
    if (k32 == 2) {
        const long long n2 = (long long)FIRST_STEPS * (cout_p / 16) * 512;
        k_pack<<<grid_for(n2), 256, 0, st>>>(w, ntap, cin, cout, cin_p, cout_p, transpose, k32, out);
        return hipGetLastError();
    }
    k_pack<<<grid_for(total), 256, 0, st>>>(w, ntap, cin, cout, cin_p, cout_p, transpose, k32, out);
    return hipGetLastError();
}

template <int KIND>
static hipError_t wgrad_lds(const WgradArgs &a, hipStream_t st)
{
    const int nf = (a.cout + 15) / 16;
    const int TZ = nf == 8 ? 2 : 4;
    const long long nvox = (long long)a.n * a.od * a.oh * a.ow;
    const long long ntiles = (long long)a.n * ((a.od + TZ - 1) / TZ) * ((a.oh + TLY - 1) / TLY) * ((a.ow + TLX - 1) / TLX);
    const long long groups_max = (nvox + a.chunk - 1) / a.chunk;          // the partial buffer holds this many
    const long long tpg = (ntiles + groups_max - 1) / groups_max;
    const long long groups = (ntiles + tpg - 1) / tpg;
    if (ntiles > 0x7fffffff || groups > 65535) return hipErrorInvalidValue;
    const dim3 g((unsigned)groups, (unsigned)(a.cin / 16), 4);
    switch (nf) {
    case 1: k_wgrad_lds<1, KIND><<<g, 256, 0, st>>>(a, (int)tpg, (int)ntiles); break;
    case 2: k_wgrad_lds<2, KIND><<<g, 256, 0, st>>>(a, (int)tpg, (int)ntiles); break;
    case 4: k_wgrad_lds<4, KIND><<<g, 256, 0, st>>>(a, (int)tpg, (int)ntiles); break;
    case 8: k_wgrad_lds<8, KIND><<<g, 256, 0, st>>>(a, (int)tpg, (int)ntiles); break;
    default: return hipErrorInvalidValue;
    }
    const long long per = 27LL * a.cin * a.cout;
    k_reduce_partials<<<grid_for(per), 256, 0, st>>>(a.partial, (int)groups, per, a.gw, a.accumulate);
    return hipGetLastError();
}

hipError_t wgrad(const WgradArgs &a, hipStream_t st)
{
    if (a.kind == KIND_C3) return wgrad_lds<KIND_C3>(a, st);
    if (a.kind == KIND_UP) return wgrad_lds<KIND_UP>(a, st);
    const int ks = a.kind == KIND_C3 || a.kind == KIND_UP ? 3 : (a.kind == KIND_DOWN ? 2 : 1);
    const int ntap = ks * ks * ks;
    const long long nvox = (long long)a.n * a.od * a.oh * a.ow;
    const int nchunk = (int)((nvox + a.chunk - 1) / a.chunk);
    const unsigned g = (unsigned)(nchunk * ntap);
    switch ((a.cout + 15) / 16) {
    case 1: k_wgrad<1><<<g, 256, 0, st>>>(a); break;
    case 2: k_wgrad<2><<<g, 256, 0, st>>>(a); break;
    case 4: k_wgrad<4><<<g, 256, 0, st>>>(a); break;
    case 8: k_wgrad<8><<<g, 256, 0, st>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    const long long per = (long long)ntap * a.cin * a.cout;
    k_reduce_partials<<<grid_for(per), 256, 0, st>>>(a.partial, nchunk, per, a.gw, a.accumulate);
    return hipGetLastError();
}

hipError_t bias_grad(const uint16_t *g, long long nvox, int cg, int g_off, int cout, float *gb, int accumulate,
                     hipStream_t st)
{
    if (cout > 128) return hipErrorInvalidValue;
    if (!accumulate) k_fill_f<<<(cout + 63) / 64, 64, 0, st>>>(gb, cout, 0.0f);
    const long long nb = (nvox + BIAS_CHUNK - 1) / BIAS_CHUNK;
    if (cout % 4 == 0 && cg % 4 == 0 && g_off % 4 == 0 && ((uintptr_t)g & 7) == 0)
        k_bias_grad4<<<(unsigned)nb, 256, 0, st>>>(g, nvox, cg, g_off, cout, gb);
    else
        k_bias_grad<<<(unsigned)nb, 256, 0, st>>>(g, nvox, cg, g_off, cout, gb);
    return hipGetLastError();
}

hipError_t relu_bwd(uint16_t *g, int cg, int g_off, const uint16_t *y, int cy, int y_off, long long nvox, int c,
                    hipStream_t st)
{
    k_relu_bwd<<<grid_for(nvox * c), 256, 0, st>>>(g, cg, g_off, y, cy, y_off, nvox, c);
    return hipGetLastError();
}

hipError_t up_bwd(const uint16_t *fine, int cf, int f_off, uint16_t *coarse, int cc, int c_off, int n, int d, int h, int w,
                  int c, hipStream_t st)
{
    k_up_bwd<<<grid_for((long long)n * d * h * w * c), 256, 0, st>>>(fine, cf, f_off, coarse, cc, c_off, n, d, h, w, c);
    return hipGetLastError();
}

hipError_t down_dgrad(const uint16_t *g, int cg, int g_off, const float *w, int cin, int cout, uint16_t *gx, int cx,
                      int x_off, int n, int d, int h, int wd, int accumulate, hipStream_t st)
{
    const long long nfine = (long long)n * d * h * wd;
    if (cin % 16 == 0 && cout % 16 == 0 && cin <= 128 && cg % 4 == 0 && g_off % 4 == 0 && nfine < 0x7fffffffLL &&
        ((uintptr_t)g & 7) == 0 && ((uintptr_t)w & 15) == 0) {
        const long long nvc = nfine / 8;
        const unsigned blocks = (unsigned)((nvc + 255) / 256);
        switch (cin / 16) {
        case 1: k_down_dgrad_mfma<1><<<blocks, 256, 0, st>>>(g, cg, g_off, w, cin, cout, gx, cx, x_off, n, d, h, wd, accumulate); break;
        case 2: k_down_dgrad_mfma<2><<<blocks, 256, 0, st>>>(g, cg, g_off, w, cin, cout, gx, cx, x_off, n, d, h, wd, accumulate); break;
        case 4: k_down_dgrad_mfma<4><<<blocks, 256, 0, st>>>(g, cg, g_off, w, cin, cout, gx, cx, x_off, n, d, h, wd, accumulate); break;
        case 8: k_down_dgrad_mfma<8><<<blocks, 256, 0, st>>>(g, cg, g_off, w, cin, cout, gx, cx, x_off, n, d, h, wd, accumulate); break;
        default:
            k_down_dgrad<<<grid_for(nfine * cin), 256, 0, st>>>(g, cg, g_off, w, cin, cout, gx, cx, x_off, n, d, h, wd,
                                                                accumulate);
        }
        return hipGetLastError();
    }
    k_down_dgrad<<<grid_for(nfine * cin), 256, 0, st>>>(g, cg, g_off, w, cin, cout, gx, cx, x_off, n, d, h, wd, accumulate);
    return hipGetLastError();
}

hipError_t to_bf16(const float *x, int cs, long long nvox, int c, uint16_t *y, int cy, int y_off, int c_pad, hipStream_t st)
{
    k_to_bf16<<<grid_for(nvox * c_pad), 256, 0, st>>>(x, cs, nvox, c, y, cy, y_off, c_pad);
    return hipGetLastError();
}

hipError_t masked_mse(const float *pred, int cp, const float *target, const float *mask, long long nvox, int c,
                      uint16_t *g, int cg, float *loss_parts, int nparts, hipStream_t st)
{
    int *slot = (int *)(loss_parts + nparts);
    k_int_slot<<<1, 1, 0, st>>>(slot, 0);
    k_mask_count<<<grid_for(nvox), 256, 0, st>>>(mask, nvox, slot);
    k_masked_mse<<<nparts, 256, 0, st>>>(pred, cp, target, mask, nvox, c, loss_parts + nparts, g, cg, loss_parts);
    k_int_slot<<<1, 1, 0, st>>>(slot, 1);
    return hipGetLastError();
}

hipError_t bbox(const float *field, int cf, int n, int R, int *box, hipStream_t st)
{
    k_bbox<<<n, 256, 0, st>>>(field, cf, R, box);
    return hipGetLastError();
}

hipError_t crop_origin(const int *box, int n, int R, int D, int H, int W, int *origin, hipStream_t st)
{
    k_crop_origin<<<(n + 63) / 64, 64, 0, st>>>(box, n, R, D, H, W, origin);
    return hipGetLastError();
}

hipError_t crop(const float *src, int c, int n, int R, const int *origin, int D, int H, int W, float *dst, int uncrop,
                hipStream_t st)
{
    const long long per = uncrop ? (long long)R * R * R : (long long)D * H * W;
    k_crop<<<grid_for(per * n * c), 256, 0, st>>>(src, c, n, R, origin, D, H, W, dst, uncrop);
    return hipGetLastError();
}

hipError_t adam(float *p, const float *g, float *m, float *v, long long n, float lr, float b1, float b2, float eps, int t,
                hipStream_t st)
{
    k_adam<<<grid_for(n), 256, 0, st>>>(p, g, m, v, n, lr, b1, b2, eps, t);
    return hipGetLastError();
}

}  // namespace nn
