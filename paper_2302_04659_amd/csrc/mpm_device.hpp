// Device helpers shared by the substep kernels and the surrogate kernels (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "mpm_kernels.hpp"
#include "mpm_math.hpp"

namespace mpm {

constexpr int WG = 256;
constexpr float SUR_VEL = 0.2f;   // velocity unit of the surrogate's inputs and outputs (m/s)
constexpr float SUR_DM = 1.0f / 32.0f;   // unit of the predicted mass change, in rho dx^3 (a change over one
                                         // control step is ~1e-3 rho dx^3; this unit brings it to O(1e-2))
// Per-block position error bar of the surrogate, in cells: the residual's
// momentum term is measured against the speed that crosses it in one
// control step, SUR_ERR_BAR dx / (n_sub dt).
constexpr float SUR_ERR_BAR = 0.02f;

__device__ __forceinline__ int xcd_remap(int b, int G)
{
    // Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
    // contiguous run of work items so neighbouring grid blocks share an L2.
    return (b & 7) * (G >> 3) + (b >> 3);
}

// Workgroups that share n units of work: the whole launch when the work
// suffices, else the smallest multiple of 8 covering it, so that every XCD
// (the dispatcher deals workgroups to the 8 XCDs in turn) still gets a share.
// The launch size must be a multiple of 8.
__device__ __forceinline__ int active_wgs(int n)
{
    return min((int)gridDim.x, (n + 7) & ~7);
}

// Two signed 32-bit terms as one 64-bit addend hi * 2^32 + lo; a sum of such
// addends (wrapping 64-bit integer adds) unpacks to the two exact sums while
// each stays inside the int32 range.
__device__ __forceinline__ unsigned long long pack2(int hi, int lo)
{
    return ((unsigned long long)(unsigned)hi << 32) + (unsigned long long)(long long)lo;
}

// The same for lo >= 0 (no borrow into hi): the two halves as they are.
__device__ __forceinline__ unsigned long long pack2_nonneg_lo(int hi, int lo)
{
    return ((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo;
}

__device__ __forceinline__ void unpack2(long long v, int &hi, int &lo)
{
    lo = (int)(unsigned)(v & 0xffffffffLL);
    hi = (int)((v - (long long)lo) >> 32);
}

__device__ __forceinline__ int cvt_rpi(float x)
{
    int r;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// Particle component c of slot j: base pointer per component (uniform) plus a
// 32-bit byte offset, so loads and stores use scalar-base addressing.
typedef __attribute__((address_space(1))) char gchar;

__device__ __forceinline__ gchar *sgpr_base(const float *p)
{
    gchar *g = (gchar *)p;
    asm("" : "+s"(g));
    return g;
}

__device__ __forceinline__ float pload(const float *P, long long ps, int c, unsigned joff)
{
    return *(const __attribute__((address_space(1))) float *)(sgpr_base(P + c * ps) + joff);
}

__device__ __forceinline__ void pstore(float *P, long long ps, int c, unsigned joff, float v)
{
    *(__attribute__((address_space(1))) float *)(sgpr_base(P + c * ps) + joff) = v;
}

// G2P prefetch: the 12 state components it reads (x, then G) of up to 64
// consecutive particle slots, copied by the wave straight into its LDS
// slice pw[c * 64 + lane] (global_load_lds: no registers held while in flight).
constexpr int PF_COMPS = 12;

// One float per lane from global src into LDS at dst_wave + lane (dst_wave is
// the wave's LDS base, the same on every lane).
__device__ __forceinline__ void lds_copy(const float *src, float *dst_wave)
{
    typedef __attribute__((address_space(3))) void lds_void;
    typedef const __attribute__((address_space(1))) void glob_void;
    __builtin_amdgcn_global_load_lds((glob_void *)src, (lds_void *)dst_wave, 4, 0, 0);
}

__device__ __forceinline__ void pf_issue(const float *P, long long ps, int first, int n_left, int lane, float *pw)
{
    if (lane >= n_left) return;
    const unsigned jo = (unsigned)(first + lane) << 2;
    typedef __attribute__((address_space(3))) void lds_void;
    typedef const __attribute__((address_space(1))) void glob_void;
#pragma unroll
    for (int c = 0; c < PF_COMPS; c++) {
        const int comp = c < 3 ? X0 + c : G00 + (c - 3);
        __builtin_amdgcn_global_load_lds((glob_void *)(sgpr_base(P + comp * ps) + jo), (lds_void *)(pw + c * 64), 4, 0, 0);
    }
}

// Waits the compiler does not insert for LDS written by global_load_lds.
__device__ __forceinline__ void wait_vmem() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
__device__ __forceinline__ void wait_lds() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

__device__ __forceinline__ long long node_index(const SceneDev &S, int B, int i, int j, int k)
{
    int nb = S.nb;
    int lb = ((i / B) * nb + (j / B)) * nb + (k / B);
    int l = ((i % B) * B + (j % B)) * B + (k % B);
    return S.grid_off + (long long)lb * (B * B * B) + l;
}

// Index of grid node (i, j, k) of scene s in the surrogate's per-scene
// arrays: the whole grid (offset cap_off[s]) or the scene's box; -1 outside
// the box.
__device__ __forceinline__ long long sur_index(const StepArgs &a, int s, int res, int i, int j, int k)
{
    if (!a.sur_org) return a.cap_off[s] + ((long long)i * res + j) * res + k;
    const int *o = a.sur_org + 3 * s;
    const int z = i - o[0], y = j - o[1], x = k - o[2];
    if (z < 0 || y < 0 || x < 0 || z >= a.sur_box[0] || y >= a.sur_box[1] || x >= a.sur_box[2]) return -1;
    return (((long long)s * a.sur_box[0] + z) * a.sur_box[1] + y) * a.sur_box[2] + x;
}

__device__ __forceinline__ int scene_of_bin(const int *off, int n_scenes, int b)
{
    int lo = 0, hi = n_scenes;          // off[lo] <= b < off[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ void particle_base(const SceneDev &S, float x, int &b, float &f, int &clamped)
{
    float xi = x * S.inv_dx;
    float fb = floorf(xi - 0.5f);
    int bi = (int)fb;
    int c = bi < 0 ? 0 : (bi > S.res - 3 ? S.res - 3 : bi);
    clamped |= (c != bi) || !(fb == fb);
    b = c;
    f = xi - (float)c;
}

// Scene constants a particle loop uses, read once into scalar registers.
// Without the copy, every particle store (which, as far as the compiler
// knows, may alias the scene table) forces a reload and a wait on all
// outstanding memory operations before the next use.
struct SceneK {
    int res;
    float dx, inv_dx, dt, mass, kstress;
};

__device__ __forceinline__ float uniform_f(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ long long uniform_ll(long long v)
{
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v), hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ SceneK scene_k(const SceneDev &S)
{
    SceneK k;
    k.res = __builtin_amdgcn_readfirstlane(S.res);
    k.dx = uniform_f(S.dx);
    k.inv_dx = uniform_f(S.inv_dx);
    k.dt = uniform_f(S.dt);
    k.mass = uniform_f(S.mass);
    k.kstress = uniform_f(S.kstress);
    return k;
}

__device__ __forceinline__ void particle_base(const SceneK &K, float x, int &b, float &f, int &clamped)
{
    float xi = x * K.inv_dx;
    float fb = floorf(xi - 0.5f);
    int bi = (int)fb;
    int c = bi < 0 ? 0 : (bi > K.res - 3 ? K.res - 3 : bi);
    clamped |= (c != bi) || !(fb == fb);
    b = c;
    f = xi - (float)c;
}

__device__ __forceinline__ Material material_of(const SceneDev &S)
{
    Material m;
    m.model = S.model;
    m.plastic = S.plastic;
    m.mu = S.mu;
    m.la = S.la;
    m.yield_eps = S.yield_eps;
    return m;
}

// Bound on |m v_c + (A d)_c| over the 27 stencil offsets d (|d_e| <= 1.5 dx).
__device__ __forceinline__ float scatter_bound(float mass, float dx, const float v[3], const float A[9])
{
    float b = 0.0f;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        float row = fabsf(A[3 * c]) + fabsf(A[3 * c + 1]) + fabsf(A[3 * c + 2]);
        b = fmaxf(b, fmaf(mass, fabsf(v[c]), 1.5f * dx * row));
    }
    return b;
}

__device__ __forceinline__ float wave_max(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ int wave_max_i(int v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ unsigned wave_or(unsigned v)
{
    for (int o = 32; o > 0; o >>= 1) v |= (unsigned)__shfl_xor((int)v, o, 64);
    return v;
}

// Sum over the 64 lanes, returned on every lane (all lanes must be active).
// An inclusive scan with DPP moves (VALU, no LDS round trip): shifts by 1, 2, 4
// and 8 inside each row of 16 lanes (lanes shifted in from outside the row read
// 0), then row 0's last lane added to row 1 and row 2's to row 3 (row_bcast:15),
// then lane 31 added to rows 2 and 3 (row_bcast:31); lane 63 ends with the total.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float t)
{
    const int moved = __builtin_amdgcn_update_dpp(0, __float_as_int(t), CTRL, ROW_MASK, 0xf, true);
    return t + __int_as_float(moved);
}

__device__ __forceinline__ float wave_total(float v)
{
    v = dpp_add<0x111, 0xf>(v);   // row_shr:1
    v = dpp_add<0x112, 0xf>(v);   // row_shr:2
    v = dpp_add<0x114, 0xf>(v);   // row_shr:4
    v = dpp_add<0x118, 0xf>(v);   // row_shr:8
    v = dpp_add<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v = dpp_add<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

}  // namespace mpm
