// HIP kernels of the MLS-MPM substep for gfx950 (MI355X).
//
// One substep (Algorithm 1, inner loop: particle to grid, grid velocity,
// grid to particle, integrate) runs as
//   k_p2g   particle-to-grid: APIC + MLS stress scatter of one binned chunk of
//           particles into an LDS tile (integer fixed-point accumulation with
//           ds_add_u32, exact and order independent), flushed to the global
//           grid with float atomics;
//   k_grid  grid velocity: v = p/m, gravity, SDF colliders, walls; it zeroes
//           (m, p) after reading them, so no separate clear pass exists;
//   k_g2p   grid-to-particle fused with the integration: velocity and APIC
//           matrix from an LDS tile of grid velocities, x += dt v,
//           F <- (I + dt C) F, Hencky + von Mises return map, and the affine
//           momentum A = m C - dt V (4/dx^2) tau(F) the next P2G scatters.
// Particles are binned by grid block (Morton order inside a scene) every
// few substeps by a counting sort (k_keys .. k_gather).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "mpm_kernels.hpp"
#include "mpm_math.hpp"

namespace mpm {

static constexpr int WG = 256;

__device__ __forceinline__ int xcd_remap(int b, int G)
{
    // Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
    // contiguous run of work items so neighbouring grid blocks share an L2.
    return (b & 7) * (G >> 3) + (b >> 3);
}

__device__ __forceinline__ int cvt_rpi(float x)
{
    int r;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

__device__ __forceinline__ long long node_index(const SceneDev &S, int B, int i, int j, int k)
{
    int nb = S.nb;
    int lb = ((i / B) * nb + (j / B)) * nb + (k / B);
    int l = ((i % B) * B + (j % B)) * B + (k % B);
    return S.grid_off + (long long)lb * (B * B * B) + l;
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

// ====================================================================== sort
__global__ __launch_bounds__(WG) void k_keys(SortArgs a)
{
    int j = blockIdx.x * WG + threadIdx.x;
    if (j >= a.N) return;
    int s = a.psc[j];
    const SceneDev &S = a.scenes[s];
    int b[3], cl = 0;
    float f;
    for (int d = 0; d < 3; d++) particle_base(S, a.P[(long long)(X0 + d) * a.pstride + j], b[d], f, cl);
    unsigned key = (unsigned)a.scene_bin_off[s] + morton3(b[0] / a.B, b[1] / a.B, b[2] / a.B);
    a.keys[j] = key;
    atomicAdd(&a.count[key], 1);
}

// Grid blocks that may receive mass: the 27-neighbourhood of every block
// holding particles (a P2G tile reaches one block beyond its own).
__global__ __launch_bounds__(WG) void k_dilate(SortArgs a)
{
    int b = blockIdx.x * WG + threadIdx.x;
    if (b >= a.T) return;
    int s = scene_of_bin(a.scene_bin_off, a.n_scenes, b);
    const SceneDev &S = a.scenes[s];
    int off = a.scene_bin_off[s];
    uint32_t m = (uint32_t)(b - off);
    int bx = compact3(m), by = compact3(m >> 1), bz = compact3(m >> 2);
    int nb = S.nb, hit = 0;
    for (int dx = -1; dx <= 1; dx++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dz = -1; dz <= 1; dz++) {
                int x = bx + dx, y = by + dy, z = bz + dz;
                if (x < 0 || y < 0 || z < 0 || x >= nb || y >= nb || z >= nb) continue;
                hit |= a.count[off + morton3(x, y, z)] > 0;
            }
    a.dil[b] = (unsigned char)hit;
    a.L.bflag[off + (bx * nb + by) * nb + bz] = hit ? 2 : 0;
}

static constexpr int SCAN_PER = 8;
static constexpr int SCAN_TILE = WG * SCAN_PER;

__device__ __forceinline__ int3 bin_triple(const SortArgs &a, int b)
{
    if (b >= a.T) return make_int3(0, 0, 0);
    int c = a.count[b];
    return make_int3(c, (c + a.CH - 1) / a.CH, (int)a.dil[b]);
}

__device__ __forceinline__ int3 add3(int3 x, int3 y) { return make_int3(x.x + y.x, x.y + y.y, x.z + y.z); }

// Exclusive scan of one int3 per thread over the workgroup; returns the total.
__device__ int3 block_exscan3(int3 v, int3 &excl)
{
    __shared__ int3 wsum[WG / 64];
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int3 inc = v;
    for (int o = 1; o < 64; o <<= 1) {
        int3 t;
        t.x = __shfl_up(inc.x, o, 64);
        t.y = __shfl_up(inc.y, o, 64);
        t.z = __shfl_up(inc.z, o, 64);
        if (lane >= o) inc = add3(inc, t);
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int3 before = make_int3(0, 0, 0), total = make_int3(0, 0, 0);
    for (int i = 0; i < WG / 64; i++) {
        if (i < w) before = add3(before, wsum[i]);
        total = add3(total, wsum[i]);
    }
    excl = make_int3(before.x + inc.x - v.x, before.y + inc.y - v.y, before.z + inc.z - v.z);
    __syncthreads();
    return total;
}

__global__ __launch_bounds__(WG) void k_scan_tiles(SortArgs a)
{
    int base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_PER;
    int3 s = make_int3(0, 0, 0);
    for (int i = 0; i < SCAN_PER; i++) s = add3(s, bin_triple(a, base + i));
    int3 ex;
    int3 tot = block_exscan3(s, ex);
    if (threadIdx.x == 0) a.tsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(WG) void k_scan_top(SortArgs a, int ntiles)
{
    int3 carry = make_int3(0, 0, 0);
    for (int base = 0; base < ntiles; base += WG) {
        int i = base + threadIdx.x;
        int3 v = i < ntiles ? a.tsum[i] : make_int3(0, 0, 0);
        int3 ex;
        int3 tot = block_exscan3(v, ex);
        if (i < ntiles) a.tsum[i] = add3(ex, carry);
        carry = add3(carry, tot);
    }
    if (threadIdx.x == 0) {
        *a.L.n_items = carry.y;
        *a.L.n_gitems = carry.z;
        a.L.scene_item_begin[a.n_scenes] = carry.y;
        a.L.scene_gitem_begin[a.n_scenes] = carry.z;
    }
}

__global__ __launch_bounds__(WG) void k_scan_emit(SortArgs a)
{
    int base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_PER;
    int3 v[SCAN_PER];
    int3 s = make_int3(0, 0, 0);
    for (int i = 0; i < SCAN_PER; i++) {
        v[i] = bin_triple(a, base + i);
        s = add3(s, v[i]);
    }
    int3 ex;
    block_exscan3(s, ex);
    int3 run = add3(ex, a.tsum[blockIdx.x]);
    for (int i = 0; i < SCAN_PER; i++) {
        int b = base + i;
        if (b < a.T) {
            a.pstart[b] = run.x;
            int sc = scene_of_bin(a.scene_bin_off, a.n_scenes, b);
            int off = a.scene_bin_off[sc];
            if (b == off) {
                a.L.scene_item_begin[sc] = run.y;
                a.L.scene_gitem_begin[sc] = run.z;
            }
            if (v[i].x > 0 || v[i].z > 0) {
                const SceneDev &S = a.scenes[sc];
                uint32_t m = (uint32_t)(b - off);
                int bx = compact3(m), by = compact3(m >> 1), bz = compact3(m >> 2);
                int lb = (bx * S.nb + by) * S.nb + bz;
                for (int c = 0; c < v[i].y; c++) {
                    Item it;
                    it.scene = sc;
                    it.block = lb;
                    it.start = run.x + c * a.CH;
                    it.count = min(a.CH, v[i].x - c * a.CH);
                    a.L.items[run.y + c] = it;
                }
                if (v[i].z) a.L.gitems[run.z] = make_int2(sc, lb);
            }
        }
        run = add3(run, v[i]);
    }
}

__global__ __launch_bounds__(WG) void k_scatter(SortArgs a)
{
    int j = blockIdx.x * WG + threadIdx.x;
    if (j >= a.N) return;
    unsigned key = a.keys[j];
    int c = atomicSub(&a.count[key], 1);
    a.perm[a.pstart[key] + c - 1] = j;
}

__global__ __launch_bounds__(WG) void k_gather(SortArgs a)
{
    int p = blockIdx.x * WG + threadIdx.x;
    if (p >= a.N) return;
    int j = a.perm[p];
#pragma unroll
    for (int c = 0; c < NCOMP; c++) a.Pn[(long long)c * a.pstride + p] = a.P[(long long)c * a.pstride + j];
}

hipError_t launch_sort(const SortArgs &a, hipStream_t st)
{
    int gN = (a.N + WG - 1) / WG, gT = (a.T + WG - 1) / WG;
    int ntiles = (a.T + SCAN_TILE - 1) / SCAN_TILE;
    if (a.N > 0) k_keys<<<gN, WG, 0, st>>>(a);
    k_dilate<<<gT, WG, 0, st>>>(a);
    k_scan_tiles<<<ntiles, WG, 0, st>>>(a);
    k_scan_top<<<1, WG, 0, st>>>(a, ntiles);
    k_scan_emit<<<ntiles, WG, 0, st>>>(a);
    if (a.N > 0) {
        k_scatter<<<gN, WG, 0, st>>>(a);
        k_gather<<<gN, WG, 0, st>>>(a);
    }
    return hipGetLastError();
}

// ====================================================================== substep pieces
__device__ __forceinline__ void load_particle_xvA(const StepArgs &a, int j, float x[3], float v[3], float A[9])
{
    const float *P = a.P;
    long long ps = a.pstride;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        x[d] = P[(X0 + d) * ps + j];
        v[d] = P[(V0 + d) * ps + j];
    }
#pragma unroll
    for (int e = 0; e < 9; e++) A[e] = P[(A00 + e) * ps + j];
}

// Slow path of P2G: scatter one particle straight into the global grid and
// queue any block that is not already on the grid-update list.
__device__ void p2g_global(const StepArgs &a, int s, const SceneDev &S, const float x[3], const float v[3],
                           const float A[9], const int b[3], const float f[3])
{
    int B = a.B;
    float w[3][3];
    for (int d = 0; d < 3; d++) bspline_w(f[d], w[d]);
    for (int ox = 0; ox < 3; ox++)
        for (int oy = 0; oy < 3; oy++)
            for (int oz = 0; oz < 3; oz++) {
                float wt = w[0][ox] * w[1][oy] * w[2][oz];
                float d[3] = {(ox - f[0]) * S.dx, (oy - f[1]) * S.dx, (oz - f[2]) * S.dx};
                long long idx = node_index(S, B, b[0] + ox, b[1] + oy, b[2] + oz);
                atomicAdd(a.gm + idx, wt * S.mass);
                atomicAdd(a.gpx + idx, wt * (S.mass * v[0] + A[0] * d[0] + A[1] * d[1] + A[2] * d[2]));
                atomicAdd(a.gpy + idx, wt * (S.mass * v[1] + A[3] * d[0] + A[4] * d[1] + A[5] * d[2]));
                atomicAdd(a.gpz + idx, wt * (S.mass * v[2] + A[6] * d[0] + A[7] * d[1] + A[8] * d[2]));
            }
    for (int cx = 0; cx < 2; cx++)
        for (int cy = 0; cy < 2; cy++)
            for (int cz = 0; cz < 2; cz++) {
                int bx = (b[0] + 2 * cx) / B, by = (b[1] + 2 * cy) / B, bz = (b[2] + 2 * cz) / B;
                if ((cx && bx == b[0] / B) || (cy && by == b[1] / B) || (cz && bz == b[2] / B)) continue;
                int lb = (bx * S.nb + by) * S.nb + bz;
                int *fl = a.L.bflag + S.bin_off + lb;
                if (*fl == 0 && atomicCAS(fl, 0, 1) == 0) {
                    int pos = atomicAdd(a.L.n_ovf, 1);
                    if (pos < a.L.ovf_cap) a.L.ovf[pos] = make_int2(s, lb);
                    else atomicOr(a.flags + s, (int)FLAG_OVERFLOW_FULL);
                }
            }
}

__device__ __forceinline__ float wave_max(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// Collider poses of scene s at substep k, written once per substep.
__device__ void write_colliders_now(const StepArgs &a, const SceneDev &S)
{
    int t = threadIdx.x;
    if (t < S.n_col) {
        ColliderNow cn;
        collider_at(a.cols[S.col_off + t], (float)a.substep * S.dt, cn);
        ((ColliderNow *)a.colnow)[S.col_off + t] = cn;
    }
}

template <int B, int PPT>
__device__ void p2g_item(const StepArgs &a, int it, const Item &item, int *tile, float *sred)
{
    constexpr int T = B + 4, T3 = T * T * T;
    const int t = threadIdx.x;
    const int s = item.scene;
    const SceneDev &S = a.scenes[s];
    const int nb = S.nb;
    const int bx = item.block / (nb * nb), by = (item.block / nb) % nb, bz = item.block % nb;
    const int org[3] = {bx * B - 1, by * B - 1, bz * B - 1};

    for (int n = t; n < 4 * T3; n += WG) tile[n] = 0;

    float xs[PPT][3], vs[PPT][3], As[PPT][9];
    int bs[PPT][3], mode[PPT];   // mode: 0 none, 1 tile, 2 global
    float fs[PPT][3];
    float bmax = 0.0f;
#pragma unroll
    for (int r = 0; r < PPT; r++) {
        int li = r * WG + t;
        mode[r] = 0;
        if (li < item.count) {
            int j = item.start + li;
            load_particle_xvA(a, j, xs[r], vs[r], As[r]);
            int cl = 0, in = 1;
#pragma unroll
            for (int d = 0; d < 3; d++) {
                particle_base(S, xs[r][d], bs[r][d], fs[r][d], cl);
                int tb = bs[r][d] - org[d];
                in &= (tb >= 0) & (tb <= B + 1);
            }
            if (cl) atomicOr(a.flags + s, (int)FLAG_CLAMPED);
            mode[r] = (in && !cl) ? 1 : 2;
            if (mode[r] == 1) {
                float bnd = 0.0f;
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    float row = fabsf(As[r][3 * c]) + fabsf(As[r][3 * c + 1]) + fabsf(As[r][3 * c + 2]);
                    bnd = fmaxf(bnd, S.mass * fabsf(vs[r][c]) + 1.5f * S.dx * row);
                }
                bmax = fmaxf(bmax, bnd);
            }
        }
    }
    bmax = wave_max(bmax);
    if ((t & 63) == 0) sred[t >> 6] = bmax;
    if (it == a.L.scene_item_begin[s]) write_colliders_now(a, S);
    __syncthreads();
    bmax = fmaxf(fmaxf(sred[0], sred[1]), fmaxf(sred[2], sred[3]));

    // Power-of-two fixed-point scales keeping every node sum below 2^30:
    // |contribution| <= w * bound, w <= 0.421875, at most item.count particles.
    const float lim = 1073741824.0f / (0.421875f * (float)item.count);
    int em = ilogbf(lim / S.mass);
    em = min(max(em, -120), 120);
    int ep = bmax > 0.0f ? ilogbf(lim / bmax) : 120;
    ep = min(max(ep, -120), 120);
    const float Sm = ldexpf(1.0f, em), Sp = ldexpf(1.0f, ep);
    const float kk = Sp / (Sm * S.mass);       // momentum scale relative to the mass-scaled weight

#pragma unroll
    for (int r = 0; r < PPT; r++) {
        if (mode[r] == 1) {
            float wx[3], wy[3], wz[3];
            bspline_w(fs[r][0], wx);
            bspline_w(fs[r][1], wy);
            bspline_w(fs[r][2], wz);
            const float msc = Sm * S.mass;
#pragma unroll
            for (int o = 0; o < 3; o++) wx[o] *= msc;
            // r(o) = kk * (m v + A (o - f) dx); increments along each axis
            float Ad[3][3], r0[3];
#pragma unroll
            for (int c = 0; c < 3; c++) {
#pragma unroll
                for (int e = 0; e < 3; e++) Ad[c][e] = kk * As[r][3 * c + e] * S.dx;
                r0[c] = kk * S.mass * vs[r][c] - (Ad[c][0] * fs[r][0] + Ad[c][1] * fs[r][1] + Ad[c][2] * fs[r][2]);
            }
            int *tb = tile + ((bs[r][0] - org[0]) * T + (bs[r][1] - org[1])) * T + (bs[r][2] - org[2]);
#pragma unroll
            for (int ox = 0; ox < 3; ox++)
#pragma unroll
                for (int oy = 0; oy < 3; oy++) {
                    float wxy = wx[ox] * wy[oy];
                    float rxy[3];
#pragma unroll
                    for (int c = 0; c < 3; c++) rxy[c] = r0[c] + (float)ox * Ad[c][0] + (float)oy * Ad[c][1];
#pragma unroll
                    for (int oz = 0; oz < 3; oz++) {
                        float w = wxy * wz[oz];
                        int o = (ox * T + oy) * T + oz;
                        atomicAdd(tb + o, cvt_rpi(w));
#pragma unroll
                        for (int c = 0; c < 3; c++)
                            atomicAdd(tb + (c + 1) * T3 + o, cvt_rpi(w * (rxy[c] + (float)oz * Ad[c][2])));
                    }
                }
        } else if (mode[r] == 2) {
            p2g_global(a, s, S, xs[r], vs[r], As[r], bs[r], fs[r]);
        }
    }
    __syncthreads();
    const float im = 1.0f / Sm, ip = 1.0f / Sp;
    for (int n = t; n < T3; n += WG) {
        int m0 = tile[n], p0 = tile[T3 + n], p1 = tile[2 * T3 + n], p2 = tile[3 * T3 + n];
        if ((m0 | p0 | p1 | p2) == 0) continue;
        int tx = n / (T * T), ty = (n / T) % T, tz = n % T;
        int gi = org[0] + tx, gj = org[1] + ty, gk = org[2] + tz;
        if (gi < 0 || gj < 0 || gk < 0 || gi >= S.res || gj >= S.res || gk >= S.res) continue;
        long long idx = node_index(S, B, gi, gj, gk);
        atomicAdd(a.gm + idx, (float)m0 * im);
        atomicAdd(a.gpx + idx, (float)p0 * ip);
        atomicAdd(a.gpy + idx, (float)p1 * ip);
        atomicAdd(a.gpz + idx, (float)p2 * ip);
    }
    __syncthreads();
}

template <int B, int PPT>
__global__ __launch_bounds__(WG) void k_p2g(StepArgs a)
{
    constexpr int T = B + 4, T3 = T * T * T;
    __shared__ int tile[4 * T3];
    __shared__ float sred[4];
    const int n_items = *a.L.n_items;
    for (int it = xcd_remap(blockIdx.x, gridDim.x); it < n_items; it += gridDim.x) {
        Item item = a.L.items[it];
        p2g_item<B, PPT>(a, it, item, tile, sred);
    }
}

// ---------------------------------------------------------------- grid update
template <int B>
__device__ void grid_block(const StepArgs &a, int s, int lb, int lane)
{
    const SceneDev &S = a.scenes[s];
    const int nb = S.nb;
    const int bx = lb / (nb * nb), by = (lb / nb) % nb, bz = lb % nb;
    const ColliderNow *cn = (const ColliderNow *)a.colnow + S.col_off;
    for (int l = lane; l < B * B * B; l += 64) {
        long long idx = S.grid_off + (long long)lb * (B * B * B) + l;
        float m = a.gm[idx], px = a.gpx[idx], py = a.gpy[idx], pz = a.gpz[idx];
        if (m == 0.0f && px == 0.0f && py == 0.0f && pz == 0.0f) continue;
        int ii[3] = {bx * B + l / (B * B), by * B + (l / B) % B, bz * B + l % B};
        if (a.cap) {
            long long c = a.cap_off[s] + ((long long)ii[0] * S.res + ii[1]) * S.res + ii[2];
            a.cap[4 * c] = m;
            a.cap[4 * c + 1] = px;
            a.cap[4 * c + 2] = py;
            a.cap[4 * c + 3] = pz;
        }
        float v[3] = {0.0f, 0.0f, 0.0f};
        if (m > 0.0f) {
            v[0] = px / m;
            v[1] = py / m;
            v[2] = pz / m;
        }
        for (int d = 0; d < 3; d++) v[d] += S.dt * S.g[d];
        float xi[3] = {ii[0] * S.dx, ii[1] * S.dx, ii[2] * S.dx};
        for (int c = 0; c < S.n_col; c++) collide_node(cn[c], xi, v);
        for (int d = 0; d < 3; d++) {
            if (ii[d] < S.bound && v[d] < 0.0f) v[d] = 0.0f;
            if (ii[d] >= S.res - S.bound && v[d] > 0.0f) v[d] = 0.0f;
        }
        a.gvx[idx] = v[0];
        a.gvy[idx] = v[1];
        a.gvz[idx] = v[2];
        a.gm[idx] = 0.0f;
        a.gpx[idx] = 0.0f;
        a.gpy[idx] = 0.0f;
        a.gpz[idx] = 0.0f;
    }
}

template <int B>
__global__ __launch_bounds__(WG) void k_grid(StepArgs a)
{
    const int lane = threadIdx.x & 63;
    const int nw = gridDim.x * (WG / 64);
    const int w0 = xcd_remap(blockIdx.x, gridDim.x) * (WG / 64) + (threadIdx.x >> 6);
    const int ng = *a.L.n_gitems;
    const int no = min(*a.L.n_ovf, a.L.ovf_cap);
    for (int w = w0; w < ng + no; w += nw) {
        int2 e = w < ng ? a.L.gitems[w] : a.L.ovf[w - ng];
        grid_block<B>(a, e.x, e.y, lane);
        if (w >= ng && lane == 0) a.L.bflag[a.scenes[e.x].bin_off + e.y] = 0;
    }
}

// ---------------------------------------------------------------- G2P + integration
template <int B>
__device__ void g2p_item(const StepArgs &a, const Item &item, float *vt)
{
    constexpr int T = B + 4, T3 = T * T * T;
    const int t = threadIdx.x;
    const int s = item.scene;
    const SceneDev &S = a.scenes[s];
    const int nb = S.nb;
    const int bx = item.block / (nb * nb), by = (item.block / nb) % nb, bz = item.block % nb;
    const int org[3] = {bx * B - 1, by * B - 1, bz * B - 1};
    for (int n = t; n < T3; n += WG) {
        int gi = org[0] + n / (T * T), gj = org[1] + (n / T) % T, gk = org[2] + n % T;
        float v0 = 0.0f, v1 = 0.0f, v2 = 0.0f;
        if (gi >= 0 && gj >= 0 && gk >= 0 && gi < S.res && gj < S.res && gk < S.res) {
            long long idx = node_index(S, B, gi, gj, gk);
            v0 = a.gvx[idx];
            v1 = a.gvy[idx];
            v2 = a.gvz[idx];
        }
        vt[n] = v0;
        vt[T3 + n] = v1;
        vt[2 * T3 + n] = v2;
    }
    __syncthreads();
    const Material mat = material_of(S);
    const float *P = a.P;
    float *Pw = a.P;
    const long long ps = a.pstride;
    int bad_any = 0, cl_any = 0;
    for (int li = t; li < item.count; li += WG) {
        const int j = item.start + li;
        float x[3], G[9];
#pragma unroll
        for (int d = 0; d < 3; d++) x[d] = P[(X0 + d) * ps + j];
#pragma unroll
        for (int e = 0; e < 9; e++) G[e] = P[(G00 + e) * ps + j];
        int b[3], cl = 0, in = 1;
        float f[3];
#pragma unroll
        for (int d = 0; d < 3; d++) {
            particle_base(S, x[d], b[d], f[d], cl);
            int tb = b[d] - org[d];
            in &= (tb >= 0) & (tb <= B + 1);
        }
        cl_any |= cl;
        float wx[3], wy[3], wz[3];
        bspline_w(f[0], wx);
        bspline_w(f[1], wy);
        bspline_w(f[2], wz);
        float vp[3] = {0.0f, 0.0f, 0.0f};
        float So[3][3] = {{0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}};   // sum w v_c o_e
        if (in) {
            const float *vb = vt + ((b[0] - org[0]) * T + (b[1] - org[1])) * T + (b[2] - org[2]);
#pragma unroll
            for (int ox = 0; ox < 3; ox++)
#pragma unroll
                for (int oy = 0; oy < 3; oy++) {
                    float wxy = wx[ox] * wy[oy];
#pragma unroll
                    for (int oz = 0; oz < 3; oz++) {
                        float w = wxy * wz[oz];
                        int o = (ox * T + oy) * T + oz;
                        float tv[3] = {w * vb[o], w * vb[T3 + o], w * vb[2 * T3 + o]};
#pragma unroll
                        for (int c = 0; c < 3; c++) {
                            vp[c] += tv[c];
                            if (ox) So[c][0] += (float)ox * tv[c];
                            if (oy) So[c][1] += (float)oy * tv[c];
                            if (oz) So[c][2] += (float)oz * tv[c];
                        }
                    }
                }
        } else {
            for (int ox = 0; ox < 3; ox++)
                for (int oy = 0; oy < 3; oy++)
                    for (int oz = 0; oz < 3; oz++) {
                        float w = wx[ox] * wy[oy] * wz[oz];
                        long long idx = node_index(S, B, b[0] + ox, b[1] + oy, b[2] + oz);
                        float tv[3] = {w * a.gvx[idx], w * a.gvy[idx], w * a.gvz[idx]};
                        for (int c = 0; c < 3; c++) {
                            vp[c] += tv[c];
                            So[c][0] += (float)ox * tv[c];
                            So[c][1] += (float)oy * tv[c];
                            So[c][2] += (float)oz * tv[c];
                        }
                    }
        }
        // C = (4/dx^2) sum w v (x_i - x_p)^T = (4/dx) (So - vp f^T)
        const float Dd = 4.0f * S.inv_dx;
        float C[9];
#pragma unroll
        for (int c = 0; c < 3; c++)
#pragma unroll
            for (int e = 0; e < 3; e++) C[3 * c + e] = Dd * (So[c][e] - vp[c] * f[e]);
#pragma unroll
        for (int d = 0; d < 3; d++) x[d] = fmaf(S.dt, vp[d], x[d]);
        // F <- (I + dt C) F  ->  G <- G + dt C + dt C G
        float Gt[9];
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int k = 0; k < 3; k++) {
                float acc = C[3 * i + k];
#pragma unroll
                for (int e = 0; e < 3; e++) acc = fmaf(C[3 * i + e], G[3 * e + k], acc);
                Gt[3 * i + k] = fmaf(S.dt, acc, G[3 * i + k]);
            }
        float tau[9], Gn[9];
        int bad = 0;
        if (mat.model == 0) {
            tau_neo_hookean(Gt, mat.mu, mat.la, tau, bad);
#pragma unroll
            for (int e = 0; e < 9; e++) Gn[e] = Gt[e];
        } else {
            hencky_update(Gt, mat, Gn, tau, bad);
        }
        bad |= !(isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]));
        bad_any |= bad;
#pragma unroll
        for (int d = 0; d < 3; d++) {
            Pw[(X0 + d) * ps + j] = x[d];
            Pw[(V0 + d) * ps + j] = vp[d];
        }
#pragma unroll
        for (int e = 0; e < 9; e++) {
            Pw[(A00 + e) * ps + j] = fmaf(S.mass, C[e], -S.kstress * tau[e]);
            Pw[(G00 + e) * ps + j] = Gn[e];
        }
    }
    if (bad_any) atomicOr(a.flags + s, (int)FLAG_NONFINITE);
    if (cl_any) atomicOr(a.flags + s, (int)FLAG_CLAMPED);
    __syncthreads();
}

template <int B>
__global__ __launch_bounds__(WG) void k_g2p(StepArgs a)
{
    constexpr int T = B + 4, T3 = T * T * T;
    __shared__ float vt[3 * T3];
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.L.n_ovf = 0;   // grid update has consumed the list
    const int n_items = *a.L.n_items;
    for (int it = xcd_remap(blockIdx.x, gridDim.x); it < n_items; it += gridDim.x) {
        Item item = a.L.items[it];
        g2p_item<B>(a, item, vt);
    }
}

hipError_t launch_p2g(const StepArgs &a, int chunk, int n_wg, hipStream_t st)
{
    n_wg = (n_wg + 7) & ~7;
    if (a.B == 4) {
        if (chunk <= 256) k_p2g<4, 1><<<n_wg, WG, 0, st>>>(a);
        else if (chunk <= 512) k_p2g<4, 2><<<n_wg, WG, 0, st>>>(a);
        else k_p2g<4, 4><<<n_wg, WG, 0, st>>>(a);
    } else {
        if (chunk <= 256) k_p2g<8, 1><<<n_wg, WG, 0, st>>>(a);
        else if (chunk <= 512) k_p2g<8, 2><<<n_wg, WG, 0, st>>>(a);
        else k_p2g<8, 4><<<n_wg, WG, 0, st>>>(a);
    }
    return hipGetLastError();
}

hipError_t launch_grid(const StepArgs &a, int n_wg, hipStream_t st)
{
    n_wg = (n_wg + 7) & ~7;
    if (a.B == 4) k_grid<4><<<n_wg, WG, 0, st>>>(a);
    else k_grid<8><<<n_wg, WG, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_g2p(const StepArgs &a, int n_wg, hipStream_t st)
{
    n_wg = (n_wg + 7) & ~7;
    if (a.B == 4) k_g2p<4><<<n_wg, WG, 0, st>>>(a);
    else k_g2p<8><<<n_wg, WG, 0, st>>>(a);
    return hipGetLastError();
}

// ====================================================================== colliders
__global__ void k_collider_advance(ColliderDev *cols, int n, const int *col_scene, const SceneDev *scenes, int steps)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    ColliderDev &cd = cols[c];
    float tk = (float)steps * scenes[col_scene[c]].dt;
    float q[4];
    quat_advance(cd.quat, cd.omega, tk, q);
    for (int d = 0; d < 3; d++) cd.pos[d] = fmaf(tk, cd.vlin[d], cd.pos[d]);
    for (int d = 0; d < 4; d++) cd.quat[d] = q[d];
}

hipError_t launch_collider_advance(ColliderDev *cols, int n_cols, const int *col_scene, const SceneDev *scenes,
                                   int n_substeps, hipStream_t st)
{
    if (n_cols > 0) k_collider_advance<<<(n_cols + 63) / 64, 64, 0, st>>>(cols, n_cols, col_scene, scenes, n_substeps);
    return hipGetLastError();
}

// ====================================================================== boundary conversions
__global__ __launch_bounds__(WG) void k_init_particles(const SceneDev *scenes, const int *psc, float *P,
                                                       long long ps, const float *x, const float *v, const float *C,
                                                       const float *F, int begin, int end)
{
    int i = begin + blockIdx.x * WG + threadIdx.x;
    if (i >= end) return;
    int k = i - begin;
    const SceneDev &S = scenes[psc[i]];
    Material mat = material_of(S);
    float G[9], Cm[9], tau[9];
    for (int e = 0; e < 9; e++) {
        G[e] = F ? F[9 * (long long)k + e] - (e % 4 == 0 ? 1.0f : 0.0f) : 0.0f;
        Cm[e] = C ? C[9 * (long long)k + e] : 0.0f;
    }
    int bad = 0;
    stress_of(G, mat, tau, bad);
    for (int d = 0; d < 3; d++) {
        P[(X0 + d) * ps + i] = x[3 * (long long)k + d];
        P[(V0 + d) * ps + i] = v ? v[3 * (long long)k + d] : 0.0f;
    }
    for (int e = 0; e < 9; e++) {
        P[(A00 + e) * ps + i] = fmaf(S.mass, Cm[e], -S.kstress * tau[e]);
        P[(G00 + e) * ps + i] = G[e];
    }
    P[PID * ps + i] = __int_as_float(i);
}

hipError_t launch_init_particles(const SceneDev *scenes, int n_scenes, const int *psc, float *P, long long pstride,
                                 const float *x, const float *v, const float *C, const float *F, int begin, int end,
                                 hipStream_t st)
{
    (void)n_scenes;
    if (end > begin) k_init_particles<<<(end - begin + WG - 1) / WG, WG, 0, st>>>(scenes, psc, P, pstride, x, v, C, F, begin, end);
    return hipGetLastError();
}

__global__ __launch_bounds__(WG) void k_get_state(const SceneDev *scenes, const int *psc, const float *P, long long ps,
                                                  int begin, int end, float *x, float *v, float *C, float *F)
{
    int j = begin + blockIdx.x * WG + threadIdx.x;
    if (j >= end) return;
    int p = __float_as_int(P[PID * ps + j]);
    long long k = p - begin;
    const SceneDev &S = scenes[psc[j]];
    for (int d = 0; d < 3; d++) {
        if (x) x[3 * k + d] = P[(X0 + d) * ps + j];
        if (v) v[3 * k + d] = P[(V0 + d) * ps + j];
    }
    float G[9];
    for (int e = 0; e < 9; e++) G[e] = P[(G00 + e) * ps + j];
    if (F)
        for (int e = 0; e < 9; e++) F[9 * k + e] = G[e] + (e % 4 == 0 ? 1.0f : 0.0f);
    if (C) {
        Material mat = material_of(S);
        float tau[9];
        int bad = 0;
        stress_of(G, mat, tau, bad);
        for (int e = 0; e < 9; e++) C[9 * k + e] = (P[(A00 + e) * ps + j] + S.kstress * tau[e]) / S.mass;
    }
}

hipError_t launch_get_state(const SceneDev *scenes, const int *psc, const float *P, long long pstride, int begin,
                            int end, float *x, float *v, float *C, float *F, hipStream_t st)
{
    if (end > begin) k_get_state<<<(end - begin + WG - 1) / WG, WG, 0, st>>>(scenes, psc, P, pstride, begin, end, x, v, C, F);
    return hipGetLastError();
}

__global__ void k_clear_f(float *p, long long n)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long st = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += st) p[i] = 0.0f;
}

hipError_t launch_clear_f(float *p, long long n, hipStream_t st)
{
    if (n > 0) {
        long long nb = (n + WG - 1) / WG;
        k_clear_f<<<(unsigned)(nb < 8192 ? nb : 8192), WG, 0, st>>>(p, n);
    }
    return hipGetLastError();
}

__global__ void k_reset_counters(int *queue, int *scene_done, int n, int *n_ovf)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && queue) queue[0] = 0;
    if (scene_done)
        for (int k = i; k < 3 * n; k += gridDim.x * blockDim.x) scene_done[k] = 0;
    (void)n_ovf;
}

hipError_t launch_reset_scene_counters(int *queue, int *scene_done, int n_scenes, int *n_ovf, hipStream_t st)
{
    k_reset_counters<<<1, WG, 0, st>>>(queue, scene_done, n_scenes, n_ovf);
    return hipGetLastError();
}

}  // namespace mpm
