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
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "mpm_device.hpp"
#include <hip/hip_ext.h>

namespace mpm {

// Timing of the substep kernels: events handed in by time_next_launch are
// recorded by the runtime at the start and the end of the next substep
// kernel launched on this thread (hipExtLaunchKernelGGL), so they time the
// kernel itself rather than the queue around it.
static thread_local hipEvent_t t_ev[2] = {nullptr, nullptr};

void time_next_launch(hipEvent_t start, hipEvent_t stop)
{
    t_ev[0] = start;
    t_ev[1] = stop;
}

template <typename... KArgs, typename... Args>
static void launch_timed(void (*kernel)(KArgs...), int n_wg, int nt, hipStream_t st, Args... args)
{
    hipEvent_t a = t_ev[0], b = t_ev[1];
    t_ev[0] = t_ev[1] = nullptr;
    if (a && b) hipExtLaunchKernelGGL(kernel, dim3(n_wg), dim3(nt), 0, st, a, b, 0, args...);
    else kernel<<<n_wg, nt, 0, st>>>(args...);
}

// ====================================================================== sort
// Runs of equal keys in consecutive lanes (the particles are nearly sorted
// from the previous sort): one atomic per run instead of one per particle.
struct KeyRun {
    int head_lane;   // first lane of this lane's run
    int len;         // run length (valid at the head lane)
};

__device__ __forceinline__ KeyRun key_run(unsigned key)
{
    const int lane = threadIdx.x & 63;
    const unsigned prev = __shfl_up(key, 1, 64);
    const bool head = lane == 0 || prev != key;
    const unsigned long long heads = __ballot(head);
    const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    KeyRun r;
    r.head_lane = 63 - __clzll(heads & upto);
    const unsigned long long after = heads & ~upto;
    const int next = after ? __ffsll((long long)after) - 1 : 64;
    r.len = next - lane;
    return r;
}

__device__ __forceinline__ unsigned particle_key(const SortArgs &a, int j)
{
    int s = a.psc[j];
    const SceneDev &S = a.scenes[s];
    int b[3], cl = 0;
    float f;
    for (int d = 0; d < 3; d++) particle_base(S, a.P[(long long)(X0 + d) * a.pstride + j], b[d], f, cl);
    return (unsigned)a.scene_bin_off[s] + morton3(b[0] / a.B, b[1] / a.B, b[2] / a.B);
}

__global__ __launch_bounds__(WG) void k_keys(SortArgs a)
{
    const int j = blockIdx.x * WG + threadIdx.x;
    const bool valid = j < a.N;
    const unsigned key = valid ? particle_key(a, j) : 0xFFFFFFFFu;
    if (valid) a.keys[j] = key;
    const KeyRun r = key_run(key);
    if (valid && r.head_lane == (int)(threadIdx.x & 63)) atomicAdd(&a.count[key], r.len);
}

// Grid blocks that receive mass from particles at home in their bin: the
// block itself and its upper neighbours (a stencil spans base .. base + 2).
// Mass a drifted particle puts one block lower is queued on the overflow
// list by P2G itself.
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
    for (int dx = -1; dx <= 0; dx++)
        for (int dy = -1; dy <= 0; dy++)
            for (int dz = -1; dz <= 0; dz++) {
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

// Inside its bin a particle's slot is scrambled (local rank r -> r * 104729 mod
// bin size, a bijection unless the prime divides the size, which then keeps
// r), so a bin's
// particles end up in an order unrelated to space: consecutive lanes of a
// P2G wave then land on distant cells, and their LDS atomics rarely collide
// on an address or a bank.  (In the order of the previous sort they arrive
// clustered cell by cell.)
constexpr long long BIN_SCRAMBLE = 104729;   // prime

__global__ __launch_bounds__(WG) void k_scatter(SortArgs a)
{
    const int j = blockIdx.x * WG + threadIdx.x;
    const bool valid = j < a.N;
    const unsigned key = valid ? a.keys[j] : 0xFFFFFFFFu;
    const KeyRun r = key_run(key);
    const int lane = threadIdx.x & 63;
    int old = 0;
    if (valid && r.head_lane == lane) old = atomicSub(&a.count[key], r.len);
    old = __shfl(old, r.head_lane, 64);
    // the run takes the local ranks [old - len, old) in lane order
    const int len = __shfl(r.len, r.head_lane, 64);
    if (valid) {
        const int b0 = a.pstart[key];
        const int size = ((int)key + 1 < a.T ? a.pstart[key + 1] : a.N) - b0;
        const int local = old - len + (lane - r.head_lane);
        const long long mul = (size % BIN_SCRAMBLE) ? BIN_SCRAMBLE : 1;   // a bijection for any size
        a.perm[b0 + (int)(((long long)local * mul) % size)] = j;
    }
}

// Order inside a work item so that the lanes of a P2G wave scatter into
// distinct LDS banks.  A particle's bank class is the tile address of its
// base node mod 64; every stencil offset adds the same constant to all
// lanes, so lanes with distinct classes hit distinct banks.  Particles are
// ranked inside their class and laid out by (rank, class): the first 64
// slots hold rank 0 of every class present, the next ones rank 1, and so on.
// Slot of (rank r, class c) = sum_c' min(count[c'], r) + #{c' < c : count[c'] > r}.
// Edge of a work item's node tile (P2G sums, G2P velocities) for grid blocks of
// edge B: the tile starts one node below the block, and a particle is handled
// in it while its base cell lies at tile coordinates 0 .. B, i.e. in the
// block (1 .. B, where the sort put it) or one cell below; its stencil then
// reaches tile nodes 0 .. B + 2.  Particles past that range since the last
// re-sort take the global path.  The material of the substep workloads sinks
// and is pushed down: the allowance below is the one that matters (on the
// measured runs at most 0.07 % of the particles leave this range between
// re-sorts every 50 substeps, 0.6 % with the allowance above instead).
template <int B> constexpr int tile_edge() { return B + 3; }
// Largest base-cell tile coordinate of a particle handled in the tile.
template <int B> constexpr int tile_bmax() { return tile_edge<B>() - 3; }

constexpr int BANK_CLASSES = 64;

template <int B>
__global__ __launch_bounds__(WG) void k_bank_order(SortArgs a)
{
    constexpr int T = tile_edge<B>();
    __shared__ int cnt[BANK_CLASSES];
    __shared__ unsigned short rank[8192];
    __shared__ unsigned char cls[8192];
    const int n_items = *a.L.n_items;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item item = a.L.items[it];
        if (threadIdx.x < BANK_CLASSES) cnt[threadIdx.x] = 0;
        __syncthreads();
        const SceneDev &S = a.scenes[item.scene];
        const int nb = S.nb;
        const int org[3] = {(item.block / (nb * nb)) * B - 1, ((item.block / nb) % nb) * B - 1, (item.block % nb) * B - 1};
        for (int li = threadIdx.x; li < item.count; li += WG) {
            const int j = a.perm[item.start + li];
            int tb[3], cl = 0;
            float f;
            for (int d = 0; d < 3; d++) {
                int b;
                particle_base(S, a.P[(long long)(X0 + d) * a.pstride + j], b, f, cl);
                tb[d] = min(max(b - org[d], 0), T - 1);
            }
            const int c = ((tb[0] * T + tb[1]) * T + tb[2]) % BANK_CLASSES;
            cls[li] = (unsigned char)c;
            rank[li] = (unsigned short)atomicAdd(&cnt[c], 1);
        }
        __syncthreads();
        for (int li = threadIdx.x; li < item.count; li += WG) {
            const int c = cls[li], r = rank[li];
            int pos = 0;
            for (int q = 0; q < BANK_CLASSES; q++) {
                const int k = cnt[q];
                pos += min(k, r) + ((q < c && k > r) ? 1 : 0);
            }
            a.perm2[item.start + pos] = a.perm[item.start + li];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(WG) void k_gather(SortArgs a)
{
    // contiguous share per XCD: the sources of a bin (scattered over that
    // bin's old range) are fetched into one L2 rather than into all eight
    int p = xcd_remap(blockIdx.x, gridDim.x) * WG + threadIdx.x;
    if (p >= a.N) return;
    int j = a.perm2[p];
    // all loads before any store: the compiler cannot tell that the two
    // buffers do not overlap, and would otherwise wait for each store
    const float *__restrict__ src = a.P;
    float *__restrict__ dst = a.Pn;
    float v[NCOMP];
#pragma unroll
    for (int c = 0; c < NCOMP; c++) v[c] = src[(long long)c * a.pstride + j];
#pragma unroll
    for (int c = 0; c < NCOMP; c++) dst[(long long)c * a.pstride + p] = v[c];
}

// Dispatch order of the work items for P2G and G2P: most particles first.
// Those kernels take one item per workgroup in workgroup order (the
// dispatcher deals workgroups to the XCDs in turn, so each XCD gets every
// eighth item of the order), and items range from a few dozen particles to
// a full chunk: in block order the largest ones could start last and hold
// the end of the launch.  A counting sort by particle count in 64 classes
// (order inside a class: arbitrary).
constexpr int ORDER_CLASSES = 64;

__device__ __forceinline__ int order_class(int count, int CH)
{
    return min(ORDER_CLASSES - 1, (int)((long long)count * ORDER_CLASSES / (CH + 1)));
}

__global__ __launch_bounds__(1024) void k_item_order(SortArgs a)
{
    __shared__ int cnt[ORDER_CLASSES];
    const int n = *a.L.n_items;
    if (threadIdx.x < ORDER_CLASSES) cnt[threadIdx.x] = 0;
    __syncthreads();
    for (int it = threadIdx.x; it < n; it += blockDim.x) atomicAdd(&cnt[order_class(a.L.items[it].count, a.CH)], 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;   // classes from the largest down: cnt[c] becomes the first slot of class c
        for (int c = ORDER_CLASSES - 1; c >= 0; c--) {
            const int k = cnt[c];
            cnt[c] = s;
            s += k;
        }
    }
    __syncthreads();
    for (int it = threadIdx.x; it < n; it += blockDim.x)
        a.L.order[atomicAdd(&cnt[order_class(a.L.items[it].count, a.CH)], 1)] = it;
}

// Scale bound of every new work item (the P2G fixed-point scale), from the
// freshly gathered particles.
__global__ __launch_bounds__(WG) void k_item_bounds(SortArgs a)
{
    __shared__ float red[WG / 64];
    const int n_items = *a.L.n_items;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item item = a.L.items[it];
        const SceneDev &S = a.scenes[item.scene];
        float b = 0.0f;
        for (int li = threadIdx.x; li < item.count; li += WG) {
            const long long j = item.start + li;
            float v[3], A[9];
            for (int d = 0; d < 3; d++) v[d] = a.Pn[(V0 + d) * a.pstride + j];
            for (int e = 0; e < 9; e++) A[e] = a.Pn[(A00 + e) * a.pstride + j];
            b = fmaxf(b, scatter_bound(S.mass, S.dx, v, A));
        }
        b = wave_max(b);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = b;
        __syncthreads();
        if (threadIdx.x == 0) {
            a.L.ibound[it] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
            a.L.icell[it] = 0;   // per-cell counts unknown: the next P2G counts
        }
        __syncthreads();
    }
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
    k_item_order<<<1, 1024, 0, st>>>(a);
    if (a.N > 0) {
        const int gN8 = (gN + 7) & ~7;    // xcd_remap (gather) needs a multiple of 8 workgroups
        k_scatter<<<gN, WG, 0, st>>>(a);
        if (a.B == 4) k_bank_order<4><<<2048, WG, 0, st>>>(a);
        else k_bank_order<8><<<2048, WG, 0, st>>>(a);
        k_gather<<<gN8, WG, 0, st>>>(a);
        k_item_bounds<<<2048, WG, 0, st>>>(a);
    }
    return hipGetLastError();
}

// ====================================================================== substep pieces
__device__ __forceinline__ void load_particle_xvA(const StepArgs &a, int jj, float x[3], float v[3], float A[9])
{
    const float *P = a.P;
    const long long ps = a.pstride;
    const unsigned jo = (unsigned)jj << 2;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        x[d] = pload(P, ps, X0 + d, jo);
        v[d] = pload(P, ps, V0 + d, jo);
    }
#pragma unroll
    for (int e = 0; e < 9; e++) A[e] = pload(P, ps, A00 + e, jo);
}

// Length of the overflow list of substep k.  Two counters alternate by
// substep parity: the G2P of substep k clears counter k & 1 (its grid update
// has consumed the list) while a P2G fused into the same launch already
// fills the list of substep k + 1; at the end of every substep both are zero.
__device__ __forceinline__ int *ovf_count(const StepArgs &a, int k) { return a.L.n_ovf + (k & 1); }

// Put a grid block that is not on the static update list on the overflow
// list (once per substep); n_ovf: the list length of the substep that
// scatters.
__device__ __forceinline__ void queue_block(const StepArgs &a, int s, int bin_off, int lb, int *n_ovf)
{
    int *fl = a.L.bflag + bin_off + lb;
    if (*fl == 0 && atomicCAS(fl, 0, 1) == 0) {
        int pos = atomicAdd(n_ovf, 1);
        if (pos < a.L.ovf_cap) a.L.ovf[pos] = make_int2(s, lb);
        else atomicOr(a.flags + s, (int)FLAG_OVERFLOW_FULL);
    }
}

// Slow path of P2G: scatter one particle straight into the global grid and
// queue any block that is not already on the grid-update list.  home: grid
// block of the particle's work item; that block and its upper neighbours are
// on the list from the sort on, so only blocks outside them are checked (each
// check waits for a global round trip).  The scene constants are copied into
// registers first: the atomics may alias the scene record for the compiler,
// which would otherwise reload it, waiting for every atomic issued so far,
// before each one.
template <int B>
__device__ void p2g_global(const StepArgs &a, int s, const SceneDev &S, const float x[3], const float v[3],
                           const float A[9], const int b[3], const float f[3], int *n_ovf, int3 home)
{
    const float mass = uniform_f(S.mass), dx = uniform_f(S.dx);
    const int nb = uniform_i(S.nb), bin_off = uniform_i(S.bin_off);
    const SceneDev Sg = {0, 0, uniform_i(S.res), nb, uniform_ll(S.grid_off)};
    float w[3][3];
#pragma unroll
    for (int d = 0; d < 3; d++) bspline_w(f[d], w[d]);
#pragma unroll
    for (int ox = 0; ox < 3; ox++)
#pragma unroll
        for (int oy = 0; oy < 3; oy++)
#pragma unroll
            for (int oz = 0; oz < 3; oz++) {
                const float wt = w[0][ox] * w[1][oy] * w[2][oz];
                const float d[3] = {(ox - f[0]) * dx, (oy - f[1]) * dx, (oz - f[2]) * dx};
                const long long idx = node_index(Sg, B, b[0] + ox, b[1] + oy, b[2] + oz);
                atomicAdd(a.gm + idx, wt * mass);
                atomicAdd(a.gpx + idx, wt * (mass * v[0] + A[0] * d[0] + A[1] * d[1] + A[2] * d[2]));
                atomicAdd(a.gpy + idx, wt * (mass * v[1] + A[3] * d[0] + A[4] * d[1] + A[5] * d[2]));
                atomicAdd(a.gpz + idx, wt * (mass * v[2] + A[6] * d[0] + A[7] * d[1] + A[8] * d[2]));
            }
#pragma unroll
    for (int cx = 0; cx < 2; cx++)
#pragma unroll
        for (int cy = 0; cy < 2; cy++)
#pragma unroll
            for (int cz = 0; cz < 2; cz++) {
                const int bx = (b[0] + 2 * cx) / B, by = (b[1] + 2 * cy) / B, bz = (b[2] + 2 * cz) / B;
                if ((cx && bx == b[0] / B) || (cy && by == b[1] / B) || (cz && bz == b[2] / B)) continue;
                const int lb = (bx * nb + by) * nb + bz;
                a.L.touched[bin_off + lb] = 1;
                if ((unsigned)(bx - home.x) > 1u || (unsigned)(by - home.y) > 1u || (unsigned)(bz - home.z) > 1u)
                    queue_block(a, s, bin_off, lb, n_ovf);
            }
}


// Rounding by addition: RND = 1.5 * 2^23, whose float spacing is 1 for sums in [2^23, 2^24).
constexpr float RND = 12582912.0f;
constexpr unsigned long long RND_PAIR = 0x4B4000004B400000ull;   // RND's bits in both halves

// Base cells a particle of a P2G tile can have (tile coordinates 0 .. tile_bmax).
template <int B> constexpr int p2g_cells() { return (tile_bmax<B>() + 1) * (tile_bmax<B>() + 1) * (tile_bmax<B>() + 1); }

// Items with more particles than this count their particles per base cell
// before scattering (below it the per-term limit already sets the scale).
constexpr int P2G_COUNT_MIN = 256;

// Power-of-two fixed-point scales of the P2G tile, keeping every node sum
// below 2^30: |contribution| <= w * bound with the weights of a node summing
// to at most wsum; and every single term within 2^22 (w <= 0.421875; rounded
// by the RND addition of scatter_packed).  A particle may be scattered into
// the tile while its scatter bound b satisfies b * sp <= lim.
struct TileScale {
    float msc;   // Sm m: mass-scaled weights
    float kk;    // Sp / (Sm m): momentum scale relative to the mass-scaled weight
    float sp;    // Sp
    float lim;
    float im, ip;   // 1 / Sm, 1 / Sp
};

__device__ __forceinline__ TileScale tile_scale(const SceneK &K, float wsum, float bmax)
{
    TileScale ts;
    ts.lim = fminf(1073741824.0f / wsum, 4194304.0f / 0.421875f);
    int em = ilogbf(ts.lim / K.mass);
    em = min(max(em, -120), 120);
    int ep = bmax > 0.0f ? ilogbf(ts.lim / bmax) : 120;
    ep = min(max(ep, -120), 120);
    const float Sm = ldexpf(1.0f, em), Sp = ldexpf(1.0f, ep);
    ts.kk = Sp / (Sm * K.mass);
    ts.msc = Sm * K.mass;
    ts.sp = Sp;
    ts.im = 1.0f / Sm;
    ts.ip = 1.0f / Sp;
    return ts;
}

// One particle's 27 stencil terms into the tile t64 (per node two 64-bit sums,
// (p_x, m) and (p_y, p_z) as (hi, lo), each the exact sum of 32-bit fixed-point
// terms packed as hi * 2^32 + lo: an integer sum, so both halves are recovered
// exactly while they fit in 32 bits); tb: the particle's base cell in tile
// coordinates, f its offset from it in cells.
template <int B>
__device__ __forceinline__ void scatter_packed(long long *t64, const int tb[3], const float f[3], const TileScale &ts,
                                               const SceneK &K, const float v[3], const float A[9])
{
    constexpr int T = tile_edge<B>(), T3 = T * T * T;
    float wx[3], wy[3], wz[3];
    bspline_w(f[0], wx);
    bspline_w(f[1], wy);
    bspline_w(f[2], wz);
#pragma unroll
    for (int o = 0; o < 3; o++) wx[o] *= ts.msc;
    // r(o) = kk * (m v + A (o - f) dx); increments along each axis
    float Ad[3][3], r0[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
#pragma unroll
        for (int e = 0; e < 3; e++) Ad[c][e] = ts.kk * A[3 * c + e] * K.dx;
        r0[c] = ts.kk * K.mass * v[c] - (Ad[c][0] * f[0] + Ad[c][1] * f[1] + Ad[c][2] * f[2]);
    }
    long long *tb0 = t64 + (tb[0] * T + tb[1]) * T + tb[2];
    // r at offset (ox, oy, oz): r0 + ox Ad_x + oy Ad_y + oz Ad_z, one add per axis step
    // (offset 0 adds nothing, 1 adds Ad, 2 adds 2 Ad)
    auto step = [](float r, float d, int o) { return o == 0 ? r : (o == 1 ? r + d : fmaf(2.0f, d, r)); };
#pragma unroll
    for (int ox = 0; ox < 3; ox++)
#pragma unroll
        for (int oy = 0; oy < 3; oy++) {
            float wxy = wx[ox] * wy[oy];
            float rxy[3];
#pragma unroll
            for (int c = 0; c < 3; c++) rxy[c] = step(step(r0[c], Ad[c][0], ox), Ad[c][1], oy);
#pragma unroll
            for (int oz = 0; oz < 3; oz++) {
                float w = wxy * wz[oz];
                int o = (ox * T + oy) * T + oz;
                // x + RND (|x| <= 2^22) holds round(x) in its low mantissa bits: bits = RND_BITS + round(x).
                // A pair of such bit patterns as hi * 2^32 + lo, minus RND_BITS * (2^32 + 1), is
                // round(x_hi) * 2^32 + round(x_lo) exactly (one 64-bit subtraction per pair).
                const unsigned b0 = __float_as_uint(fmaf(wxy, wz[oz], RND));   // mass term
                const unsigned b1 = __float_as_uint(fmaf(w, step(rxy[0], Ad[0][2], oz), RND));
                const unsigned b2 = __float_as_uint(fmaf(w, step(rxy[1], Ad[1][2], oz), RND));
                const unsigned b3 = __float_as_uint(fmaf(w, step(rxy[2], Ad[2][2], oz), RND));
                atomicAdd((unsigned long long *)(tb0 + o), ((unsigned long long)b1 << 32 | b0) - RND_PAIR);
                atomicAdd((unsigned long long *)(tb0 + T3 + o), ((unsigned long long)b2 << 32 | b3) - RND_PAIR);
            }
        }
}

// The tile's node sums into the global grid: marks the grid blocks that
// received mass, queues lower neighbour blocks off the update list.
template <int B, int NT>
__device__ void flush_packed(const StepArgs &a, int s, const SceneDev &S, const int org[3], const long long *t64,
                             const TileScale &ts, int *n_ovf)
{
    constexpr int T = tile_edge<B>(), T3 = T * T * T;
    const int home[3] = {(org[0] + 1) / B, (org[1] + 1) / B, (org[2] + 1) / B};
    // neighbour blocks (home - 1 .. home + 1 per axis, bit (cx * 3 + cy) * 3 + cz) below the home
    // block along some axis that received mass: queued once per wave after the node loop (the
    // home block and its upper neighbours are on the update list already)
    unsigned lower = 0;
    // scene constants in registers: the grid atomics may alias the scene record for the
    // compiler, which would otherwise reload it (waiting for the atomics) on every node
    const int res = uniform_i(S.res), nb = uniform_i(S.nb), bin_off = uniform_i(S.bin_off);
    const SceneDev Sg = {0, 0, res, nb, uniform_ll(S.grid_off)};
    for (int n = threadIdx.x; n < T3; n += NT) {
        int m0, p0, p1, p2;
        unpack2(t64[n], p0, m0);
        unpack2(t64[T3 + n], p1, p2);
        if ((m0 | p0 | p1 | p2) == 0) continue;
        int tx = n / (T * T), ty = (n / T) % T, tz = n % T;
        int gi = org[0] + tx, gj = org[1] + ty, gk = org[2] + tz;
        if (gi < 0 || gj < 0 || gk < 0 || gi >= res || gj >= res || gk >= res) continue;
        const int lb = ((gi / B) * nb + (gj / B)) * nb + (gk / B);
        a.L.touched[bin_off + lb] = 1;
        if (tx == 0 || ty == 0 || tz == 0)
            lower |= 1u << (((gi / B - home[0] + 1) * 3 + (gj / B - home[1] + 1)) * 3 + (gk / B - home[2] + 1));
        const long long idx = node_index(Sg, B, gi, gj, gk);
        atomicAdd(a.gm + idx, (float)m0 * ts.im);
        atomicAdd(a.gpx + idx, (float)p0 * ts.ip);
        atomicAdd(a.gpy + idx, (float)p1 * ts.ip);
        atomicAdd(a.gpz + idx, (float)p2 * ts.ip);
    }
    lower = wave_or(lower);
    const int lane = threadIdx.x & 63;
    if (lane < 27 && ((lower >> lane) & 1u)) {
        const int lb = ((home[0] - 1 + lane / 9) * nb + (home[1] - 1 + (lane / 3) % 3)) * nb + (home[2] - 1 + lane % 3);
        queue_block(a, s, bin_off, lb, n_ovf);
    }
}

template <int B, int NT = WG>
__device__ void p2g_item(const StepArgs &a, int it, const Item &item, int *tile, int *cells)
{
    constexpr int T = tile_edge<B>(), T3 = T * T * T, NC = p2g_cells<B>();
    const int t = threadIdx.x;
    const int s = item.scene;
    const SceneDev &S = a.scenes[s];
    const int nb = S.nb;
    const int bx = item.block / (nb * nb), by = (item.block / nb) % nb, bz = item.block % nb;
    const int org[3] = {bx * B - 1, by * B - 1, bz * B - 1};
    const int3 home = make_int3(bx, by, bz);
    const SceneK K = scene_k(S);
    // largest particle count of a base cell, left by the G2P that moved the
    // particles (0 after a re-sort or a surrogate step: count here)
    const int known = item.count > P2G_COUNT_MIN ? a.L.icell[it] : 0;
    const bool count_cells = item.count > P2G_COUNT_MIN && known <= 0;

    // the first particle's state is in flight while the tile is cleared; the
    // next one's is loaded while the current one scatters
    float xn[3], vn[3], An[9];
    if (t < item.count) load_particle_xvA(a, item.start + t, xn, vn, An);
    // LDS tile: per node two 64-bit sums, (p_x, m) and (p_y, p_z) as (hi, lo),
    // each the exact sum of 32-bit fixed-point terms packed as hi * 2^32 + lo
    // (an integer sum, so both halves are recovered exactly while they fit in
    // 32 bits)
    long long *t64 = (long long *)tile;
    for (int n = t; n < 2 * T3; n += NT) t64[n] = 0;
    if (count_cells) {
        for (int n = t; n < NC + 1; n += NT) cells[n] = 0;   // cells[NC]: the maximum
    }
    // bound of this item's particles, left by the previous G2P (or the sort)
    const float bmax = a.L.ibound[it];
    __syncthreads();
    if (t == 0 && !a.keep_bound && !a.chain) a.L.ibound[it] = 0.0f;   // this substep's G2P accumulates the next bound

    // Node sums of weights: a node receives w <= 0.5, 0.75, 0.5 per axis from
    // particles whose base cell is 0, 1, 2 cells below it, so the weights
    // reaching one node add up to at most 1.75^3 = 5.359375 times the largest
    // number of particles sharing a base cell (and never more than
    // 0.421875 * count).  Large items count their particles per base cell
    // first (the same in-tile test as the scatter below).
    float wsum = 0.421875f * (float)item.count;
    if (count_cells) {
        for (int base = 0; base < item.count; base += NT) {
            const int li = base + t;
            if (li >= item.count) break;
            const unsigned jo = (unsigned)(item.start + li) << 2;
            int cl = 0, in = 1, c = 0;
#pragma unroll
            for (int d = 0; d < 3; d++) {
                int bp;
                float f;
                particle_base(K, pload(a.P, a.pstride, X0 + d, jo), bp, f, cl);
                const int tb = bp - org[d];
                in &= (tb >= 0) & (tb <= tile_bmax<B>());
                c = c * (tile_bmax<B>() + 1) + tb;
            }
            if (in && !cl) atomicAdd(cells + c, 1);
        }
        __syncthreads();
        int mx = 0;
        for (int n = t; n < NC; n += NT) mx = max(mx, cells[n]);
        mx = wave_max_i(mx);
        if ((t & 63) == 0) atomicMax(cells + NC, mx);
        __syncthreads();
        if (a.chain && t == 0) a.L.icell[it] = cells[NC];   // the fused G2P's scale
        wsum = fminf(wsum, 5.359375f * (float)max(cells[NC], 1));
    } else if (known > 0) {
        wsum = fminf(wsum, 5.359375f * (float)known);
    }

    const TileScale ts = tile_scale(K, wsum, bmax);

    for (int li = t; li < item.count; li += NT) {
        float x[3], v[3], A[9], f[3];
#pragma unroll
        for (int d = 0; d < 3; d++) {
            x[d] = xn[d];
            v[d] = vn[d];
        }
#pragma unroll
        for (int e = 0; e < 9; e++) A[e] = An[e];
        if (li + NT < item.count) load_particle_xvA(a, item.start + li + NT, xn, vn, An);
        int bp[3];
        int cl = 0, in = 1;
#pragma unroll
        for (int d = 0; d < 3; d++) {
            particle_base(K, x[d], bp[d], f[d], cl);
            int tb = bp[d] - org[d];
            in &= (tb >= 0) & (tb <= tile_bmax<B>());
        }
        if (cl) atomicOr(a.flags + s, (int)FLAG_CLAMPED);
        if (!in || cl) {
            p2g_global<B>(a, s, S, x, v, A, bp, f, ovf_count(a, a.substep), home);
            continue;
        }
        const int tb[3] = {bp[0] - org[0], bp[1] - org[1], bp[2] - org[2]};
        scatter_packed<B>(t64, tb, f, ts, K, v, A);
    }
    __syncthreads();
    flush_packed<B, NT>(a, s, S, org, t64, ts, ovf_count(a, a.substep));
    __syncthreads();
}

template <int B, int NT>
__global__ __launch_bounds__(NT, 5) void k_p2g(StepArgs a)
{
    constexpr int T = tile_edge<B>(), T3 = T * T * T;
    __shared__ __align__(16) int tile[4 * T3];
    __shared__ int cells[p2g_cells<B>() + 1];
    const int n_items = *a.L.n_items;
    const int G = active_wgs(n_items);
    if ((int)blockIdx.x >= G) return;
    // items in dispatch order, most particles first (L.order)
    for (int r = blockIdx.x; r < n_items; r += G) {
        const int it = a.L.order[r];
        Item item = a.L.items[it];
        if (!a.active[item.scene]) continue;
        p2g_item<B, NT>(a, it, item, tile, cells);
    }
}

// ---------------------------------------------------------------- grid update
// cl: this wave's LDS copy of the scene's colliders (at most
// MAX_COLLIDERS_PER_SCENE).
// The node loop stores to the grid; reading the colliders and the scene
// constants from LDS and registers keeps the compiler from reloading them
// from global memory (and waiting for the stores) on every node.
// EXTRA = false: a plain substep (no capture, no surrogate arrays), built
// without that code so that it keeps its registers and occupancy.
template <int B, bool EXTRA = true>
__device__ void grid_block(const StepArgs &a, int s, int lb, int lane, ColliderNow *cl)
{
    const SceneDev &S = a.scenes[s];
    unsigned char *tf = a.L.touched + S.bin_off + lb;
    if (!*tf) return;          // no P2G wrote into this block: every (m, p) in it is zero
    const int nb = S.nb;
    const int bx = lb / (nb * nb), by = (lb / nb) % nb, bz = lb % nb;
    const int n_col = __builtin_amdgcn_readfirstlane(S.n_col);
    const int bound = __builtin_amdgcn_readfirstlane(S.bound);
    const SceneK K = scene_k(S);
    const float gdt[3] = {K.dt * uniform_f(S.g[0]), K.dt * uniform_f(S.g[1]), K.dt * uniform_f(S.g[2])};
    const long long goff = S.grid_off;
    {
        // this substep's collider poses, one lane per collider
        if (lane < n_col) {
            ColliderNow cn;
            collider_at(a.cols[S.col_off + lane], (float)a.substep * K.dt, cn);
            cl[lane] = cn;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // B^3 is a multiple of 64: every lane runs every iteration, so the wave sums of the
    // collider wrenches below see all lanes (a lane on an empty node adds zero)
    for (int l = lane; l < B * B * B; l += 64) {
        long long idx = goff + (long long)lb * (B * B * B) + l;
        float m = a.gm[idx], px = a.gpx[idx], py = a.gpy[idx], pz = a.gpz[idx];
        const bool live = !(m == 0.0f && px == 0.0f && py == 0.0f && pz == 0.0f);
        if (!__any(live)) continue;
        int ii[3] = {bx * B + l / (B * B), by * B + (l / B) % B, bz * B + l % B};
        if (EXTRA && a.cap && live) {
            long long c = a.cap_off[s] + ((long long)ii[0] * K.res + ii[1]) * K.res + ii[2];
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
        for (int d = 0; d < 3; d++) v[d] += gdt[d];
        float xi[3] = {ii[0] * K.dx, ii[1] * K.dx, ii[2] * K.dx};
        for (int c = 0; c < (a.contact == 1 ? 0 : n_col); c++) {   // contact 1: particle penalty only
            const float v0[3] = {v[0], v[1], v[2]};
            const bool hit = collide_node(cl[c], xi, v, a.sdf) && live && m > 0.0f;
            // two-way coupling: the collider receives minus the momentum its projection gives
            // the node, and minus its moment about the collider centre; one wave sum and one
            // atomic per component, only where the wave touched this collider
            if (a.wrench && __any(hit)) {
                float dp[3], r[3];
                for (int d = 0; d < 3; d++) {
                    dp[d] = hit ? m * (v[d] - v0[d]) : 0.0f;
                    r[d] = xi[d] - cl[c].c[d];
                }
                const float w6[6] = {dp[0], dp[1], dp[2], r[1] * dp[2] - r[2] * dp[1], r[2] * dp[0] - r[0] * dp[2],
                                     r[0] * dp[1] - r[1] * dp[0]};
                float *acc = a.wrench + 6 * (long long)(S.col_off + c);
                float tot[6];
#pragma unroll
                for (int j = 0; j < 6; j++) tot[j] = wave_total(w6[j]);
                if (lane == 0)
#pragma unroll
                    for (int j = 0; j < 6; j++) atomicAdd(acc + j, -tot[j]);
            }
        }
        if (!live) continue;
        for (int d = 0; d < 3; d++) {
            if (ii[d] < bound && v[d] < 0.0f) v[d] = 0.0f;
            if (ii[d] >= K.res - bound && v[d] > 0.0f) v[d] = 0.0f;
        }
        const long long c = EXTRA && a.dense ? sur_index(a, s, K.res, ii[0], ii[1], ii[2]) : -1;
        if (EXTRA && a.dense && c < 0 && a.out_mass && m > 0.0f) atomicAdd(a.out_mass + s, m);   // outside the box
        if (EXTRA && c >= 0) {   // (m, p / m) of the P2G, before gravity, colliders and walls
            const float im = m > 0.0f ? 1.0f / m : 0.0f;
            *(float4 *)(a.dense + 4 * c) = make_float4(m, px * im, py * im, pz * im);
            if (a.feat) {
                const float inv = S.vol / (S.mass * S.dx * S.dx * S.dx);   // 1 / (rho dx^3)
                float *fp = a.feat + c * a.cf;
                fp[0] = m * inv;
                fp[1] = px * inv * (1.0f / SUR_VEL);
                fp[2] = py * inv * (1.0f / SUR_VEL);
                fp[3] = pz * inv * (1.0f / SUR_VEL);
            }
        }
        a.gvx[idx] = v[0];
        a.gvy[idx] = v[1];
        a.gvz[idx] = v[2];
        a.gm[idx] = 0.0f;
        a.gpx[idx] = 0.0f;
        a.gpy[idx] = 0.0f;
        a.gpz[idx] = 0.0f;
    }
    if (lane == 0) *tf = 0;
}

// The wave that takes the first static grid block of scene s also leaves the
// scene's collider poses of this substep in a.colnow for the G2P (penalty
// contact reads them there).
__device__ __forceinline__ void publish_colliders(const StepArgs &a, int w, int s, int lane)
{
    if (w != a.L.scene_gitem_begin[s]) return;
    const SceneDev &S = a.scenes[s];
    if (lane < S.n_col) {
        ColliderNow cn;
        collider_at(a.cols[S.col_off + lane], (float)a.substep * S.dt, cn);
        ((ColliderNow *)a.colnow)[S.col_off + lane] = cn;
    }
}

template <int B, bool EXTRA>
__global__ __launch_bounds__(WG, (B == 8 && !EXTRA) ? 7 : 1) void k_grid(StepArgs a)
{
    const int lane = threadIdx.x & 63;
    __shared__ ColliderNow cls[WG / 64][MAX_COLLIDERS_PER_SCENE];
    const int ng = *a.L.n_gitems;
    const int no = min(*ovf_count(a, a.substep), a.L.ovf_cap);
    const int G = active_wgs((ng + no + WG / 64 - 1) / (WG / 64));
    if ((int)blockIdx.x >= G) return;
    const int nw = G * (WG / 64);
    const int w0 = xcd_remap(blockIdx.x, G) * (WG / 64) + (threadIdx.x >> 6);
    for (int w = w0; w < ng + no; w += nw) {
        int2 e = w < ng ? a.L.gitems[w] : a.L.ovf[w - ng];
        if (w < ng) publish_colliders(a, w, e.x, lane);
        grid_block<B, EXTRA>(a, e.x, e.y, lane, cls[threadIdx.x >> 6]);
        if (w >= ng && lane == 0) a.L.bflag[a.scenes[e.x].bin_off + e.y] = 0;
    }
}

// ---------------------------------------------------------------- G2P + integration
// PEN: particle penalty contact after the position update (MPM_OPT_CONTACT 1 or 2).
// cells: LDS of p2g_cells<B>() + 1 ints; the item's particles are counted per
// base cell of their new position (as the next P2G's tile sees them) and the
// largest count is left in L.icell[it] for that P2G's fixed-point scale.
// FUSE: the P2G of substep a.substep + 1 follows in the same pass: each
// particle, once advanced, is scattered from registers into the fixed-point
// LDS tile t64 (as p2g_item's), which is flushed to the grid at the end of the
// item; only x and G are stored (v and A live on in the grid, and the G2P
// that ends the run of fused substeps stores them).  The tile's scale has to
// be fixed before any particle has moved, so it comes from the state this
// G2P starts from: the largest particle count of a base cell (L.icell) and
// the scatter bound (L.ibound, with 1/8 headroom).  Both stay bounds of the
// scattered state because a particle goes into the tile only if it kept its
// base cell (so no cell gains particles) and its bound stays within the
// scale; any other particle is scattered straight into the grid.  The item's
// L.ibound and L.icell are then replaced by those of the advanced state.
template <int B, bool PF, bool PEN, int NT = WG, bool FUSE = false>
__device__ void g2p_item(const StepArgs &a, int it, const Item &item, float *vt, float *pf, int *cells,
                         long long *t64 = nullptr)
{
    constexpr int T = tile_edge<B>(), T3 = T * T * T, NC = p2g_cells<B>();
    const int t = threadIdx.x;
    const int s = item.scene;
    const SceneDev &S = a.scenes[s];
    const int nb = S.nb;
    const int bx = item.block / (nb * nb), by = (item.block / nb) % nb, bz = item.block % nb;
    const int org[3] = {bx * B - 1, by * B - 1, bz * B - 1};
    const int3 home = make_int3(bx, by, bz);
    const long long ps = a.pstride;
    const int lane = t & 63;
    float *pw = PF ? pf + uniform_i(t >> 6) * (PF_COMPS * 64) : nullptr;
    // scene constants in registers before any copy into LDS (the copies may alias memory for
    // the compiler, which would reload them after each one)
    const Material mat = material_of(S);
    const SceneK K = scene_k(S);
    const SceneDev Sn = {0, 0, K.res, uniform_i(S.nb), uniform_ll(S.grid_off)};   // for node_index
    TileScale ts{};
    if (FUSE) {
        const int known = item.count > P2G_COUNT_MIN ? a.L.icell[it] : 0;
        float wsum = 0.421875f * (float)item.count;
        if (known > 0) wsum = fminf(wsum, 5.359375f * (float)known);
        // floor: 2^-20 of the momentum of a particle crossing a cell per substep (a state at rest
        // has bound 0)
        const float floor_b = 9.5367431640625e-7f * K.mass * K.dx / K.dt;
        ts = tile_scale(K, wsum, fmaxf(1.125f * a.L.ibound[it], floor_b));
        for (int n = t; n < 2 * T3; n += NT) t64[n] = 0;
    }
    for (int n = t; n < NC + 1; n += NT) cells[n] = 0;
    {
        const int res = Sn.res;
        // the wave's first 64 particles: x and G copied into LDS while the tile is staged
        if (PF) pf_issue(a.P, ps, item.start + (t - lane), item.count - (t - lane), lane, pw);
        // tile nodes copied straight into LDS, all in flight at once; nodes outside the grid are zeroed
        for (int n0 = t - lane; n0 < T3; n0 += NT) {
            const int n = n0 + lane;
            if (n >= T3) break;
            int gi = org[0] + n / (T * T), gj = org[1] + (n / T) % T, gk = org[2] + n % T;
            if (gi >= 0 && gj >= 0 && gk >= 0 && gi < res && gj < res && gk < res) {
                long long idx = node_index(Sn, B, gi, gj, gk);
                lds_copy(a.gvx + idx, vt + n0);
                lds_copy(a.gvy + idx, vt + T3 + n0);
                lds_copy(a.gvz + idx, vt + 2 * T3 + n0);
            } else {
                vt[n] = 0.0f;
                vt[T3 + n] = 0.0f;
                vt[2 * T3 + n] = 0.0f;
            }
        }
        wait_vmem();
    }
    __syncthreads();
    if (FUSE && t == 0) a.L.ibound[it] = 0.0f;   // read by every thread above; the advanced state's bound follows
    int bad_any = 0, cl_any = 0;
    float bnd = 0.0f;
    // penalty contact: this substep's collider poses of the scene (uniform), the per-lane sums of
    // the momentum and its moment given to the particles, and which colliders were touched
    const ColliderNow *cn = (const ColliderNow *)a.colnow + S.col_off;
    const int pen_ncol = PEN ? uniform_i(S.n_col) : 0;
    const float pen_rate = 0.25f / K.dt;
    float pacc[PEN ? MAX_COLLIDERS_PER_SCENE : 1][6] = {};
    unsigned pen_hit = 0;
    // wave-uniform loop: lane li = k0 + lane of each 64-particle batch
    for (int k0 = t - lane; k0 < item.count; k0 += NT) {
        const int li = k0 + lane;
        const unsigned jo = (unsigned)(item.start + li) << 2;
        float x[3], G[9];
        if (PF) {
#pragma unroll
            for (int d = 0; d < 3; d++) x[d] = pw[d * 64 + lane];
#pragma unroll
            for (int e = 0; e < 9; e++) G[e] = pw[(3 + e) * 64 + lane];
            wait_lds();
            // the next batch streams into LDS while this one computes
            pf_issue(a.P, ps, item.start + k0 + NT, item.count - (k0 + NT), lane, pw);
        }
        if (li >= item.count) {
            if (PF) wait_vmem();
            continue;
        }
        if (!PF) {
#pragma unroll
            for (int d = 0; d < 3; d++) x[d] = pload(a.P, ps, X0 + d, jo);
#pragma unroll
            for (int e = 0; e < 9; e++) G[e] = pload(a.P, ps, G00 + e, jo);
        }
        int b[3], cl = 0, in = 1;
        float f[3];
#pragma unroll
        for (int d = 0; d < 3; d++) {
            particle_base(K, x[d], b[d], f[d], cl);
            int tb = b[d] - org[d];
            in &= (tb >= 0) & (tb <= tile_bmax<B>());
        }
        cl_any |= cl;
        float wx[3], wy[3], wz[3];
        bspline_w(f[0], wx);
        bspline_w(f[1], wy);
        bspline_w(f[2], wz);
        float vp[3] = {0.0f, 0.0f, 0.0f};
        float So[3][3] = {{0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}};   // sum w v_c o_e
        if (in) {
            // separable gather: reduce over z, then y, then x
            const float *vb = vt + ((b[0] - org[0]) * T + (b[1] - org[1])) * T + (b[2] - org[2]);
            const float wz2 = 2.0f * wz[2], wy2 = 2.0f * wy[2], wx2 = 2.0f * wx[2];
#pragma unroll
            for (int ox = 0; ox < 3; ox++) {
                float A[3] = {0.0f, 0.0f, 0.0f}, By[3] = {0.0f, 0.0f, 0.0f}, Bz[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int oy = 0; oy < 3; oy++) {
                    const int o = (ox * T + oy) * T;
#pragma unroll
                    for (int c = 0; c < 3; c++) {
                        const float v0 = vb[c * T3 + o], v1 = vb[c * T3 + o + 1], v2 = vb[c * T3 + o + 2];
                        const float az = fmaf(wz[0], v0, fmaf(wz[1], v1, wz[2] * v2));
                        const float bzv = fmaf(wz[1], v1, wz2 * v2);
                        A[c] = fmaf(wy[oy], az, A[c]);
                        if (oy == 1) By[c] = fmaf(wy[1], az, By[c]);
                        if (oy == 2) By[c] = fmaf(wy2, az, By[c]);
                        Bz[c] = fmaf(wy[oy], bzv, Bz[c]);
                    }
                }
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    vp[c] = fmaf(wx[ox], A[c], vp[c]);
                    if (ox == 1) So[c][0] = fmaf(wx[1], A[c], So[c][0]);
                    if (ox == 2) So[c][0] = fmaf(wx2, A[c], So[c][0]);
                    So[c][1] = fmaf(wx[ox], By[c], So[c][1]);
                    So[c][2] = fmaf(wx[ox], Bz[c], So[c][2]);
                }
            }
        } else {
            // outside the tile (drifted since the re-sort): the nodes straight from the grid, nine
            // at a time in flight, with the scene constants in registers (the particle stores may
            // alias the scene record for the compiler, which would reload it and wait for them)
            for (int ox = 0; ox < 3; ox++) {
                float g[9][3];
#pragma unroll
                for (int q = 0; q < 9; q++) {
                    const long long idx = node_index(Sn, B, b[0] + ox, b[1] + q / 3, b[2] + q % 3);
                    g[q][0] = a.gvx[idx];
                    g[q][1] = a.gvy[idx];
                    g[q][2] = a.gvz[idx];
                }
#pragma unroll
                for (int q = 0; q < 9; q++) {
                    const int oy = q / 3, oz = q % 3;
                    const float w = wx[ox] * wy[oy] * wz[oz];
#pragma unroll
                    for (int c = 0; c < 3; c++) {
                        const float tv = w * g[q][c];
                        vp[c] += tv;
                        So[c][0] += (float)ox * tv;
                        So[c][1] += (float)oy * tv;
                        So[c][2] += (float)oz * tv;
                    }
                }
            }
        }
        // C = (4/dx^2) sum w v (x_i - x_p)^T = (4/dx) (So - vp f^T)
        const float Dd = 4.0f * K.inv_dx;
        float C[9];
#pragma unroll
        for (int c = 0; c < 3; c++)
#pragma unroll
            for (int e = 0; e < 3; e++) C[3 * c + e] = Dd * fmaf(-vp[c], f[e], So[c][e]);
#pragma unroll
        for (int d = 0; d < 3; d++) x[d] = fmaf(K.dt, vp[d], x[d]);
        // base cell of the new position in this item's P2G tile
        int bn[3], tbn[3], inn = 1, cln = 0;
        float fn[3];
        {
            int c = 0;
#pragma unroll
            for (int d = 0; d < 3; d++) {
                particle_base(K, x[d], bn[d], fn[d], cln);
                tbn[d] = bn[d] - org[d];
                inn &= (tbn[d] >= 0) & (tbn[d] <= tile_bmax<B>());
                c = c * (tile_bmax<B>() + 1) + tbn[d];
            }
            if (inn && !cln) atomicAdd(cells + c, 1);
        }
        if (PEN) {
            // inside collider c at the new position: v += -phi n / (4 dt), a spring of stiffness
            // m / (4 dt^2) along the outward normal (the stored v, hence the next scatter bound,
            // includes it)
#pragma unroll
            for (int c = 0; c < (PEN ? MAX_COLLIDERS_PER_SCENE : 1); c++) {
                if (c >= pen_ncol) break;
                float nrm[3];
                const float phi = sdf_eval(cn[c], x, nrm, a.sdf);
                if (phi < 0.0f) {
                    float dp[3], r[3];
#pragma unroll
                    for (int d = 0; d < 3; d++) {
                        const float dv = -phi * pen_rate * nrm[d];
                        vp[d] += dv;
                        dp[d] = K.mass * dv;
                        r[d] = x[d] - cn[c].c[d];
                    }
                    pacc[c][0] += dp[0];
                    pacc[c][1] += dp[1];
                    pacc[c][2] += dp[2];
                    pacc[c][3] += r[1] * dp[2] - r[2] * dp[1];
                    pacc[c][4] += r[2] * dp[0] - r[0] * dp[2];
                    pacc[c][5] += r[0] * dp[1] - r[1] * dp[0];
                    pen_hit |= 1u << c;
                }
            }
        }
        // F <- (I + dt C) F  ->  G <- G + dt C + dt C G
        float Gt[9];
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int k = 0; k < 3; k++) {
                float acc = C[3 * i + k];
#pragma unroll
                for (int e = 0; e < 3; e++) acc = fmaf(C[3 * i + e], G[3 * e + k], acc);
                Gt[3 * i + k] = fmaf(K.dt, acc, G[3 * i + k]);
            }
        float tau[9], Gn[9];
        int bad = 0;
        if (mat.model == 0) {
            tau_neo_hookean(Gt, mat.mu, mat.la, tau, bad);
#pragma unroll
            for (int e = 0; e < 9; e++) Gn[e] = Gt[e];
        } else if (mat.model == 2) {
            fluid_update(Gt, mat, Gn, tau, bad);
        } else {
            hencky_update(Gt, mat, Gn, tau, bad);
        }
        bad |= !(isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]));
        bad_any |= bad;
        // the prefetch has had the whole computation to land; waiting here (not at
        // the top of the next batch) keeps the wait off this batch's stores
        if (PF) wait_vmem();
#pragma unroll
        for (int d = 0; d < 3; d++) {
            pstore(a.P, ps, X0 + d, jo, x[d]);
            if (!FUSE) pstore(a.P, ps, V0 + d, jo, vp[d]);
        }
        float An[9];
#pragma unroll
        for (int e = 0; e < 9; e++) {
            An[e] = fmaf(K.mass, C[e], -K.kstress * tau[e]);
            if (!FUSE) pstore(a.P, ps, A00 + e, jo, An[e]);
            pstore(a.P, ps, G00 + e, jo, Gn[e]);
        }
        // a non-finite v or A (the next P2G would scatter it as garbage)
        const float sb = scatter_bound(K.mass, K.dx, vp, An);
        bad_any |= !(sb <= 3.0e38f);
        bnd = fmaxf(bnd, sb);
        if (FUSE) {
            const bool kept = bn[0] == b[0] && bn[1] == b[1] && bn[2] == b[2];
            if (inn && !cln && kept && sb * ts.sp <= ts.lim) scatter_packed<B>(t64, tbn, fn, ts, K, vp, An);
            else p2g_global<B>(a, s, S, x, vp, An, bn, fn, ovf_count(a, a.substep + 1), home);
        }
    }
    bnd = wave_max(bnd);
    if ((t & 63) == 0 && bnd > 0.0f) atomicMax((int *)(a.L.ibound + it), __float_as_int(bnd));
    if (PEN && a.wrench) {
        // the colliders receive minus what the penalty gave the particles: one wave sum and
        // one atomic per component, for the colliders a lane of the wave touched
#pragma unroll
        for (int c = 0; c < (PEN ? MAX_COLLIDERS_PER_SCENE : 1); c++) {
            if (c >= pen_ncol) break;
            if (!__any((pen_hit >> c) & 1u)) continue;
            float tot[6];
#pragma unroll
            for (int j = 0; j < 6; j++) tot[j] = wave_total(pacc[c][j]);
            if ((t & 63) == 0)
#pragma unroll
                for (int j = 0; j < 6; j++) atomicAdd(a.wrench + 6 * (long long)(S.col_off + c) + j, -tot[j]);
        }
    }
    if (bad_any) atomicOr(a.flags + s, (int)FLAG_NONFINITE);
    if (cl_any) atomicOr(a.flags + s, (int)FLAG_CLAMPED);
    __syncthreads();
    if (FUSE) flush_packed<B, NT>(a, s, S, org, t64, ts, ovf_count(a, a.substep + 1));
    int mx = 0;
    for (int n = t; n < NC; n += NT) mx = max(mx, cells[n]);
    mx = wave_max_i(mx);
    if ((t & 63) == 0) atomicMax(cells + NC, mx);
    __syncthreads();
    if (t == 0) a.L.icell[it] = cells[NC];
}

template <int B, bool PEN, int NT>
__global__ __launch_bounds__(NT, 4) void k_g2p(StepArgs a)
{
    constexpr int T = tile_edge<B>(), T3 = T * T * T;
    __shared__ float vt[3 * T3];
    __shared__ float pf[(NT / 64) * PF_COMPS * 64];
    __shared__ int cells[p2g_cells<B>() + 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicExch(ovf_count(a, a.substep), 0);   // consumed by the grid update
    const int n_items = *a.L.n_items;
    const int G = active_wgs(n_items);
    if ((int)blockIdx.x >= G) return;
    for (int r = blockIdx.x; r < n_items; r += G) {   // most particles first (L.order)
        const int it = a.L.order[r];
        Item item = a.L.items[it];
        if (!a.active[item.scene]) continue;
        g2p_item<B, true, PEN, NT>(a, it, item, vt, pf, cells);
    }
}

// G2P of substep a.substep fused with the P2G of substep a.substep + 1 (one
// pass over the particles; the grid update sits between two such launches).
// LDS: the velocity tile, the fixed-point tile and the base-cell counts (40 KB
// at block edge 8: four workgroups of 256 threads per CU).  x and G go straight
// into registers: the LDS prefetch slices of k_g2p would cost a workgroup per
// CU (measured 2.5 % slower on the 256-scene workload, 1.6 % on the heap).
// With penalty contact the kernel needs more registers than four workgroups
// leave, and keeps the prefetch.
template <int B, bool PEN, int NT>
__global__ __launch_bounds__(NT, 4) void k_g2p2g(StepArgs a)
{
    constexpr int T = tile_edge<B>(), T3 = T * T * T;
    __shared__ float vt[3 * T3];
    __shared__ float pf[PEN ? (NT / 64) * PF_COMPS * 64 : 1];
    __shared__ __align__(16) long long t64[2 * T3];
    __shared__ int cells[p2g_cells<B>() + 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicExch(ovf_count(a, a.substep), 0);   // consumed by the grid update
    const int n_items = *a.L.n_items;
    const int G = active_wgs(n_items);
    if ((int)blockIdx.x >= G) return;
    for (int r = blockIdx.x; r < n_items; r += G) {   // most particles first (L.order)
        const int it = a.L.order[r];
        Item item = a.L.items[it];
        if (!a.active[item.scene]) continue;
        g2p_item<B, PEN, PEN, NT, true>(a, it, item, vt, pf, cells, t64);
    }
}

template <int NT>
static void launch_g2p2g_nt(const StepArgs &a, int n_wg, hipStream_t st)
{
    const bool pen = a.contact != 0;
    if (a.B == 4) {
        if (pen) launch_timed(k_g2p2g<4, true, NT>, n_wg, NT, st, a);
        else launch_timed(k_g2p2g<4, false, NT>, n_wg, NT, st, a);
    } else {
        if (pen) launch_timed(k_g2p2g<8, true, NT>, n_wg, NT, st, a);
        else launch_timed(k_g2p2g<8, false, NT>, n_wg, NT, st, a);
    }
}

hipError_t launch_g2p2g(const StepArgs &a, int n_wg, hipStream_t st)
{
    if (a.nt == 512) n_wg /= 2;
    n_wg = (n_wg + 7) & ~7;
    if (a.nt == 512) launch_g2p2g_nt<512>(a, n_wg, st);
    else launch_g2p2g_nt<WG>(a, n_wg, st);
    return hipGetLastError();
}

hipError_t launch_p2g(const StepArgs &a, int chunk, int n_wg, hipStream_t st)
{
    (void)chunk;
    if (a.nt == 512) n_wg /= 2;   // the same threads in workgroups of twice the size
    n_wg = (n_wg + 7) & ~7;
    if (a.nt == 512) {
        if (a.B == 4) launch_timed(k_p2g<4, 512>, n_wg, 512, st, a);
        else launch_timed(k_p2g<8, 512>, n_wg, 512, st, a);
    } else {
        if (a.B == 4) launch_timed(k_p2g<4, WG>, n_wg, WG, st, a);
        else launch_timed(k_p2g<8, WG>, n_wg, WG, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_grid(const StepArgs &a, int n_wg, hipStream_t st)
{
    n_wg = (n_wg + 7) & ~7;
    const bool extra = a.cap || a.dense;
    if (a.B == 4) {
        if (extra) launch_timed(k_grid<4, true>, n_wg, WG, st, a);
        else launch_timed(k_grid<4, false>, n_wg, WG, st, a);
    } else {
        if (extra) launch_timed(k_grid<8, true>, n_wg, WG, st, a);
        else launch_timed(k_grid<8, false>, n_wg, WG, st, a);
    }
    return hipGetLastError();
}

template <int NT>
static void launch_g2p_nt(const StepArgs &a, int n_wg, hipStream_t st)
{
    const bool pen = a.contact != 0;
    if (a.B == 4) {
        if (pen) launch_timed(k_g2p<4, true, NT>, n_wg, NT, st, a);
        else launch_timed(k_g2p<4, false, NT>, n_wg, NT, st, a);
    } else {
        if (pen) launch_timed(k_g2p<8, true, NT>, n_wg, NT, st, a);
        else launch_timed(k_g2p<8, false, NT>, n_wg, NT, st, a);
    }
}

hipError_t launch_g2p(const StepArgs &a, int n_wg, hipStream_t st)
{
    if (a.nt == 512) n_wg /= 2;   // the same threads in workgroups of twice the size
    n_wg = (n_wg + 7) & ~7;
    if (a.nt == 512) launch_g2p_nt<512>(a, n_wg, st);
    else launch_g2p_nt<WG>(a, n_wg, st);
    return hipGetLastError();
}

// ---------------------------------------------------------------- one-launch substep
// One cooperative launch per substep over all scenes: every workgroup is
// resident at once (the launch is sized from the kernel's occupancy and the
// runtime refuses a larger one), and the three phases of the substep are
// separated by grid-wide barriers: P2G over all work items, the grid update
// over every listed block (one wave per block), G2P over all work items.
// Within a phase the workgroups stride over the work as the separate kernels
// do.  The phases share one LDS allocation (the P2G tile, or the G2P
// velocity tile and prefetch slices).
template <int B, bool PEN>
__global__ __launch_bounds__(WG, 4) void k_substep_coop(StepArgs a)
{
    constexpr int T = tile_edge<B>(), T3 = T * T * T;
    constexpr int P2G_WORDS = 4 * T3;
    constexpr int G2P_WORDS = 3 * T3 + (WG / 64) * PF_COMPS * 64;
    __shared__ __align__(16) int smem[P2G_WORDS > G2P_WORDS ? P2G_WORDS : G2P_WORDS];
    __shared__ int cells[p2g_cells<B>() + 1];
    __shared__ ColliderNow cls[WG / 64][MAX_COLLIDERS_PER_SCENE];
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    const int G = gridDim.x;   // a multiple of 8: every workgroup takes part in every phase
    const int n_items = *a.L.n_items;
    // P2G, items in reverse order: the G2P of the previous substep walked them forward, so the
    // particles it wrote last are still in the memory-side cache
    for (int r = xcd_remap(blockIdx.x, G); r < n_items; r += G) {
        const int it = n_items - 1 - r;
        const Item item = a.L.items[it];
        if (!a.active[item.scene]) continue;
        p2g_item<B, WG>(a, it, item, smem, cells);
    }
    grid.sync();
    {
        const int lane = threadIdx.x & 63;
        const int ng = *a.L.n_gitems;
        const int no = min(*ovf_count(a, a.substep), a.L.ovf_cap);
        const int nw = G * (WG / 64);
        const int w0 = xcd_remap(blockIdx.x, G) * (WG / 64) + (threadIdx.x >> 6);
        for (int w = w0; w < ng + no; w += nw) {
            const int2 e = w < ng ? a.L.gitems[w] : a.L.ovf[w - ng];
            if (w < ng) publish_colliders(a, w, e.x, lane);
            grid_block<B, false>(a, e.x, e.y, lane, cls[threadIdx.x >> 6]);
            if (w >= ng && lane == 0) a.L.bflag[a.scenes[e.x].bin_off + e.y] = 0;
        }
    }
    grid.sync();
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicExch(ovf_count(a, a.substep), 0);   // consumed by the grid update
    float *vt = (float *)smem;
    for (int it = xcd_remap(blockIdx.x, G); it < n_items; it += G) {
        const Item item = a.L.items[it];
        if (!a.active[item.scene]) continue;
        g2p_item<B, true, PEN, WG>(a, it, item, vt, vt + 3 * T3, cells);
    }
}

// Workgroups of the cooperative substep (a multiple of 8): at most what can
// be resident at once (the kernel's occupancy), and no more per CU than
// per_cu_cap.  Each grid-wide barrier costs about 0.1 us per workgroup on
// MI355X (cfg2, one 65,536-particle scene: 94 / 146 / 260 us per substep
// at 1 / 2 / 4 workgroups per CU), so small problems take fewer; 0 on error.
template <int B, bool PEN>
static int coop_workgroups(int cus, int per_cu_cap)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_substep_coop<B, PEN>, WG, 0) != hipSuccess) return 0;
    per_cu = min(per_cu, max(per_cu_cap, 1));
    return (per_cu * cus) & ~7;
}

hipError_t launch_persistent(const StepArgs &a, int cus, int per_cu_cap, hipStream_t st)
{
    const bool pen = a.contact != 0;
    const void *fn;
    int G;
    if (a.B == 4) {
        fn = pen ? (const void *)k_substep_coop<4, true> : (const void *)k_substep_coop<4, false>;
        G = pen ? coop_workgroups<4, true>(cus, per_cu_cap) : coop_workgroups<4, false>(cus, per_cu_cap);
    } else {
        fn = pen ? (const void *)k_substep_coop<8, true> : (const void *)k_substep_coop<8, false>;
        G = pen ? coop_workgroups<8, true>(cus, per_cu_cap) : coop_workgroups<8, false>(cus, per_cu_cap);
    }
    if (G <= 0) return hipErrorInvalidConfiguration;
    StepArgs args = a;
    void *params[] = {(void *)&args};
    return hipLaunchCooperativeKernel(fn, dim3(G), dim3(WG), params, 0, st);
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
size_t collider_now_bytes() { return sizeof(ColliderNow); }

__global__ void k_wrench_out(const SceneDev *scenes, int n_scenes, int max_col, float *acc, float *out)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;   // (scene, slot, component)
    if (e >= n_scenes * max_col * 6) return;
    const int s = e / (max_col * 6), k = (e / 6) % max_col, j = e % 6;
    const SceneDev &S = scenes[s];
    float val = 0.0f;
    if (k < S.n_col) {
        float *p = acc + 6 * (long long)(S.col_off + k) + j;
        val = *p;
        *p = 0.0f;
    }
    out[e] = val;
}

hipError_t launch_wrench_out(const SceneDev *scenes, int n_scenes, int max_col, float *acc, float *out, hipStream_t st)
{
    const int n = n_scenes * max_col * 6;
    if (n > 0) k_wrench_out<<<(n + 255) / 256, 256, 0, st>>>(scenes, n_scenes, max_col, acc, out);
    return hipGetLastError();
}

// A non-finite x, v, C or F (or an F whose stress is not defined) sets the
// scene's FLAG_NONFINITE: inside a substep the fixed-point P2G would turn it
// into finite garbage rather than propagate it.
__global__ __launch_bounds__(WG) void k_init_particles(const SceneDev *scenes, const int *psc, float *P,
                                                       long long ps, const float *x, const float *v, const float *C,
                                                       const float *F, int begin, int end, int *flags)
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
    float chk = 0.0f;   // NaN or infinity in any input makes it fail the test below
    for (int d = 0; d < 3; d++) {
        const float xv = x[3 * (long long)k + d], vv = v ? v[3 * (long long)k + d] : 0.0f;
        chk += fabsf(xv) + fabsf(vv);
        P[(X0 + d) * ps + i] = xv;
        P[(V0 + d) * ps + i] = vv;
    }
    for (int e = 0; e < 9; e++) chk += fabsf(G[e]) + fabsf(Cm[e]) + fabsf(tau[e]);
    if (bad || !(chk <= 3.0e38f)) atomicOr(flags + psc[i], (int)FLAG_NONFINITE);
    for (int e = 0; e < 9; e++) {
        P[(A00 + e) * ps + i] = fmaf(S.mass, Cm[e], -S.kstress * tau[e]);
        P[(G00 + e) * ps + i] = G[e];
    }
    P[PID * ps + i] = __int_as_float(i);
}

hipError_t launch_init_particles(const SceneDev *scenes, int n_scenes, const int *psc, float *P, long long pstride,
                                 const float *x, const float *v, const float *C, const float *F, int begin, int end,
                                 int *flags, hipStream_t st)
{
    (void)n_scenes;
    if (end > begin)
        k_init_particles<<<(end - begin + WG - 1) / WG, WG, 0, st>>>(scenes, psc, P, pstride, x, v, C, F, begin, end, flags);
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

__global__ void k_fill_i(int *p, long long n, int v)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_i(int *p, long long n, int v, hipStream_t st)
{
    if (n > 0) {
        long long nb = (n + WG - 1) / WG;
        k_fill_i<<<(unsigned)(nb < 4096 ? nb : 4096), WG, 0, st>>>(p, n, v);
    }
    return hipGetLastError();
}

}  // namespace mpm
