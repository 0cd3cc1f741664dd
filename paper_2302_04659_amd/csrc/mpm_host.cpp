// Host runtime and C ABI of the MI355X MLS-MPM library.
//
// The context owns every device buffer: particle state (two struct-of-arrays
// buffers that the counting sort ping-pongs between), one dense grid per
// scene in block-linear order, the sort / work-list arrays, collider tables
// and a small pinned staging ring for collider uploads.  mpm_step queues
// substeps (sort when due, P2G, grid update, G2P) on the context stream and
// returns; only mpm_sync and host-side reads wait.
#include <hip/hip_runtime.h>

#include <sys/stat.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/mpm.h"
#include "../../include/mpm_nn.h"
#include "mpm_kernels.hpp"
#include "mpm_types.hpp"
#include "sur_net.hpp"

static_assert(MPM_MAX_COLLIDERS == mpm::MAX_COLLIDERS_PER_SCENE, "grid kernel LDS collider slots");

using namespace mpm;

namespace {

constexpr int STAGE_RING = 4;

struct GraphKey {
    int parity, since_sort, sort_every;
    bool operator<(const GraphKey &o) const
    {
        if (parity != o.parity) return parity < o.parity;
        if (since_sort != o.since_sort) return since_sort < o.since_sort;
        return sort_every < o.sort_every;
    }
};

// A captured 25-substep control step and the context state it leaves.
struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    int end_parity = 0, end_since_sort = 0;
    long long n_sorts = 0;   // re-sorts the captured control step contains
};

constexpr int GRAPH_BLOCK = 25;

}  // namespace

struct mpm_ctx_s {
    int dev = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int cus = 256;

    int n_scenes = 0;
    int N = 0;
    long long pstride = 0;
    std::vector<SceneDev> h_scenes;
    std::vector<mpm_scene_desc> descs;
    std::vector<ColliderDev> h_cols;
    std::vector<int> h_col_scene;
    std::vector<float> h_sdf;        // samples of every SDF-volume collider, concatenated
    float *d_sdf = nullptr;
    int max_col = 0;

    SceneDev *d_scenes = nullptr;
    int *d_psc = nullptr;
    float *d_P[2] = {nullptr, nullptr};
    int cur = 0;

    long long n_nodes = 0;
    float *d_grid = nullptr;   // 7 arrays of n_nodes: m, px, py, pz, vx, vy, vz
    ColliderDev *d_cols = nullptr;
    void *d_colnow = nullptr;
    int *d_col_scene = nullptr;

    // sort and work lists
    int B = 4, CH = 2048, sort_every = 25, since_sort = 1 << 30;
    int nt = 256;                    // threads per workgroup of P2G and G2P (MPM_OPT_WG)
    int T = 0, T_cap = 0;
    int *d_scene_bin_off = nullptr;
    unsigned *d_keys = nullptr;
    int *d_count = nullptr, *d_pstart = nullptr, *d_perm = nullptr;
    int3 *d_tsum = nullptr;
    unsigned char *d_dil = nullptr;
    Lists L{};
    int items_cap = 0;
    int *d_flags = nullptr;

    // per-scene step mask (1 = step), dense per-scene grid offsets
    int *d_active = nullptr;
    // grid surrogate: re-splat grid and residual sums
    float *d_sur_gend = nullptr, *d_sur_acc = nullptr, *d_sur_out = nullptr;
    int *d_sur_nfb = nullptr;
    float *d_wrench = nullptr;       // per collider: [6] impulse and angular impulse received, summed
    float *d_wrench_out = nullptr;   // [n_scenes][max_col][6] staging for mpm_get_collider_wrenches

    // library-owned surrogate (mpm_surrogate_load / mpm_step_blocks): network and per-block arrays
    mpm::SurNet *net = nullptr;
    int *d_sb_box = nullptr, *d_sb_origin = nullptr;
    float *d_sb_feat = nullptr, *d_sb_grid0 = nullptr, *d_sb_pred = nullptr, *d_sb_res = nullptr;
    long long sb_nodes = 0;          // box nodes the per-block arrays hold
    std::vector<int> h_sb_box;
    std::vector<float> h_sb_res;     // residuals of the last surrogate block

    // debug capture of the P2G grid
    int capture = 0;
    float *d_cap = nullptr;
    long long *d_cap_off = nullptr;
    long long cap_nodes = 0;

    int persistent = 0, graph = 0;
    int fuse = 1;                    // MPM_OPT_FUSE: G2P and the next P2G in one launch
    int contact = 0;                 // MPM_OPT_CONTACT
    std::map<GraphKey, GraphEntry> graphs;

    // per-kernel-class timing with HIP events on the context stream
    int timing = 0;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
    double kt_ms[MPM_KCLASSES] = {};
    long long kt_n[MPM_KCLASSES] = {};
    // work queued since the last reset (mpm_get_counters)
    long long cnt[MPM_NCOUNTERS] = {};

    // io
    float *d_io = nullptr;
    float *h_stage[STAGE_RING] = {};
    hipEvent_t stage_ev[STAGE_RING] = {};
    int stage_next = 0;

    std::string last_error;
};

namespace {

#define HIPCHK(expr)                                                                    \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            ctx->last_error = std::string(#expr) + ": " + hipGetErrorString(e_);        \
            return e_ == hipErrorOutOfMemory ? MPM_ERR_OOM : MPM_ERR_HIP;               \
        }                                                                               \
    } while (0)

#define ARGCHK(cond, msg)                   \
    do {                                    \
        if (!(cond)) {                      \
            if (ctx) ctx->last_error = msg; \
            return MPM_ERR_ARG;             \
        }                                   \
    } while (0)

template <typename T>
hipError_t dalloc(T **p, size_t n)
{
    return hipMalloc((void **)p, std::max<size_t>(n, 1) * sizeof(T));
}

bool valid_res(int r) { return r == 16 || r == 32 || r == 64 || r == 128 || r == 256; }

mpm_status validate_desc(mpm_ctx ctx, const mpm_scene_desc &d, int i)
{
    char buf[160];
    auto bad = [&](const char *what) {
        std::snprintf(buf, sizeof buf, "scene %d: %s", i, what);
        if (ctx) ctx->last_error = buf;
        return MPM_ERR_ARG;
    };
    if (d.n_particles < 0) return bad("n_particles < 0");
    if (d.n_particles > 0 && !d.x) return bad("x is NULL");
    if (!valid_res(d.res)) return bad("res must be 16, 32, 64, 128 or 256");
    if (!(d.dx > 0) || !std::isfinite(d.dx)) return bad("dx must be > 0");
    if (!(d.dt > 0) || !std::isfinite(d.dt)) return bad("dt must be > 0");
    if (d.bound < 0 || 2 * d.bound >= d.res) return bad("bound out of range");
    if (!(d.particle_volume > 0)) return bad("particle_volume must be > 0");
    if (d.mat.model < 0 || d.mat.model > 2) return bad("unknown material model");
    if (!(d.mat.E > 0) || !(d.mat.nu > -1.0f && d.mat.nu < 0.5f) || !(d.mat.rho > 0)) return bad("bad material");
    if (d.mat.yield_form != 0 && d.mat.yield_form != 1) return bad("yield_form must be 0 or 1");
    if (d.n_colliders < 0 || d.n_colliders > MPM_MAX_COLLIDERS) return bad("n_colliders out of range");
    if (d.n_colliders > 0 && !d.colliders) return bad("colliders is NULL");
    for (int k = 0; k < d.n_colliders; k++) {
        const mpm_collider_shape &c = d.colliders[k];
        if (c.type < 0 || c.type > 2) return bad("unknown collider type");
        if (c.type == 2) {
            if (!c.sdf) return bad("SDF volume: sdf is NULL");
            long long n = 1;
            for (int a = 0; a < 3; a++) {
                if (c.sdf_dims[a] < 2) return bad("SDF volume: every dimension must be >= 2");
                if (!std::isfinite(c.sdf_origin[a])) return bad("SDF volume: origin not finite");
                n *= c.sdf_dims[a];
            }
            if (!(c.sdf_cell > 0) || !std::isfinite(c.sdf_cell)) return bad("SDF volume: cell must be > 0");
            if (n > (1LL << 28)) return bad("SDF volume: too many samples");
            for (long long i = 0; i < n; i++)
                if (!std::isfinite(c.sdf[i])) return bad("SDF volume: non-finite sample");
        }
        if (!(c.friction >= 0)) return bad("collider friction must be >= 0");
        if (c.type == 0 && !(c.half_extents[0] >= 0 && c.half_extents[1] >= 0 && c.half_extents[2] >= 0))
            return bad("box half extents must be >= 0");
        if (c.type == 1 && !(c.radius >= 0 && c.half_length >= 0)) return bad("capsule radius / half length must be >= 0");
    }
    for (int g = 0; g < 3; g++)
        if (!std::isfinite(d.gravity[g])) return bad("gravity not finite");
    for (long long k = 0; k < 3LL * d.n_particles; k++) {
        if (!std::isfinite(d.x[k])) return bad("x not finite");
        if (d.v && !std::isfinite(d.v[k])) return bad("v not finite");
    }
    return MPM_OK;
}

SceneDev make_scene(const mpm_scene_desc &d, int p_begin, int col_off, int B)
{
    SceneDev S{};
    S.p_begin = p_begin;
    S.p_end = p_begin + d.n_particles;
    S.res = d.res;
    S.nb = d.res / B;
    S.col_off = col_off;
    S.n_col = d.n_colliders;
    S.bound = d.bound;
    S.model = d.mat.model;
    double E = d.mat.E, nu = d.mat.nu;
    double mu = E / (2 * (1 + nu)), la = E * nu / ((1 + nu) * (1 - 2 * nu));
    S.plastic = d.mat.model == 1 && d.mat.yield_stress > 0 && std::isfinite(d.mat.yield_stress);
    double ye = S.plastic ? d.mat.yield_stress / (2 * mu) : INFINITY;
    if (d.mat.yield_form == 1) ye *= std::sqrt(2.0 / 3.0);
    S.dx = d.dx;
    S.inv_dx = (float)(1.0 / d.dx);
    S.dt = d.dt;
    for (int a = 0; a < 3; a++) S.g[a] = d.gravity[a];
    S.mu = (float)mu;
    S.la = (float)la;
    S.yield_eps = (float)ye;
    S.vol = d.particle_volume;
    S.mass = (float)((double)d.mat.rho * d.particle_volume);
    S.kstress = (float)((double)d.dt * d.particle_volume * 4.0 / ((double)d.dx * d.dx));
    S.D = (float)(4.0 / ((double)d.dx * d.dx));
    return S;
}

void clear_graphs(mpm_ctx ctx)
{
    for (auto &g : ctx->graphs) (void)hipGraphExecDestroy(g.second.exec);
    ctx->graphs.clear();
}

mpm_status set_block(mpm_ctx ctx, int B)
{
    // (Re)build the per-scene grid offsets and bin tables for block edge B.
    ctx->B = B;
    long long goff = 0;
    int boff = 0;
    std::vector<int> bin_off(ctx->n_scenes + 1);
    for (int s = 0; s < ctx->n_scenes; s++) {
        SceneDev &S = ctx->h_scenes[s];
        S.nb = S.res / B;
        S.grid_off = goff;
        S.bin_off = boff;
        bin_off[s] = boff;
        goff += (long long)S.res * S.res * S.res;
        boff += S.nb * S.nb * S.nb;
    }
    bin_off[ctx->n_scenes] = boff;
    ctx->T = boff;
    if (boff > ctx->T_cap) {
        ctx->last_error = "bin table larger than allocated";
        return MPM_ERR_STATE;
    }
    HIPCHK(hipMemcpyAsync(ctx->d_scenes, ctx->h_scenes.data(), sizeof(SceneDev) * ctx->n_scenes,
                          hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->d_scene_bin_off, bin_off.data(), sizeof(int) * (ctx->n_scenes + 1),
                          hipMemcpyHostToDevice, ctx->stream));
    // the grid layout changed: every (m, p) must be zero and every v finite
    HIPCHK(launch_clear_f(ctx->d_grid, 7 * ctx->n_nodes, ctx->stream));
    if (ctx->L.touched) HIPCHK(hipMemsetAsync(ctx->L.touched, 0, ctx->T_cap, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->since_sort = 1 << 30;
    clear_graphs(ctx);
    return MPM_OK;
}

hipEvent_t take_event(mpm_ctx ctx)
{
    if (!ctx->ev_pool.empty()) {
        hipEvent_t e = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Times one launch when timing is on: a single substep kernel (P2G, grid,
// G2P, G2P2G) through events the runtime records at the kernel's own start
// and end; the sort (several kernels) and the cooperative substep through
// events recorded on the stream around them.
struct KTimer {
    mpm_ctx ctx;
    int cls;
    bool own;
    hipEvent_t a = nullptr, b = nullptr;
    KTimer(mpm_ctx c, int k) : ctx(c), cls(k), own(k == MPM_K_SORT || k == MPM_K_PERSISTENT)
    {
        if (ctx->timing) {
            a = take_event(ctx);
            b = take_event(ctx);
            if (a && b) {
                if (own) (void)hipEventRecord(a, ctx->stream);
                else time_next_launch(a, b);
            }
        }
    }
    ~KTimer()
    {
        if (ctx->timing && a && b) {
            if (own) (void)hipEventRecord(b, ctx->stream);
            else time_next_launch(nullptr, nullptr);   // the launch took them (or failed before)
            ctx->ev_pending.push_back({cls, {a, b}});
        }
    }
};

hipError_t resolve_timing(mpm_ctx ctx)
{
    for (auto &p : ctx->ev_pending) {
        hipError_t e = hipEventSynchronize(p.second.second);
        if (e != hipSuccess) return e;
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, p.second.first, p.second.second);
        if (e != hipSuccess) return e;
        ctx->kt_ms[p.first] += ms;
        ctx->kt_n[p.first] += 1;
        ctx->ev_pool.push_back(p.second.first);
        ctx->ev_pool.push_back(p.second.second);
    }
    ctx->ev_pending.clear();
    return hipSuccess;
}

SortArgs sort_args(mpm_ctx ctx)
{
    SortArgs a{};
    a.scenes = ctx->d_scenes;
    a.n_scenes = ctx->n_scenes;
    a.psc = ctx->d_psc;
    a.P = ctx->d_P[ctx->cur];
    a.Pn = ctx->d_P[1 - ctx->cur];
    a.pstride = ctx->pstride;
    a.N = ctx->N;
    a.T = ctx->T;
    a.scene_bin_off = ctx->d_scene_bin_off;
    a.keys = ctx->d_keys;
    a.count = ctx->d_count;
    a.pstart = ctx->d_pstart;
    a.perm = ctx->d_perm;
    a.perm2 = (int *)ctx->d_keys;   // the keys are dead once the scatter has run
    a.tsum = ctx->d_tsum;
    a.dil = ctx->d_dil;
    a.L = ctx->L;
    a.B = ctx->B;
    a.CH = ctx->CH;
    return a;
}

StepArgs step_args(mpm_ctx ctx, int substep)
{
    StepArgs a{};
    a.scenes = ctx->d_scenes;
    a.n_scenes = ctx->n_scenes;
    a.P = ctx->d_P[ctx->cur];
    a.pstride = ctx->pstride;
    long long n = ctx->n_nodes;
    a.gm = ctx->d_grid;
    a.gpx = ctx->d_grid + n;
    a.gpy = ctx->d_grid + 2 * n;
    a.gpz = ctx->d_grid + 3 * n;
    a.gvx = ctx->d_grid + 4 * n;
    a.gvy = ctx->d_grid + 5 * n;
    a.gvz = ctx->d_grid + 6 * n;
    a.cap = ctx->capture ? ctx->d_cap : nullptr;
    a.cap_off = ctx->d_cap_off;
    a.cols = ctx->d_cols;
    a.colnow = ctx->d_colnow;
    a.L = ctx->L;
    a.flags = ctx->d_flags;
    a.substep = substep;
    a.B = ctx->B;
    a.active = ctx->d_active;
    a.dense = nullptr;
    a.feat = nullptr;
    a.cf = 0;
    a.keep_bound = 0;
    a.wrench = ctx->d_wrench;
    a.sdf = ctx->d_sdf;
    a.contact = ctx->contact;
    a.nt = ctx->nt;
    a.chain = 0;
    return a;
}

mpm_status do_sort(mpm_ctx ctx)
{
    KTimer kt(ctx, MPM_K_SORT);
    HIPCHK(launch_sort(sort_args(ctx), ctx->stream));
    ctx->cnt[MPM_CNT_SORTS]++;
    ctx->cur = 1 - ctx->cur;
    ctx->since_sort = 0;
    return MPM_OK;
}

// Workgroups per launch.  The particle kernels stride statically over work
// items of uneven size; launching many more workgroups than fit at once lets
// the hardware dispatcher hand the remaining items to whichever CU frees up
// first (measured on cfg3: P2G and G2P best at 32 per CU, the grid update,
// whose unit is one wave per block, at 16).
int substep_wgs(mpm_ctx ctx) { return ctx->cus * 32; }
int grid_wgs(mpm_ctx ctx) { return ctx->cus * 16; }

// Queue n substeps (sort when due, P2G, grid, G2P) and the collider advance.
// With fusion on, a run of substeps with no re-sort inside is queued as
// P2G, grid, (G2P2G, grid) x (run - 1), G2P: the G2P of one substep and the
// P2G of the next share a pass over the particles, and the state at the end
// of the run (and at a re-sort) is complete again.
mpm_status queue_plain(mpm_ctx ctx, int n)
{
    int i = 0;
    while (i < n) {
        if (ctx->since_sort >= ctx->sort_every) {
            mpm_status st = do_sort(ctx);
            if (st != MPM_OK) return st;
        }
        if (ctx->persistent && !ctx->capture) {
            StepArgs a = step_args(ctx, i);
            KTimer kt(ctx, MPM_K_PERSISTENT);
            // about one work item per workgroup: the grid-wide barriers cost per workgroup
            const long long per_cu = ((long long)ctx->N + (long long)ctx->CH * ctx->cus - 1) / ((long long)ctx->CH * ctx->cus);
            HIPCHK(launch_persistent(a, ctx->cus, (int)std::min<long long>(per_cu, 64), ctx->stream));
            ctx->since_sort++;
            ctx->cnt[MPM_CNT_SUBSTEPS]++;
            ctx->cnt[MPM_CNT_HOST_SUBSTEPS]++;
            i++;
            continue;
        }
        // substeps until the end of the call or the next re-sort
        const int run = ctx->fuse ? std::min(n - i, ctx->sort_every - ctx->since_sort) : 1;
        {
            KTimer kt(ctx, MPM_K_P2G);
            StepArgs a = step_args(ctx, i);
            a.chain = run > 1;   // the fused G2P reads the scatter bound and cell count of this state
            HIPCHK(launch_p2g(a, ctx->CH, substep_wgs(ctx), ctx->stream));
        }
        for (int k = i; k < i + run; k++) {
            StepArgs a = step_args(ctx, k);
            if (ctx->capture) HIPCHK(launch_clear_f(ctx->d_cap, 4 * ctx->cap_nodes, ctx->stream));
            {
                KTimer kt(ctx, MPM_K_GRID);
                HIPCHK(launch_grid(a, grid_wgs(ctx), ctx->stream));
            }
            if (k + 1 < i + run) {
                KTimer kt(ctx, MPM_K_G2P2G);
                HIPCHK(launch_g2p2g(a, substep_wgs(ctx), ctx->stream));
            } else {
                KTimer kt(ctx, MPM_K_G2P);
                HIPCHK(launch_g2p(a, substep_wgs(ctx), ctx->stream));
            }
        }
        ctx->since_sort += run;
        ctx->cnt[MPM_CNT_SUBSTEPS] += run;
        ctx->cnt[MPM_CNT_HOST_SUBSTEPS] += run;
        i += run;
    }
    HIPCHK(launch_collider_advance(ctx->d_cols, (int)ctx->h_cols.size(), ctx->d_col_scene, ctx->d_scenes, n,
                                   ctx->stream));
    return MPM_OK;
}

// One control step of GRAPH_BLOCK substeps replayed from a captured hipGraph
// (captured on first use for the current buffer parity and sort phase).
mpm_status queue_graph_block(mpm_ctx ctx)
{
    GraphKey key{ctx->cur, std::min(ctx->since_sort, ctx->sort_every), ctx->sort_every};
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
        const int cur0 = ctx->cur, ss0 = ctx->since_sort;
        long long cnt0[MPM_NCOUNTERS];
        std::copy(ctx->cnt, ctx->cnt + MPM_NCOUNTERS, cnt0);
        ctx->since_sort = key.since_sort;
        HIPCHK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
        mpm_status st = queue_plain(ctx, GRAPH_BLOCK);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(ctx->stream, &g);
        const long long captured_sorts = ctx->cnt[MPM_CNT_SORTS] - cnt0[MPM_CNT_SORTS];
        std::copy(cnt0, cnt0 + MPM_NCOUNTERS, ctx->cnt);   // captured, not run
        if (st != MPM_OK || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            ctx->cur = cur0;
            ctx->since_sort = ss0;
            if (st == MPM_OK) HIPCHK(e);
            return st;
        }
        GraphEntry ent;
        e = hipGraphInstantiate(&ent.exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            ctx->cur = cur0;
            ctx->since_sort = ss0;
            HIPCHK(e);
        }
        ent.end_parity = ctx->cur;
        ent.end_since_sort = ctx->since_sort;
        ent.n_sorts = captured_sorts;
        ctx->cur = cur0;
        it = ctx->graphs.emplace(key, ent).first;
    }
    HIPCHK(hipGraphLaunch(it->second.exec, ctx->stream));
    ctx->cnt[MPM_CNT_GRAPH_LAUNCHES]++;
    ctx->cnt[MPM_CNT_SUBSTEPS] += GRAPH_BLOCK;
    ctx->cnt[MPM_CNT_SORTS] += it->second.n_sorts;
    ctx->cur = it->second.end_parity;
    ctx->since_sort = it->second.end_since_sort;
    return MPM_OK;
}

mpm_status queue_substeps(mpm_ctx ctx, int n)
{
    if (ctx->graph && !ctx->timing && !ctx->capture && !ctx->persistent) {
        while (n >= GRAPH_BLOCK) {
            mpm_status st = queue_graph_block(ctx);
            if (st != MPM_OK) return st;
            n -= GRAPH_BLOCK;
        }
    }
    return n > 0 ? queue_plain(ctx, n) : MPM_OK;
}

// Copies between caller memory and a device buffer of the context.
mpm_status to_device(mpm_ctx ctx, void *dst, const void *src, size_t bytes, int on_device)
{
    if (bytes == 0) return MPM_OK;
    HIPCHK(hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, ctx->stream));
    if (!on_device) HIPCHK(hipStreamSynchronize(ctx->stream));
    return MPM_OK;
}

mpm_status from_device(mpm_ctx ctx, void *dst, const void *src, size_t bytes, int on_device)
{
    if (bytes == 0) return MPM_OK;
    HIPCHK(hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, ctx->stream));
    if (!on_device) HIPCHK(hipStreamSynchronize(ctx->stream));
    return MPM_OK;
}

void scene_range(mpm_ctx ctx, int scene, int &b, int &e)
{
    if (scene < 0) {
        b = 0;
        e = ctx->N;
    } else {
        b = ctx->h_scenes[scene].p_begin;
        e = ctx->h_scenes[scene].p_end;
    }
}

void release(mpm_ctx ctx)
{
    if (!ctx) return;
    hipSetDevice(ctx->dev);
    if (ctx->stream) hipStreamSynchronize(ctx->stream);
    clear_graphs(ctx);
    surnet_destroy(ctx->net);
    for (auto &p : ctx->ev_pending) {
        ctx->ev_pool.push_back(p.second.first);
        ctx->ev_pool.push_back(p.second.second);
    }
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    void *bufs[] = {ctx->d_scenes, ctx->d_psc, ctx->d_P[0], ctx->d_P[1], ctx->d_grid, ctx->d_cols, ctx->d_colnow,
                    ctx->d_col_scene, ctx->d_scene_bin_off, ctx->d_keys, ctx->d_count, ctx->d_pstart, ctx->d_perm,
                    ctx->d_tsum, ctx->d_dil, ctx->L.items, ctx->L.gitems, ctx->L.n_items, ctx->L.n_gitems,
                    ctx->L.scene_item_begin, ctx->L.scene_gitem_begin, ctx->L.bflag, ctx->L.ovf, ctx->L.n_ovf, ctx->L.ibound, ctx->L.icell, ctx->L.touched,
                    ctx->L.order, ctx->d_flags, ctx->d_cap, ctx->d_cap_off, ctx->d_io,
                    ctx->d_active, ctx->d_sur_gend, ctx->d_sur_acc, ctx->d_sur_out, ctx->d_sur_nfb,
                    ctx->d_wrench, ctx->d_wrench_out, ctx->d_sdf, ctx->d_sb_box, ctx->d_sb_origin, ctx->d_sb_feat,
                    ctx->d_sb_grid0, ctx->d_sb_pred, ctx->d_sb_res};
    for (void *p : bufs)
        if (p) hipFree(p);
    for (int i = 0; i < STAGE_RING; i++) {
        if (ctx->h_stage[i]) hipHostFree(ctx->h_stage[i]);
        if (ctx->stage_ev[i]) hipEventDestroy(ctx->stage_ev[i]);
    }
    if (ctx->own_stream && ctx->stream) hipStreamDestroy(ctx->stream);
    delete ctx;
}

mpm_status create_impl(mpm_ctx ctx, const mpm_scene_desc *scenes, int n_scenes)
{
    ctx->n_scenes = n_scenes;
    ctx->descs.assign(scenes, scenes + n_scenes);
    long long N = 0;
    for (int s = 0; s < n_scenes; s++) N += scenes[s].n_particles;
    if (N > (1LL << 30)) {
        ctx->last_error = "too many particles";
        return MPM_ERR_ARG;
    }
    ctx->N = (int)N;
    ctx->pstride = std::max<long long>(N, 1);
    int p = 0;
    for (int s = 0; s < n_scenes; s++) {
        const mpm_scene_desc &d = scenes[s];
        ctx->h_scenes.push_back(make_scene(d, p, (int)ctx->h_cols.size(), 4));
        for (int k = 0; k < d.n_colliders; k++) {
            const mpm_collider_shape &c = d.colliders[k];
            ColliderDev cd{};
            cd.type = c.type;
            for (int a = 0; a < 3; a++) cd.he[a] = c.half_extents[a];
            cd.radius = c.radius;
            cd.half_length = c.half_length;
            cd.friction = c.friction;
            cd.quat[0] = 1.0f;
            if (c.type == 2) {
                const long long n = (long long)c.sdf_dims[0] * c.sdf_dims[1] * c.sdf_dims[2];
                cd.sdf_off = (int)ctx->h_sdf.size();
                ctx->h_sdf.insert(ctx->h_sdf.end(), c.sdf, c.sdf + n);
                for (int a = 0; a < 3; a++) {
                    cd.sdf_dims[a] = c.sdf_dims[a];
                    cd.sdf_origin[a] = c.sdf_origin[a];
                }
                cd.sdf_cell = c.sdf_cell;
            }
            ctx->h_cols.push_back(cd);
            ctx->h_col_scene.push_back(s);
        }
        ctx->max_col = std::max(ctx->max_col, d.n_colliders);
        p += d.n_particles;
    }
    // sizes
    long long nodes = 0;
    int T4 = 0;
    for (int s = 0; s < n_scenes; s++) {
        int r = scenes[s].res;
        nodes += (long long)r * r * r;
        T4 += (r / 4) * (r / 4) * (r / 4);
    }
    ctx->n_nodes = nodes;
    ctx->T_cap = T4;
    ctx->items_cap = (int)std::min<long long>(N / 64 + T4 + 8, 1LL << 30);

    HIPCHK(dalloc(&ctx->d_scenes, n_scenes));
    HIPCHK(dalloc(&ctx->d_psc, N));
    for (int b = 0; b < 2; b++) HIPCHK(dalloc(&ctx->d_P[b], (size_t)NCOMP * ctx->pstride));
    HIPCHK(dalloc(&ctx->d_grid, (size_t)7 * nodes));
    HIPCHK(dalloc(&ctx->d_cols, ctx->h_cols.size()));
    HIPCHK(hipMalloc(&ctx->d_colnow, std::max<size_t>(ctx->h_cols.size(), 1) * collider_now_bytes()));
    if (ctx->h_sdf.size() > (size_t)INT32_MAX) {
        ctx->last_error = "SDF volumes: more than 2^31 samples in total";
        return MPM_ERR_ARG;
    }
    HIPCHK(dalloc(&ctx->d_sdf, std::max<size_t>(ctx->h_sdf.size(), 1)));
    if (!ctx->h_sdf.empty())
        HIPCHK(hipMemcpy(ctx->d_sdf, ctx->h_sdf.data(), sizeof(float) * ctx->h_sdf.size(), hipMemcpyHostToDevice));
    HIPCHK(dalloc(&ctx->d_wrench, std::max<size_t>(ctx->h_cols.size(), 1) * 6));
    HIPCHK(dalloc(&ctx->d_wrench_out, std::max<size_t>((size_t)n_scenes * ctx->max_col, 1) * 6));
    HIPCHK(dalloc(&ctx->d_col_scene, ctx->h_cols.size()));
    HIPCHK(dalloc(&ctx->d_scene_bin_off, n_scenes + 1));
    HIPCHK(dalloc(&ctx->d_keys, N));
    HIPCHK(dalloc(&ctx->d_count, T4));
    HIPCHK(dalloc(&ctx->d_pstart, T4));
    HIPCHK(dalloc(&ctx->d_perm, N));
    HIPCHK(dalloc(&ctx->d_tsum, (T4 + 2047) / 2048 + 1));
    HIPCHK(dalloc(&ctx->d_dil, T4));
    HIPCHK(dalloc(&ctx->L.items, ctx->items_cap));
    HIPCHK(dalloc(&ctx->L.ibound, ctx->items_cap));
    HIPCHK(dalloc(&ctx->L.icell, ctx->items_cap));
    HIPCHK(dalloc(&ctx->L.order, ctx->items_cap));
    HIPCHK(dalloc(&ctx->L.gitems, T4));
    HIPCHK(dalloc(&ctx->L.n_items, 1));
    HIPCHK(dalloc(&ctx->L.n_gitems, 1));
    HIPCHK(dalloc(&ctx->L.scene_item_begin, n_scenes + 1));
    HIPCHK(dalloc(&ctx->L.scene_gitem_begin, n_scenes + 1));
    HIPCHK(dalloc(&ctx->L.bflag, T4));
    HIPCHK(dalloc(&ctx->L.touched, T4));
    HIPCHK(dalloc(&ctx->L.ovf, T4));
    HIPCHK(dalloc(&ctx->L.n_ovf, 2));
    ctx->L.ovf_cap = T4;
    HIPCHK(dalloc(&ctx->d_flags, n_scenes));
    HIPCHK(dalloc(&ctx->d_active, n_scenes));
    HIPCHK(launch_fill_i(ctx->d_active, n_scenes, 1, ctx->stream));
    {
        std::vector<long long> off(n_scenes);
        long long tot = 0;
        for (int s = 0; s < n_scenes; s++) {
            off[s] = tot;
            long long r = scenes[s].res;
            tot += r * r * r;
        }
        ctx->cap_nodes = tot;
        HIPCHK(dalloc(&ctx->d_cap_off, n_scenes));
        HIPCHK(hipMemcpy(ctx->d_cap_off, off.data(), sizeof(long long) * n_scenes, hipMemcpyHostToDevice));
    }
    HIPCHK(dalloc(&ctx->d_io, (size_t)24 * N));
    for (int i = 0; i < STAGE_RING; i++) {
        size_t bytes = std::max<size_t>(ctx->h_cols.size(), 1) * sizeof(ColliderDev) + 64;
        HIPCHK(hipHostMalloc((void **)&ctx->h_stage[i], bytes, hipHostMallocDefault));
        HIPCHK(hipEventCreateWithFlags(&ctx->stage_ev[i], hipEventDisableTiming));
    }
    HIPCHK(hipMemsetAsync(ctx->d_count, 0, sizeof(int) * T4, ctx->stream));
    HIPCHK(hipMemsetAsync(ctx->L.bflag, 0, sizeof(int) * T4, ctx->stream));
    HIPCHK(hipMemsetAsync(ctx->L.touched, 0, T4, ctx->stream));
    HIPCHK(hipMemsetAsync(ctx->L.n_ovf, 0, 2 * sizeof(int), ctx->stream));
    HIPCHK(hipMemsetAsync(ctx->L.n_items, 0, sizeof(int), ctx->stream));
    HIPCHK(hipMemsetAsync(ctx->L.n_gitems, 0, sizeof(int), ctx->stream));
    HIPCHK(hipMemsetAsync(ctx->d_flags, 0, sizeof(int) * n_scenes, ctx->stream));
    HIPCHK(hipMemsetAsync(ctx->d_wrench, 0, sizeof(float) * 6 * std::max<size_t>(ctx->h_cols.size(), 1), ctx->stream));
    HIPCHK(hipMemsetAsync(ctx->d_P[0], 0, sizeof(float) * NCOMP * ctx->pstride, ctx->stream));
    HIPCHK(hipMemsetAsync(ctx->d_P[1], 0, sizeof(float) * NCOMP * ctx->pstride, ctx->stream));
    if (!ctx->h_cols.empty()) {
        HIPCHK(hipMemcpyAsync(ctx->d_cols, ctx->h_cols.data(), sizeof(ColliderDev) * ctx->h_cols.size(),
                              hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(hipMemcpyAsync(ctx->d_col_scene, ctx->h_col_scene.data(), sizeof(int) * ctx->h_col_scene.size(),
                              hipMemcpyHostToDevice, ctx->stream));
    }
    std::vector<int> psc(N);
    for (int s = 0; s < n_scenes; s++)
        for (int i = ctx->h_scenes[s].p_begin; i < ctx->h_scenes[s].p_end; i++) psc[i] = s;
    HIPCHK(hipMemcpyAsync(ctx->d_psc, psc.data(), sizeof(int) * N, hipMemcpyHostToDevice, ctx->stream));
    mpm_status st = set_block(ctx, 4);
    if (st != MPM_OK) return st;
    // particles: upload x, v per scene into d_io and convert
    for (int s = 0; s < n_scenes; s++) {
        const mpm_scene_desc &d = scenes[s];
        if (d.n_particles == 0) continue;
        float *dx_ = ctx->d_io, *dv_ = ctx->d_io + 3LL * d.n_particles;
        HIPCHK(hipMemcpy(dx_, d.x, sizeof(float) * 3 * d.n_particles, hipMemcpyHostToDevice));
        if (d.v) HIPCHK(hipMemcpy(dv_, d.v, sizeof(float) * 3 * d.n_particles, hipMemcpyHostToDevice));
        HIPCHK(launch_init_particles(ctx->d_scenes, n_scenes, ctx->d_psc, ctx->d_P[ctx->cur], ctx->pstride, dx_,
                                     d.v ? dv_ : nullptr, nullptr, nullptr, ctx->h_scenes[s].p_begin,
                                     ctx->h_scenes[s].p_end, ctx->d_flags, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    st = do_sort(ctx);
    if (st != MPM_OK) return st;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return MPM_OK;
}

}  // namespace

extern "C" {

const char *mpm_status_string(mpm_status s)
{
    switch (s) {
    case MPM_OK: return "ok";
    case MPM_WARN_CLAMPED: return "warning: particle stencil clamped at the grid edge";
    case MPM_WARN_FALLBACK: return "warning: fallback";
    case MPM_ERR_ARG: return "invalid argument";
    case MPM_ERR_HIP: return "HIP runtime error";
    case MPM_ERR_OOM: return "out of device memory";
    case MPM_ERR_NONFINITE: return "non-finite particle state";
    case MPM_ERR_STATE: return "call not valid in the current state";
    }
    return "unknown status";
}

const char *mpm_last_error(mpm_ctx ctx) { return ctx ? ctx->last_error.c_str() : "null context"; }

mpm_status mpm_create(const mpm_scene_desc *scenes, int n_scenes, void *hip_stream, mpm_ctx *out)
{
    mpm_ctx ctx = nullptr;
    if (!out) return MPM_ERR_ARG;
    *out = nullptr;
    if (!scenes || n_scenes <= 0 || n_scenes > (1 << 20)) return MPM_ERR_ARG;
    for (int s = 0; s < n_scenes; s++) {
        mpm_status st = validate_desc(nullptr, scenes[s], s);
        if (st != MPM_OK) return st;
    }
    ctx = new mpm_ctx_s();
    if (hipGetDevice(&ctx->dev) != hipSuccess) {
        delete ctx;
        return MPM_ERR_HIP;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, ctx->dev) == hipSuccess) ctx->cus = prop.multiProcessorCount;
    if (hip_stream) {
        ctx->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
            delete ctx;
            return MPM_ERR_HIP;
        }
        ctx->own_stream = true;
    }
    mpm_status st = create_impl(ctx, scenes, n_scenes);
    if (st != MPM_OK) {
        std::fprintf(stderr, "mpm_create: %s\n", ctx->last_error.c_str());
        release(ctx);
        return st;
    }
    *out = ctx;
    return MPM_OK;
}

mpm_status mpm_destroy(mpm_ctx ctx)
{
    release(ctx);
    return MPM_OK;
}

int mpm_num_scenes(mpm_ctx ctx) { return ctx ? ctx->n_scenes : 0; }
int mpm_num_particles(mpm_ctx ctx, int scene)
{
    if (!ctx) return 0;
    if (scene < 0) return ctx->N;
    if (scene >= ctx->n_scenes) return 0;
    return ctx->h_scenes[scene].p_end - ctx->h_scenes[scene].p_begin;
}
int mpm_max_colliders(mpm_ctx ctx) { return ctx ? ctx->max_col : 0; }
int mpm_res(mpm_ctx ctx, int scene)
{
    if (!ctx || scene < 0 || scene >= ctx->n_scenes) return 0;
    return ctx->h_scenes[scene].res;
}

mpm_status mpm_set_colliders(mpm_ctx ctx, const float *poses, const float *velocities, int on_device)
{
    ARGCHK(ctx, "null context");
    ARGCHK(poses && velocities, "poses / velocities must not be NULL");
    if (ctx->h_cols.empty()) return MPM_OK;
    hipSetDevice(ctx->dev);
    int K = ctx->max_col;
    std::vector<float> hp((size_t)ctx->n_scenes * K * 7), hv((size_t)ctx->n_scenes * K * 6);
    if (on_device) {
        HIPCHK(hipMemcpyAsync(hp.data(), poses, hp.size() * 4, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipMemcpyAsync(hv.data(), velocities, hv.size() * 4, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    } else {
        std::memcpy(hp.data(), poses, hp.size() * 4);
        std::memcpy(hv.data(), velocities, hv.size() * 4);
    }
    for (size_t c = 0; c < ctx->h_cols.size(); c++) {
        int s = ctx->h_col_scene[c];
        int k = (int)c - ctx->h_scenes[s].col_off;
        const float *P = &hp[((size_t)s * K + k) * 7];
        const float *V = &hv[((size_t)s * K + k) * 6];
        for (int i = 0; i < 13; i++) ARGCHK(std::isfinite(i < 7 ? P[i] : V[i - 7]), "non-finite collider pose");
        ColliderDev &cd = ctx->h_cols[c];
        for (int a = 0; a < 3; a++) {
            cd.pos[a] = P[a];
            cd.vlin[a] = V[a];
            cd.omega[a] = V[3 + a];
        }
        for (int a = 0; a < 4; a++) cd.quat[a] = P[3 + a];
    }
    int slot = ctx->stage_next;
    ctx->stage_next = (slot + 1) % STAGE_RING;
    HIPCHK(hipEventSynchronize(ctx->stage_ev[slot]));
    std::memcpy(ctx->h_stage[slot], ctx->h_cols.data(), sizeof(ColliderDev) * ctx->h_cols.size());
    HIPCHK(hipMemcpyAsync(ctx->d_cols, ctx->h_stage[slot], sizeof(ColliderDev) * ctx->h_cols.size(),
                          hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipEventRecord(ctx->stage_ev[slot], ctx->stream));
    return MPM_OK;
}

mpm_status mpm_get_collider_wrenches(mpm_ctx ctx, float *out, int on_device)
{
    ARGCHK(ctx, "null context");
    ARGCHK(out, "out must not be NULL");
    hipSetDevice(ctx->dev);
    const size_t n = (size_t)ctx->n_scenes * ctx->max_col * 6;
    if (n == 0) return MPM_OK;
    HIPCHK(launch_wrench_out(ctx->d_scenes, ctx->n_scenes, ctx->max_col, ctx->d_wrench, ctx->d_wrench_out, ctx->stream));
    return from_device(ctx, out, ctx->d_wrench_out, sizeof(float) * n, on_device);
}

mpm_status mpm_step(mpm_ctx ctx, int n_substeps)
{
    ARGCHK(ctx, "null context");
    ARGCHK(n_substeps >= 0, "n_substeps must be >= 0");
    if (n_substeps == 0) return MPM_OK;
    hipSetDevice(ctx->dev);
    return queue_substeps(ctx, n_substeps);
}

mpm_status mpm_sync(mpm_ctx ctx)
{
    ARGCHK(ctx, "null context");
    hipSetDevice(ctx->dev);
    HIPCHK(hipStreamSynchronize(ctx->stream));
    std::vector<int> fl(ctx->n_scenes);
    HIPCHK(hipMemcpy(fl.data(), ctx->d_flags, sizeof(int) * ctx->n_scenes, hipMemcpyDeviceToHost));
    int any = 0;
    for (int f : fl) any |= f;
    if (any) HIPCHK(hipMemset(ctx->d_flags, 0, sizeof(int) * ctx->n_scenes));
    if (any & FLAG_NONFINITE) {
        ctx->last_error = "non-finite particle state";
        return MPM_ERR_NONFINITE;
    }
    if (any & FLAG_OVERFLOW_FULL) {
        ctx->last_error = "overflow grid-block list full";
        return MPM_ERR_STATE;
    }
    if (any & FLAG_CLAMPED) return MPM_WARN_CLAMPED;
    return MPM_OK;
}

mpm_status mpm_get_state(mpm_ctx ctx, int scene, float *x, float *v, float *C, float *F, int on_device)
{
    ARGCHK(ctx, "null context");
    ARGCHK(scene >= -1 && scene < ctx->n_scenes, "scene out of range");
    hipSetDevice(ctx->dev);
    int b, e;
    scene_range(ctx, scene, b, e);
    long long n = e - b;
    float *dx_ = ctx->d_io, *dv_ = dx_ + 3 * n, *dC_ = dv_ + 3 * n, *dF_ = dC_ + 9 * n;
    HIPCHK(launch_get_state(ctx->d_scenes, ctx->d_psc, ctx->d_P[ctx->cur], ctx->pstride, b, e, x ? dx_ : nullptr,
                            v ? dv_ : nullptr, C ? dC_ : nullptr, F ? dF_ : nullptr, ctx->stream));
    mpm_status st = MPM_OK;
    if (x && (st = from_device(ctx, x, dx_, 12 * n, on_device)) != MPM_OK) return st;
    if (v && (st = from_device(ctx, v, dv_, 12 * n, on_device)) != MPM_OK) return st;
    if (C && (st = from_device(ctx, C, dC_, 36 * n, on_device)) != MPM_OK) return st;
    if (F && (st = from_device(ctx, F, dF_, 36 * n, on_device)) != MPM_OK) return st;
    return MPM_OK;
}

mpm_status mpm_get_particles(mpm_ctx ctx, int scene, float *x, float *v, float *F, int on_device)
{
    ARGCHK(x, "x must not be NULL");
    return mpm_get_state(ctx, scene, x, v, nullptr, F, on_device);
}

mpm_status mpm_particle_view(mpm_ctx ctx, const float **x, const float **y, const float **z, int *slot_begin)
{
    ARGCHK(ctx, "null context");
    ARGCHK(x && y && z, "x, y and z must not be NULL");
    const float *P = ctx->d_P[ctx->cur];
    *x = P + (long long)X0 * ctx->pstride;
    *y = P + (long long)X1 * ctx->pstride;
    *z = P + (long long)X2 * ctx->pstride;
    if (slot_begin) {
        for (int s = 0; s < ctx->n_scenes; s++) slot_begin[s] = ctx->h_scenes[s].p_begin;
        slot_begin[ctx->n_scenes] = ctx->n_scenes ? ctx->h_scenes[ctx->n_scenes - 1].p_end : 0;
    }
    return MPM_OK;
}

mpm_status mpm_set_state(mpm_ctx ctx, int scene, const float *x, const float *v, const float *C, const float *F,
                         int on_device)
{
    ARGCHK(ctx, "null context");
    ARGCHK(scene >= -1 && scene < ctx->n_scenes, "scene out of range");
    ARGCHK(x && v && C && F, "x, v, C and F are required");
    hipSetDevice(ctx->dev);
    int b, e;
    scene_range(ctx, scene, b, e);
    long long n = e - b;
    float *dx_ = ctx->d_io, *dv_ = dx_ + 3 * n, *dC_ = dv_ + 3 * n, *dF_ = dC_ + 9 * n;
    if (!on_device) {
        for (long long k = 0; k < 3 * n; k++) ARGCHK(std::isfinite(x[k]) && std::isfinite(v[k]), "non-finite x / v");
    }
    mpm_status st;
    if ((st = to_device(ctx, dx_, x, 12 * n, on_device)) != MPM_OK) return st;
    if ((st = to_device(ctx, dv_, v, 12 * n, on_device)) != MPM_OK) return st;
    if ((st = to_device(ctx, dC_, C, 36 * n, on_device)) != MPM_OK) return st;
    if ((st = to_device(ctx, dF_, F, 36 * n, on_device)) != MPM_OK) return st;
    HIPCHK(launch_init_particles(ctx->d_scenes, ctx->n_scenes, ctx->d_psc, ctx->d_P[ctx->cur], ctx->pstride, dx_, dv_,
                                 dC_, dF_, b, e, ctx->d_flags, ctx->stream));
    ctx->since_sort = 1 << 30;
    return MPM_OK;
}

mpm_status mpm_get_grid(mpm_ctx ctx, int scene, float *m, float *p, int on_device)
{
    ARGCHK(ctx, "null context");
    ARGCHK(scene >= 0 && scene < ctx->n_scenes, "scene out of range");
    if (!ctx->capture || !ctx->d_cap) {
        ctx->last_error = "grid capture is off";
        return MPM_ERR_STATE;
    }
    hipSetDevice(ctx->dev);
    long long r = ctx->h_scenes[scene].res, nn = r * r * r;
    long long off = 0;
    for (int s = 0; s < scene; s++) off += (long long)ctx->h_scenes[s].res * ctx->h_scenes[s].res * ctx->h_scenes[s].res;
    std::vector<float> h(4 * nn);
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipMemcpy(h.data(), ctx->d_cap + 4 * off, sizeof(float) * 4 * nn, hipMemcpyDeviceToHost));
    std::vector<float> hm(nn), hp(3 * nn);
    for (long long i = 0; i < nn; i++) {
        hm[i] = h[4 * i];
        for (int a = 0; a < 3; a++) hp[3 * i + a] = h[4 * i + 1 + a];
    }
    if (on_device) {
        if (m) HIPCHK(hipMemcpy(m, hm.data(), sizeof(float) * nn, hipMemcpyHostToDevice));
        if (p) HIPCHK(hipMemcpy(p, hp.data(), sizeof(float) * 3 * nn, hipMemcpyHostToDevice));
    } else {
        if (m) std::memcpy(m, hm.data(), sizeof(float) * nn);
        if (p) std::memcpy(p, hp.data(), sizeof(float) * 3 * nn);
    }
    return MPM_OK;
}

mpm_status mpm_set_option(mpm_ctx ctx, int option, int value)
{
    ARGCHK(ctx, "null context");
    hipSetDevice(ctx->dev);
    switch (option) {
    case MPM_OPT_SORT_EVERY:
        ARGCHK(value >= 1, "sort_every must be >= 1");
        ctx->sort_every = value;
        clear_graphs(ctx);
        return MPM_OK;
    case MPM_OPT_BLOCK: {
        ARGCHK(value == 4 || value == 8, "block must be 4 or 8");
        if (value == ctx->B) return MPM_OK;
        HIPCHK(hipStreamSynchronize(ctx->stream));
        return set_block(ctx, value);
    }
    case MPM_OPT_CHUNK:
        ARGCHK(value >= 64 && value <= 8192, "chunk must be in [64, 8192]");
        ctx->CH = value;
        ctx->since_sort = 1 << 30;
        clear_graphs(ctx);
        return MPM_OK;
    case MPM_OPT_PERSISTENT:
        ARGCHK(value == 0 || value == 1, "persistent must be 0 or 1");
        ctx->persistent = value;
        clear_graphs(ctx);
        return MPM_OK;
    case MPM_OPT_GRAPH:
        ARGCHK(value == 0 || value == 1, "graph must be 0 or 1");
        ctx->graph = value;
        return MPM_OK;
    case MPM_OPT_FUSE:
        ARGCHK(value == 0 || value == 1, "fuse must be 0 or 1");
        ctx->fuse = value;
        clear_graphs(ctx);   // the captured kernels depend on it
        return MPM_OK;
    case MPM_OPT_WG:
        ARGCHK(value == 256 || value == 512, "workgroup size must be 256 or 512");
        ctx->nt = value;
        clear_graphs(ctx);   // the captured kernels depend on it
        return MPM_OK;
    case MPM_OPT_CONTACT:
        ARGCHK(value >= 0 && value <= 2, "contact must be 0, 1 or 2");
        ctx->contact = value;
        clear_graphs(ctx);   // the captured kernels depend on it
        return MPM_OK;
    case MPM_OPT_CAPTURE_GRID:
        ARGCHK(value == 0 || value == 1, "capture must be 0 or 1");
        if (value && !ctx->d_cap) {
            HIPCHK(dalloc(&ctx->d_cap, (size_t)4 * ctx->cap_nodes));
            HIPCHK(launch_clear_f(ctx->d_cap, 4 * ctx->cap_nodes, ctx->stream));
        }
        ctx->capture = value;
        return MPM_OK;
    case MPM_OPT_TIMING:
        ARGCHK(value == 0 || value == 1, "timing must be 0 or 1");
        ctx->timing = value;
        return MPM_OK;
    }
    ctx->last_error = "unknown option";
    return MPM_ERR_ARG;
}

mpm_status mpm_get_option(mpm_ctx ctx, int option, int *value)
{
    ARGCHK(ctx && value, "null argument");
    switch (option) {
    case MPM_OPT_SORT_EVERY: *value = ctx->sort_every; return MPM_OK;
    case MPM_OPT_BLOCK: *value = ctx->B; return MPM_OK;
    case MPM_OPT_CHUNK: *value = ctx->CH; return MPM_OK;
    case MPM_OPT_PERSISTENT: *value = ctx->persistent; return MPM_OK;
    case MPM_OPT_GRAPH: *value = ctx->graph; return MPM_OK;
    case MPM_OPT_CONTACT: *value = ctx->contact; return MPM_OK;
    case MPM_OPT_WG: *value = ctx->nt; return MPM_OK;
    case MPM_OPT_FUSE: *value = ctx->fuse; return MPM_OK;
    case MPM_OPT_CAPTURE_GRID: *value = ctx->capture; return MPM_OK;
    case MPM_OPT_TIMING: *value = ctx->timing; return MPM_OK;
    }
    ctx->last_error = "unknown option";
    return MPM_ERR_ARG;
}

mpm_status mpm_get_timing(mpm_ctx ctx, double *ms_total, long long *launches, int reset)
{
    ARGCHK(ctx, "null context");
    hipSetDevice(ctx->dev);
    HIPCHK(resolve_timing(ctx));
    for (int k = 0; k < MPM_KCLASSES; k++) {
        if (ms_total) ms_total[k] = ctx->kt_ms[k];
        if (launches) launches[k] = ctx->kt_n[k];
        if (reset) {
            ctx->kt_ms[k] = 0.0;
            ctx->kt_n[k] = 0;
        }
    }
    return MPM_OK;
}

mpm_status mpm_get_counters(mpm_ctx ctx, long long *out, int reset)
{
    ARGCHK(ctx && out, "null argument");
    std::copy(ctx->cnt, ctx->cnt + MPM_NCOUNTERS, out);
    if (reset) std::fill(ctx->cnt, ctx->cnt + MPM_NCOUNTERS, 0LL);
    return MPM_OK;
}

mpm_status mpm_get_order(mpm_ctx ctx, int *pid_out)
{
    ARGCHK(ctx && pid_out, "null argument");
    hipSetDevice(ctx->dev);
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (ctx->N > 0)
        HIPCHK(hipMemcpy(pid_out, ctx->d_P[ctx->cur] + (size_t)PID * ctx->pstride, sizeof(int) * ctx->N,
                         hipMemcpyDeviceToHost));
    return MPM_OK;
}

mpm_status mpm_set_scene_mask(mpm_ctx ctx, const int *active)
{
    ARGCHK(ctx, "null context");
    hipSetDevice(ctx->dev);
    std::vector<int> h(ctx->n_scenes, 1);
    if (active)
        for (int s = 0; s < ctx->n_scenes; s++) h[s] = active[s] != 0;
    HIPCHK(hipMemcpyAsync(ctx->d_active, h.data(), sizeof(int) * ctx->n_scenes, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return MPM_OK;
}

namespace {

// The grid resolution shared by every scene, or 0.
int common_res(mpm_ctx ctx)
{
    int r = ctx->n_scenes > 0 ? ctx->h_scenes[0].res : 0;
    for (int s = 1; s < ctx->n_scenes; s++)
        if (ctx->h_scenes[s].res != r) return 0;
    return r;
}

// The surrogate arrays of a call: per-scene boxes (origin on the device) or the whole grid.
mpm_status sur_box(mpm_ctx ctx, StepArgs &a, int R, const int *origin, int D, int H, int W)
{
    if (!origin) return MPM_OK;
    ARGCHK(D > 0 && H > 0 && W > 0 && D <= R && H <= R && W <= R, "box size must be in 1 .. res");
    a.sur_org = origin;
    a.sur_box[0] = D;
    a.sur_box[1] = H;
    a.sur_box[2] = W;
    return MPM_OK;
}

}  // namespace

mpm_status mpm_sur_bbox(mpm_ctx ctx, int *box)
{
    ARGCHK(ctx, "null context");
    ARGCHK(box, "box must not be NULL");
    const int R = common_res(ctx);
    ARGCHK(R > 0, "the surrogate needs one grid resolution for all scenes");
    hipSetDevice(ctx->dev);
    HIPCHK(launch_sur_bbox(step_args(ctx, 0), R, box, ctx->stream));
    return MPM_OK;
}

mpm_status mpm_sur_features(mpm_ctx ctx, float *feat, int cf, float *grid0, const int *origin, int D, int H, int W)
{
    ARGCHK(ctx, "null context");
    ARGCHK(feat && grid0, "feat and grid0 must not be NULL");
    ARGCHK(cf >= 8, "cf must be >= 8");
    const int R = common_res(ctx);
    ARGCHK(R > 0, "the surrogate needs one grid resolution for all scenes");
    hipSetDevice(ctx->dev);
    if (ctx->since_sort >= ctx->sort_every) {   // due, or the state was set: work lists and scatter bounds
        mpm_status st = do_sort(ctx);
        if (st != MPM_OK) return st;
    }
    StepArgs a = step_args(ctx, 0);
    mpm_status st = sur_box(ctx, a, R, origin, D, H, W);
    if (st != MPM_OK) return st;
    HIPCHK(launch_colliders_now(a, (int)ctx->h_cols.size(), ctx->d_col_scene, ctx->stream));
    HIPCHK(launch_sur_init(a, R, feat, cf, grid0, ctx->stream));
    a.dense = grid0;
    a.feat = feat;
    a.cf = cf;
    a.keep_bound = 1;   // the state does not change: its scatter bounds stay valid
    a.wrench = nullptr;   // not a substep: no impulse on the colliders
    HIPCHK(launch_p2g(a, ctx->CH, substep_wgs(ctx), ctx->stream));
    HIPCHK(launch_grid(a, grid_wgs(ctx), ctx->stream));
    HIPCHK(launch_fill_i(ctx->L.n_ovf, 2, 0, ctx->stream));   // the overflow list has been consumed
    return MPM_OK;
}

namespace {

// One surrogate control step (mpm_sur_block); with MPM_SUR_SYNC, *host_fb (when
// not NULL) receives the number of scenes that fell back.
mpm_status sur_block_impl(mpm_ctx ctx, const float *pred, int cp, const float *grid0, const int *origin, int D, int H,
                          int W, float threshold, int flags, float *residual, int *n_fallback, int *host_fb)
{
    ARGCHK(pred && grid0, "pred and grid0 must not be NULL");
    ARGCHK(cp >= 4 && cp % 4 == 0, "cp must be a multiple of 4 and >= 4");
    ARGCHK(threshold >= 0.0f, "threshold must be >= 0");
    ARGCHK((flags & ~(MPM_SUR_NO_FALLBACK | MPM_SUR_SYNC)) == 0, "unknown flag");
    const int R = common_res(ctx);
    ARGCHK(R > 0, "the surrogate needs one grid resolution for all scenes");
    hipSetDevice(ctx->dev);
    {
        StepArgs chk = step_args(ctx, 0);
        mpm_status st = sur_box(ctx, chk, R, origin, D, H, W);
        if (st != MPM_OK) return st;
    }
    if (!ctx->d_sur_gend) HIPCHK(dalloc(&ctx->d_sur_gend, (size_t)4 * ctx->cap_nodes));
    if (!ctx->d_sur_acc) HIPCHK(dalloc(&ctx->d_sur_acc, (size_t)4 * ctx->n_scenes));
    if (!ctx->d_sur_out) HIPCHK(dalloc(&ctx->d_sur_out, (size_t)ctx->n_scenes));
    if (!ctx->d_sur_nfb) HIPCHK(dalloc(&ctx->d_sur_nfb, 1));
    const int nsub = GRAPH_BLOCK;
    const int fallback = !(flags & MPM_SUR_NO_FALLBACK);
    if (ctx->since_sort >= ctx->sort_every) {
        mpm_status st = do_sort(ctx);
        if (st != MPM_OK) return st;
    }
    // snapshot into the sort's other buffer (dead until the next sort); only a fallback reads it
    if (fallback)
        HIPCHK(hipMemcpyAsync(ctx->d_P[1 - ctx->cur], ctx->d_P[ctx->cur], sizeof(float) * NCOMP * ctx->pstride,
                              hipMemcpyDeviceToDevice, ctx->stream));
    StepArgs a = step_args(ctx, 0);
    sur_box(ctx, a, R, origin, D, H, W);
    HIPCHK(launch_sur_advance(a, grid0, pred, cp, nsub, substep_wgs(ctx), ctx->stream));
    // re-splat the advanced particles (on the same box; mass landing outside it is counted)
    StepArgs r = step_args(ctx, nsub);
    sur_box(ctx, r, R, origin, D, H, W);
    const long long box_nodes = origin ? (long long)ctx->n_scenes * D * H * W : ctx->cap_nodes;
    HIPCHK(launch_clear_f(ctx->d_sur_gend, 4 * box_nodes, ctx->stream));
    HIPCHK(launch_clear_f(ctx->d_sur_out, ctx->n_scenes, ctx->stream));
    r.dense = ctx->d_sur_gend;
    r.out_mass = ctx->d_sur_out;
    a.out_mass = ctx->d_sur_out;   // read by the residual
    r.keep_bound = 1;   // bounds now cover both the start and the advanced state
    r.wrench = nullptr;   // the re-splat is a check, not a substep
    HIPCHK(launch_p2g(r, ctx->CH, substep_wgs(ctx), ctx->stream));
    HIPCHK(launch_grid(r, grid_wgs(ctx), ctx->stream));
    HIPCHK(launch_fill_i(ctx->L.n_ovf, 2, 0, ctx->stream));
    HIPCHK(launch_clear_f(ctx->d_sur_acc, 4 * ctx->n_scenes, ctx->stream));
    HIPCHK(launch_sur_residual(a, R, grid0, pred, cp, ctx->d_sur_gend, ctx->d_sur_acc, ctx->stream));
    HIPCHK(launch_fill_i(ctx->d_sur_nfb, 1, 0, ctx->stream));
    HIPCHK(launch_sur_decide(a, ctx->d_sur_acc, nsub, threshold, fallback, residual, ctx->d_active, ctx->d_sur_nfb,
                             ctx->stream));
    if (n_fallback)
        HIPCHK(hipMemcpyAsync(n_fallback, ctx->d_sur_nfb, sizeof(int), hipMemcpyDeviceToDevice, ctx->stream));
    bool run_plain = fallback;
    if (flags & MPM_SUR_SYNC) {
        int h = 0;
        HIPCHK(hipMemcpyAsync(&h, ctx->d_sur_nfb, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        run_plain = fallback && h > 0;
        if (host_fb) *host_fb = h;
    }
    if (run_plain) {
        // scenes over the threshold: back to the snapshot, then plain substeps on those scenes only
        HIPCHK(launch_sur_restore(ctx->d_P[1 - ctx->cur], ctx->d_P[ctx->cur], ctx->pstride, ctx->d_psc, ctx->d_active,
                                  ctx->N, ctx->stream));
        mpm_status st = queue_substeps(ctx, nsub);
        HIPCHK(launch_fill_i(ctx->d_active, ctx->n_scenes, 1, ctx->stream));
        if (st != MPM_OK) return st;
    } else {
        HIPCHK(launch_fill_i(ctx->d_active, ctx->n_scenes, 1, ctx->stream));
        HIPCHK(launch_collider_advance(ctx->d_cols, (int)ctx->h_cols.size(), ctx->d_col_scene, ctx->d_scenes, nsub,
                                       ctx->stream));
        ctx->since_sort += nsub;
    }
    return MPM_OK;
}

}  // namespace

mpm_status mpm_sur_block(mpm_ctx ctx, const float *pred, int cp, const float *grid0, const int *origin, int D, int H,
                         int W, float threshold, int flags, float *residual, int *n_fallback)
{
    ARGCHK(ctx, "null context");
    return sur_block_impl(ctx, pred, cp, grid0, origin, D, H, W, threshold, flags, residual, n_fallback, nullptr);
}

mpm_status mpm_surrogate_load(mpm_ctx ctx, const void *weights, size_t bytes)
{
    ARGCHK(ctx, "null context");
    ARGCHK(weights, "weights must not be NULL");
    ARGCHK(common_res(ctx) > 0, "the surrogate needs one grid resolution for all scenes");
    hipSetDevice(ctx->dev);
    std::string err;
    int code = 0;
    mpm::SurNet *net = mpm::surnet_load(weights, bytes, ctx->stream, &err, &code);
    if (!net) {
        ctx->last_error = err;
        return code == -1 ? MPM_ERR_ARG : (code == -3 ? MPM_ERR_OOM : MPM_ERR_HIP);
    }
    if (mpm::surnet_cin(net) > 8 || mpm::surnet_cout(net) % 4) {
        mpm::surnet_destroy(net);
        ctx->last_error = "the surrogate network must read at most the 8 feature channels and give a multiple of 4 "
                          "output channels";
        return MPM_ERR_ARG;
    }
    mpm::surnet_destroy(ctx->net);
    ctx->net = net;
    return MPM_OK;
}

namespace {

// Box of one surrogate block: the largest stencil extent of the batch plus a
// margin of SB_MARGIN nodes on each side, rounded up to a multiple of 8 (the
// network halves it twice) and at most the grid.
constexpr int SB_MARGIN = 4;

void block_box(const std::vector<int> &box, int n, int R, int dims[3])
{
    for (int d = 0; d < 3; d++) {
        int ext = 0;
        for (int s = 0; s < n; s++) ext = std::max(ext, box[6 * s + 3 + d] - box[6 * s + d]);
        ext += 2 * SB_MARGIN;
        ext = (ext + 7) / 8 * 8;
        dims[d] = std::min(R, std::max(8, ext));
    }
}

}  // namespace

mpm_status mpm_step_blocks(mpm_ctx ctx, int n_blocks, int use_surrogate, float residual_threshold,
                           int *fallback_count)
{
    ARGCHK(ctx, "null context");
    ARGCHK(n_blocks >= 0, "n_blocks must be >= 0");
    ARGCHK(residual_threshold >= 0.0f, "residual_threshold must be >= 0");
    hipSetDevice(ctx->dev);
    if (fallback_count) *fallback_count = 0;
    if (!use_surrogate) return queue_substeps(ctx, GRAPH_BLOCK * n_blocks);
    if (!ctx->net) {
        ctx->last_error = "no surrogate loaded (mpm_surrogate_load)";
        return MPM_ERR_STATE;
    }
    const int R = common_res(ctx);
    ARGCHK(R > 0, "the surrogate needs one grid resolution for all scenes");
    const int S = ctx->n_scenes;
    if (S == 0 || n_blocks == 0) return MPM_OK;
    if (!ctx->d_sb_box) HIPCHK(dalloc(&ctx->d_sb_box, (size_t)6 * S));
    if (!ctx->d_sb_origin) HIPCHK(dalloc(&ctx->d_sb_origin, (size_t)3 * S));
    if (!ctx->d_sb_res) HIPCHK(dalloc(&ctx->d_sb_res, (size_t)S));
    ctx->h_sb_box.resize((size_t)6 * S);
    const int cout = mpm::surnet_cout(ctx->net);
    int total = 0;
    for (int b = 0; b < n_blocks; b++) {
        mpm_status st = mpm_sur_bbox(ctx, ctx->d_sb_box);
        if (st != MPM_OK) return st;
        HIPCHK(hipMemcpyAsync(ctx->h_sb_box.data(), ctx->d_sb_box, sizeof(int) * 6 * S, hipMemcpyDeviceToHost,
                              ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        int dims[3];
        block_box(ctx->h_sb_box, S, R, dims);
        const long long nodes = (long long)S * dims[0] * dims[1] * dims[2];
        if (nodes > ctx->sb_nodes) {
            for (float **p : {&ctx->d_sb_feat, &ctx->d_sb_grid0, &ctx->d_sb_pred})
                if (*p) {
                    (void)hipFree(*p);
                    *p = nullptr;
                }
            ctx->sb_nodes = 0;
            HIPCHK(dalloc(&ctx->d_sb_feat, (size_t)8 * nodes));
            HIPCHK(dalloc(&ctx->d_sb_grid0, (size_t)4 * nodes));
            HIPCHK(dalloc(&ctx->d_sb_pred, (size_t)cout * nodes));
            ctx->sb_nodes = nodes;
        }
        if (mpm_nn_crop_origin(ctx->d_sb_box, S, R, dims[0], dims[1], dims[2], ctx->d_sb_origin, ctx->stream) != 0) {
            ctx->last_error = "surrogate box origin failed";
            return MPM_ERR_HIP;
        }
        st = mpm_sur_features(ctx, ctx->d_sb_feat, 8, ctx->d_sb_grid0, ctx->d_sb_origin, dims[0], dims[1], dims[2]);
        if (st != MPM_OK) return st;
        std::string err;
        const int r = mpm::surnet_forward(ctx->net, ctx->d_sb_feat, 8, S, dims[0], dims[1], dims[2], ctx->d_sb_pred,
                                          ctx->stream, &err);
        if (r != 0) {
            ctx->last_error = err;
            return r == -3 ? MPM_ERR_OOM : (r == -1 ? MPM_ERR_ARG : MPM_ERR_HIP);
        }
        int fb = 0;
        st = sur_block_impl(ctx, ctx->d_sb_pred, cout, ctx->d_sb_grid0, ctx->d_sb_origin, dims[0], dims[1], dims[2],
                            residual_threshold, MPM_SUR_SYNC, ctx->d_sb_res, nullptr, &fb);
        if (st != MPM_OK) return st;
        total += fb;
    }
    ctx->h_sb_res.resize(S);
    HIPCHK(hipMemcpyAsync(ctx->h_sb_res.data(), ctx->d_sb_res, sizeof(float) * S, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (fallback_count) *fallback_count = total;
    return total > 0 ? MPM_WARN_FALLBACK : MPM_OK;
}

mpm_status mpm_surrogate_residuals(mpm_ctx ctx, float *out)
{
    ARGCHK(ctx && out, "null argument");
    if ((int)ctx->h_sb_res.size() != ctx->n_scenes) {
        ctx->last_error = "no surrogate block has run (mpm_step_blocks)";
        return MPM_ERR_STATE;
    }
    std::copy(ctx->h_sb_res.begin(), ctx->h_sb_res.end(), out);
    return MPM_OK;
}

mpm_status mpm_sur_targets(mpm_ctx ctx, const float *g0, const float *g1, float *target, int ct, float *mask)
{
    ARGCHK(ctx, "null context");
    ARGCHK(g0 && g1 && target && mask, "null argument");
    ARGCHK(ct >= 4, "ct must be >= 4");
    const int R = common_res(ctx);
    ARGCHK(R > 0, "the surrogate needs one grid resolution for all scenes");
    hipSetDevice(ctx->dev);
    StepArgs a = step_args(ctx, 0);
    HIPCHK(launch_sur_targets(a, R, g0, g1, ct, target, mask, ctx->stream));
    return MPM_OK;
}

// Tuning results, keyed by device architecture, grid resolutions and
// particle-count bucket: kept for the life of the process and in a text file
// (one "key block chunk sort_every wg persistent fuse" line per tuning, the last one
// for a key wins), so that a later process on the same kind of workload starts tuned.
static std::map<std::string, std::vector<int>> g_tune_cache;

static std::string tune_key(mpm_ctx ctx)
{
    hipDeviceProp_t prop;
    std::string k = "dev";
    if (hipGetDeviceProperties(&prop, ctx->dev) == hipSuccess) k = prop.gcnArchName;
    for (char &c : k)
        if (c == ' ') c = '_';
    int resmask = 0;
    for (auto &S : ctx->h_scenes) resmask |= S.res;
    int bucket = 0;
    while ((1LL << bucket) < (long long)ctx->N) bucket++;
    char buf[128];
    std::snprintf(buf, sizeof buf, "|res%d|n2^%d|s%d|t2", resmask, bucket, ctx->n_scenes > 1 ? 1 : 0);
    return k + buf;
}

// The cache file: $MPM_AUTOTUNE_CACHE, else $XDG_CACHE_HOME/mpm_mi355x_autotune.txt,
// else $HOME/.cache/mpm_mi355x_autotune.txt ("" when none can be named).
static std::string tune_file()
{
    if (const char *f = std::getenv("MPM_AUTOTUNE_CACHE")) return f;
    if (const char *x = std::getenv("XDG_CACHE_HOME")) return std::string(x) + "/mpm_mi355x_autotune.txt";
    if (const char *h = std::getenv("HOME")) return std::string(h) + "/.cache/mpm_mi355x_autotune.txt";
    return "";
}

static bool tune_file_lookup(const std::string &path, const std::string &key, std::vector<int> &best)
{
    if (path.empty()) return false;
    std::FILE *f = std::fopen(path.c_str(), "r");
    if (!f) return false;
    char line[512], k[256];
    int v[6];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        if (std::sscanf(line, "%255s %d %d %d %d %d %d", k, &v[0], &v[1], &v[2], &v[3], &v[4], &v[5]) != 7) continue;
        if (key == k && (v[0] == 4 || v[0] == 8) && v[1] >= 64 && v[1] <= 8192 && v[2] >= 1 &&
            (v[3] == 256 || v[3] == 512) && (v[4] == 0 || v[4] == 1) && (v[5] == 0 || v[5] == 1)) {
            best.assign(v, v + 6);
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

static void tune_file_store(const std::string &path, const std::string &key, const std::vector<int> &best)
{
    if (path.empty()) return;
    std::string dir = path.substr(0, path.find_last_of('/'));
    if (!dir.empty() && dir != path) (void)mkdir(dir.c_str(), 0755);
    if (std::FILE *f = std::fopen(path.c_str(), "a")) {
        std::fprintf(f, "%s %d %d %d %d %d %d\n", key.c_str(), best[0], best[1], best[2], best[3], best[4], best[5]);
        std::fclose(f);
    }
}

namespace {

// Device and host resources of one tuning run, released on every return.
struct TuneScratch {
    float *snap = nullptr;
    ColliderDev *csnap = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~TuneScratch()
    {
        if (snap) (void)hipFree(snap);
        if (csnap) (void)hipFree(csnap);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

}  // namespace

mpm_status mpm_autotune(mpm_ctx ctx, int substeps, char *report, size_t report_len)
{
    ARGCHK(ctx, "null context");
    ARGCHK(substeps >= 1 && substeps <= 1000, "substeps must be in [1, 1000]");
    hipSetDevice(ctx->dev);
    if (report && report_len) report[0] = 0;
    const std::string key = tune_key(ctx), path = tune_file();
    std::string rep;
    std::vector<int> best;
    auto hit = g_tune_cache.find(key);
    if (hit != g_tune_cache.end()) {
        best = hit->second;
        rep = "{\"cached\": true, \"source\": \"process\"";
    } else if (tune_file_lookup(path, key, best)) {
        g_tune_cache[key] = best;
        rep = "{\"cached\": true, \"source\": \"file\"";
    } else {
        // snapshot the particle state and the collider table
        const long long N = ctx->N;
        TuneScratch ts;
        HIPCHK(dalloc(&ts.snap, (size_t)24 * std::max<long long>(N, 1)));
        HIPCHK(dalloc(&ts.csnap, std::max<size_t>(ctx->h_cols.size(), 1)));
        float *sx = ts.snap, *sv = sx + 3 * N, *sC = sv + 3 * N, *sF = sC + 9 * N;
        mpm_status st = mpm_get_state(ctx, -1, sx, sv, sC, sF, 1);
        if (st != MPM_OK) return st;
        if (!ctx->h_cols.empty())
            HIPCHK(hipMemcpyAsync(ts.csnap, ctx->d_cols, sizeof(ColliderDev) * ctx->h_cols.size(),
                                  hipMemcpyDeviceToDevice, ctx->stream));
        // the trials' collider impulses are not the caller's: keep the accumulated wrenches
        std::vector<float> wsnap(6 * std::max<size_t>(ctx->h_cols.size(), 1));
        HIPCHK(hipMemcpyAsync(wsnap.data(), ctx->d_wrench, sizeof(float) * wsnap.size(), hipMemcpyDeviceToHost,
                              ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        const int saved[6] = {ctx->B, ctx->CH, ctx->sort_every, ctx->nt, ctx->persistent, ctx->fuse};
        ctx->persistent = 0;
        const int saved_timing = ctx->timing, saved_graph = ctx->graph;
        ctx->timing = 0;
        ctx->graph = 0;
        HIPCHK(hipEventCreate(&ts.e0));
        HIPCHK(hipEventCreate(&ts.e1));
        float best_ms = 1e30f;
        rep = "{\"cached\": false, \"trials\": [";
        bool first = true;
        // one trial: ms per substep of (B, CH, SE, WG, fused launches) on the snapshot, the sort included
        auto trial = [&](int B, int CH, int SE, int NT, int FU, mpm_status &st2) -> float {
            if (B != ctx->B && (st2 = set_block(ctx, B)) != MPM_OK) return -1.0f;
            ctx->CH = CH;
            ctx->sort_every = SE;
            ctx->nt = NT;
            ctx->fuse = FU;
            if ((st2 = mpm_set_state(ctx, -1, sx, sv, sC, sF, 1)) != MPM_OK) return -1.0f;
            if (!ctx->h_cols.empty() &&
                hipMemcpyAsync(ctx->d_cols, ts.csnap, sizeof(ColliderDev) * ctx->h_cols.size(),
                               hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess) {
                st2 = MPM_ERR_HIP;
                return -1.0f;
            }
            // one re-sort period untimed first (a state at rest speeds up over its first
            // substeps, which the fused launches' tile scale, taken from the previous
            // substep's bound, lags behind), then enough substeps that re-sorts are
            // amortised as in use, a re-sort included
            if ((st2 = queue_plain(ctx, SE)) != MPM_OK) return -1.0f;
            const int n = std::max(substeps, SE);
            float ms = 0.0f;
            if (hipEventRecord(ts.e0, ctx->stream) != hipSuccess) { st2 = MPM_ERR_HIP; return -1.0f; }
            if ((st2 = queue_plain(ctx, n)) != MPM_OK) return -1.0f;
            if (hipEventRecord(ts.e1, ctx->stream) != hipSuccess || hipEventSynchronize(ts.e1) != hipSuccess ||
                hipEventElapsedTime(&ms, ts.e0, ts.e1) != hipSuccess) {
                st2 = MPM_ERR_HIP;
                return -1.0f;
            }
            const float per = ms / n;
            char buf[192];
            std::snprintf(buf, sizeof buf,
                          "%s{\"block\": %d, \"chunk\": %d, \"sort_every\": %d, \"wg\": %d, \"persistent\": %d, "
                          "\"fuse\": %d, \"ms_per_substep\": %.5f}",
                          first ? "" : ", ", B, CH, SE, NT, ctx->persistent, FU, per);
            rep += buf;
            first = false;
            if (per < best_ms) {
                best_ms = per;
                best = {B, CH, SE, NT, ctx->persistent, FU};
            }
            st2 = MPM_OK;
            return per;
        };
        const int Bs[2] = {4, 8}, CHs[3] = {512, 2048, 8192}, SEs[4] = {10, 25, 50, 100};
        for (int B : Bs)
            for (int CH : CHs)
                for (int SE : SEs)
                    for (int FU = 0; FU < 2; FU++) {
                        trial(B, CH, SE, 256, FU, st);
                        if (st != MPM_OK) return st;
                    }
        // the workgroup size at the best (block, chunk, cadence, launches)
        {
            const std::vector<int> b256 = best;
            trial(b256[0], b256[1], b256[2], 512, b256[5], st);
            if (st != MPM_OK) return st;
        }
        // one cooperative launch per substep at the best so far
        {
            const std::vector<int> b = best;
            ctx->persistent = 1;
            trial(b[0], b[1], b[2], b[3], 0, st);
            ctx->persistent = 0;
            if (st != MPM_OK) return st;
        }
        rep += "]";
        // restore the state the caller had
        if (ctx->B != saved[0] && (st = set_block(ctx, saved[0])) != MPM_OK) return st;
        ctx->CH = saved[1];
        ctx->sort_every = saved[2];
        ctx->nt = saved[3];
        ctx->persistent = saved[4];
        ctx->fuse = saved[5];
        if ((st = mpm_set_state(ctx, -1, sx, sv, sC, sF, 1)) != MPM_OK) return st;
        if (!ctx->h_cols.empty())
            HIPCHK(hipMemcpyAsync(ctx->d_cols, ts.csnap, sizeof(ColliderDev) * ctx->h_cols.size(),
                                  hipMemcpyDeviceToDevice, ctx->stream));
        HIPCHK(hipMemcpyAsync(ctx->d_wrench, wsnap.data(), sizeof(float) * wsnap.size(), hipMemcpyHostToDevice,
                              ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        ctx->timing = saved_timing;
        ctx->graph = saved_graph;
        g_tune_cache[key] = best;
        tune_file_store(path, key, best);
    }
    mpm_status st;
    if (best[0] != ctx->B && (st = set_block(ctx, best[0])) != MPM_OK) return st;
    ctx->CH = best[1];
    ctx->sort_every = best[2];
    ctx->nt = best[3];
    ctx->persistent = best[4];
    ctx->fuse = best[5];
    ctx->since_sort = 1 << 30;
    clear_graphs(ctx);
    char buf[256];
    std::snprintf(buf, sizeof buf,
                  ", \"key\": \"%s\", \"best\": {\"block\": %d, \"chunk\": %d, \"sort_every\": %d, \"wg\": %d, "
                  "\"persistent\": %d, \"fuse\": %d}}",
                  key.c_str(), best[0], best[1], best[2], best[3], best[4], best[5]);
    rep += buf;
    if (report && report_len) {
        std::strncpy(report, rep.c_str(), report_len - 1);
        report[report_len - 1] = 0;
    }
    return MPM_OK;
}

}  // extern "C"
