// Surrogate support kernels (gfx950): the grid input of the network, the
// particle advance over one control step from a grid prediction, the
// re-splat residual, the per-scene fallback decision and restore, and the
// training targets.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "mpm_device.hpp"

namespace mpm {

// ====================================================================== grid surrogate
// A learned grid model stands in for one control step of n_sub substeps.
// Its input at every node is (m, p) from a P2G of the current state, the
// distance to the nearest collider and that collider's velocity; its output
// is the change of the node mass and of the P2G velocity p / m over the
// control step.  The particles then advance with the mean of the start and
// end grid velocities, add the predicted change to their velocity and APIC
// matrix, and a P2G of the advanced particles checks the prediction
// (residual gate).

// Collider poses of every scene at substep a.substep (for the dense pass).
__global__ void k_colliders_now(StepArgs a, int n_cols, const int *col_scene)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cols) return;
    ColliderNow cn;
    collider_at(a.cols[c], (float)a.substep * a.scenes[col_scene[c]].dt, cn);
    ((ColliderNow *)a.colnow)[c] = cn;
}

hipError_t launch_colliders_now(const StepArgs &a, int n_cols, const int *col_scene, hipStream_t st)
{
    if (n_cols > 0) k_colliders_now<<<(n_cols + 63) / 64, 64, 0, st>>>(a, n_cols, col_scene);
    return hipGetLastError();
}

// Every node of every scene's surrogate box (the whole grid without a box):
// collider channels of the input (4: clipped distance to the nearest
// collider in cells, 5-7: that collider's velocity at the node where it is
// closer than 3 cells), zeros in channels 0-3 (the grid update fills the
// nodes that receive mass) and above 7, and a zero start grid.
__global__ __launch_bounds__(WG) void k_sur_init(StepArgs a, int res, float *feat, int cf, float *grid0)
{
    const int D = a.sur_org ? a.sur_box[0] : res, H = a.sur_org ? a.sur_box[1] : res, W = a.sur_org ? a.sur_box[2] : res;
    const long long per = (long long)D * H * W, total = per * a.n_scenes;
    for (long long e = (long long)blockIdx.x * WG + threadIdx.x; e < total; e += (long long)gridDim.x * WG) {
        const int s = (int)(e / per);
        const long long c = e - (long long)s * per;
        const SceneDev &S = a.scenes[s];
        int i = (int)(c / ((long long)H * W)), j = (int)((c / W) % H), k = (int)(c % W);
        if (a.sur_org) {
            i += a.sur_org[3 * s];
            j += a.sur_org[3 * s + 1];
            k += a.sur_org[3 * s + 2];
        }
        const float xi[3] = {i * S.dx, j * S.dx, k * S.dx};
        float phi_min = 3.0f * S.dx, vel[3] = {0.0f, 0.0f, 0.0f};
        const ColliderNow *cn = (const ColliderNow *)a.colnow + S.col_off;
        for (int q = 0; q < S.n_col; q++) {
            float n[3];
            const float phi = sdf_eval(cn[q], xi, n, a.sdf);
            if (phi < phi_min) {
                phi_min = phi;
                const float r[3] = {xi[0] - cn[q].c[0], xi[1] - cn[q].c[1], xi[2] - cn[q].c[2]};
                vel[0] = cn[q].v[0] + (cn[q].w[1] * r[2] - cn[q].w[2] * r[1]);
                vel[1] = cn[q].v[1] + (cn[q].w[2] * r[0] - cn[q].w[0] * r[2]);
                vel[2] = cn[q].v[2] + (cn[q].w[0] * r[1] - cn[q].w[1] * r[0]);
            }
        }
        float *fp = feat + e * cf;
        fp[0] = 0.0f;
        fp[1] = 0.0f;
        fp[2] = 0.0f;
        fp[3] = 0.0f;
        fp[4] = fminf(fmaxf(phi_min * S.inv_dx, -3.0f), 3.0f);
        for (int d = 0; d < 3; d++) fp[5 + d] = vel[d] * (1.0f / SUR_VEL);
        for (int q = 8; q < cf; q++) fp[q] = 0.0f;
        *(float4 *)(grid0 + 4 * e) = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
}

hipError_t launch_sur_init(const StepArgs &a, int res, float *feat, int cf, float *grid0, hipStream_t st)
{
    const long long per = a.sur_org ? (long long)a.sur_box[0] * a.sur_box[1] * a.sur_box[2] : (long long)res * res * res;
    const long long nb = (per * a.n_scenes + WG - 1) / WG;
    if (nb > 0) k_sur_init<<<(unsigned)(nb < 16384 ? nb : 16384), WG, 0, st>>>(a, res, feat, cf, grid0);
    return hipGetLastError();
}

// Per scene, the box of grid nodes the particles' P2G stencils reach (base
// node .. base + 2 on each axis): box[6 s ..] = (lo i, j, k, hi i, j, k),
// inclusive; all zero for a scene without particles.  Workgroup (x, s) takes
// a stride of scene s's particles.
__global__ __launch_bounds__(WG) void k_sur_bbox(StepArgs a, int *box)
{
    __shared__ int red[6][WG / 64];
    const int s = blockIdx.y;
    const SceneDev &S = a.scenes[s];
    const SceneK K = scene_k(S);
    int lo[3] = {K.res, K.res, K.res}, hi[3] = {-1, -1, -1};
    for (int p = S.p_begin + blockIdx.x * WG + threadIdx.x; p < S.p_end; p += gridDim.x * WG) {
        int cl = 0;
        for (int d = 0; d < 3; d++) {
            int b;
            float f;
            particle_base(K, a.P[(long long)(X0 + d) * a.pstride + p], b, f, cl);
            lo[d] = min(lo[d], b);
            hi[d] = max(hi[d], b + 2);
        }
    }
    for (int d = 0; d < 3; d++)
        for (int o = 32; o > 0; o >>= 1) {
            lo[d] = min(lo[d], __shfl_xor(lo[d], o, 64));
            hi[d] = max(hi[d], __shfl_xor(hi[d], o, 64));
        }
    if ((threadIdx.x & 63) == 0)
        for (int d = 0; d < 3; d++) {
            red[d][threadIdx.x >> 6] = lo[d];
            red[3 + d][threadIdx.x >> 6] = hi[d];
        }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int d = threadIdx.x;
        int l = red[d][0], h = red[3 + d][0];
        for (int w = 1; w < WG / 64; w++) {
            l = min(l, red[d][w]);
            h = max(h, red[3 + d][w]);
        }
        if (h >= 0) {
            atomicMin(box + 6 * s + d, l);
            atomicMax(box + 6 * s + 3 + d, h);
        }
    }
}

// Empty scenes (no particle reached the reduction) get an all-zero box.
__global__ void k_sur_bbox_final(int n, int *box)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    if (box[6 * s + 3] < 0)
        for (int d = 0; d < 6; d++) box[6 * s + d] = 0;
}

__global__ void k_sur_bbox_init(int n, int res, int *box)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < 6 * n) box[e] = (e % 6) < 3 ? res : -1;
}

hipError_t launch_sur_bbox(const StepArgs &a, int res, int *box, hipStream_t st)
{
    if (a.n_scenes <= 0) return hipSuccess;
    k_sur_bbox_init<<<(6 * a.n_scenes + 255) / 256, 256, 0, st>>>(a.n_scenes, res, box);
    k_sur_bbox<<<dim3(16, a.n_scenes), WG, 0, st>>>(a, box);
    k_sur_bbox_final<<<(a.n_scenes + 63) / 64, 64, 0, st>>>(a.n_scenes, box);
    return hipGetLastError();
}

// Start and predicted end velocity of one node (dense scene-major index c).
__device__ __forceinline__ void sur_node(const float *grid0, const float *pred, int cp, long long c, float vs[3],
                                         float dv[3])
{
    const float4 g = *(const float4 *)(grid0 + 4 * c);
    const float4 p = *(const float4 *)(pred + c * cp);
    vs[0] = g.y;
    vs[1] = g.z;
    vs[2] = g.w;
    dv[0] = p.x * SUR_VEL;
    dv[1] = p.y * SUR_VEL;
    dv[2] = p.z * SUR_VEL;
}

// Advance the particles of one item over the control step from the predicted
// grid: x += T v_mid, F <- (I + T C_mid) F (+ return map), v += the change
// interpolated to the particle, C += its APIC gradient, and the affine
// momentum A for the next substep's P2G (the stored A = m C - k tau(F) takes
// m dC and the change of the stress term).
template <int B>
__device__ void sur_advance_item(const StepArgs &a, int it, const Item &item, float *vt, const float *grid0,
                                 const float *pred, int cp, int n_sub)
{
    constexpr int T = B + 4, T3 = T * T * T;
    const int t = threadIdx.x;
    const int s = item.scene;
    const SceneDev &S = a.scenes[s];
    const int nb = S.nb;
    const int bx = item.block / (nb * nb), by = (item.block / nb) % nb, bz = item.block % nb;
    const int org[3] = {bx * B - 1, by * B - 1, bz * B - 1};
    for (int n = t; n < T3; n += WG) {
        const int gi = org[0] + n / (T * T), gj = org[1] + (n / T) % T, gk = org[2] + n % T;
        float vs[3] = {0.0f, 0.0f, 0.0f}, dv[3] = {0.0f, 0.0f, 0.0f};
        if (gi >= 0 && gj >= 0 && gk >= 0 && gi < S.res && gj < S.res && gk < S.res) {
            const long long c = sur_index(a, s, S.res, gi, gj, gk);
            if (c >= 0) sur_node(grid0, pred, cp, c, vs, dv);   // outside the box: no material, no change
        }
        for (int d = 0; d < 3; d++) {
            vt[d * T3 + n] = fmaf(0.5f, dv[d], vs[d]);
            vt[(3 + d) * T3 + n] = dv[d];
        }
    }
    __syncthreads();
    const Material mat = material_of(S);
    const SceneK K = scene_k(S);
    const long long ps = a.pstride;
    const float Tb = (float)n_sub * K.dt;
    const float Dd = 4.0f * K.inv_dx;
    int bad_any = 0, cl_any = 0;
    float bnd = 0.0f;
    for (int li = t; li < item.count; li += WG) {
        const unsigned jo = (unsigned)(item.start + li) << 2;
        float x[3], G[9], v[3], A[9];
        for (int d = 0; d < 3; d++) x[d] = pload(a.P, ps, X0 + d, jo);
        for (int d = 0; d < 3; d++) v[d] = pload(a.P, ps, V0 + d, jo);
        for (int e = 0; e < 9; e++) A[e] = pload(a.P, ps, A00 + e, jo);
        for (int e = 0; e < 9; e++) G[e] = pload(a.P, ps, G00 + e, jo);
        int b[3], cl = 0, in = 1;
        float f[3];
        for (int d = 0; d < 3; d++) {
            particle_base(K, x[d], b[d], f[d], cl);
            const int tb = b[d] - org[d];
            in &= (tb >= 0) & (tb <= B + 1);
        }
        cl_any |= cl;
        float w[3][3];
        for (int d = 0; d < 3; d++) bspline_w(f[d], w[d]);
        float vm[3] = {0.0f, 0.0f, 0.0f}, ve[3] = {0.0f, 0.0f, 0.0f};
        float Sm[3][3] = {{0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}};
        float Se[3][3] = {{0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}};
        for (int ox = 0; ox < 3; ox++)
            for (int oy = 0; oy < 3; oy++)
                for (int oz = 0; oz < 3; oz++) {
                    const float wt = w[0][ox] * w[1][oy] * w[2][oz];
                    float um[3], ue[3];
                    if (in) {
                        const int n = ((b[0] - org[0] + ox) * T + (b[1] - org[1] + oy)) * T + (b[2] - org[2] + oz);
                        for (int d = 0; d < 3; d++) {
                            um[d] = vt[d * T3 + n];
                            ue[d] = vt[(3 + d) * T3 + n];
                        }
                    } else {
                        float vs[3] = {0.0f, 0.0f, 0.0f}, dv[3] = {0.0f, 0.0f, 0.0f};
                        const long long c = sur_index(a, s, K.res, b[0] + ox, b[1] + oy, b[2] + oz);
                        if (c >= 0) sur_node(grid0, pred, cp, c, vs, dv);
                        for (int d = 0; d < 3; d++) {
                            um[d] = fmaf(0.5f, dv[d], vs[d]);
                            ue[d] = dv[d];
                        }
                    }
                    const float o[3] = {(float)ox, (float)oy, (float)oz};
                    for (int c = 0; c < 3; c++) {
                        vm[c] = fmaf(wt, um[c], vm[c]);
                        ve[c] = fmaf(wt, ue[c], ve[c]);
                        for (int e = 0; e < 3; e++) {
                            Sm[c][e] = fmaf(wt * o[e], um[c], Sm[c][e]);
                            Se[c][e] = fmaf(wt * o[e], ue[c], Se[c][e]);
                        }
                    }
                }
        // C = (4/dx^2) sum w v (x_i - x_p)^T = (4/dx) (S - v f^T); "e" sums hold the change
        float Cm[9], Ce[9];
        for (int c = 0; c < 3; c++)
            for (int e = 0; e < 3; e++) {
                Cm[3 * c + e] = Dd * fmaf(-vm[c], f[e], Sm[c][e]);
                Ce[3 * c + e] = Dd * fmaf(-ve[c], f[e], Se[c][e]);
            }
        for (int d = 0; d < 3; d++) x[d] = fmaf(Tb, vm[d], x[d]);
        float Gt[9];
        for (int i = 0; i < 3; i++)
            for (int k = 0; k < 3; k++) {
                float acc = Cm[3 * i + k];
                for (int e = 0; e < 3; e++) acc = fmaf(Cm[3 * i + e], G[3 * e + k], acc);
                Gt[3 * i + k] = fmaf(Tb, acc, G[3 * i + k]);
            }
        // stress of the start F (the stored A holds m C - k tau(F))
        float tau0[9];
        int bad = 0;
        stress_of(G, mat, tau0, bad);
        float tau[9], Gn[9];
        if (mat.model == 0) {
            tau_neo_hookean(Gt, mat.mu, mat.la, tau, bad);
            for (int e = 0; e < 9; e++) Gn[e] = Gt[e];
        } else if (mat.model == 2) {
            fluid_update(Gt, mat, Gn, tau, bad);
        } else {
            hencky_update(Gt, mat, Gn, tau, bad);
        }
        bad |= !(isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]));
        bad_any |= bad;
        float vn[3];
        for (int d = 0; d < 3; d++) {
            vn[d] = v[d] + ve[d];
            pstore(a.P, ps, X0 + d, jo, x[d]);
            pstore(a.P, ps, V0 + d, jo, vn[d]);
        }
        float An[9];
        for (int e = 0; e < 9; e++) {
            // m (C + dC) - k tau(F_new) = A + k (tau(F) - tau(F_new)) + m dC
            An[e] = fmaf(K.mass, Ce[e], fmaf(K.kstress, tau0[e] - tau[e], A[e]));
            pstore(a.P, ps, A00 + e, jo, An[e]);
            pstore(a.P, ps, G00 + e, jo, Gn[e]);
        }
        // a non-finite v or A: flagged, so that the scene falls back
        const float sb = scatter_bound(K.mass, K.dx, vn, An);
        bad_any |= !(sb <= 3.0e38f);
        bnd = fmaxf(bnd, sb);
    }
    bnd = wave_max(bnd);
    if ((t & 63) == 0 && bnd > 0.0f) atomicMax((int *)(a.L.ibound + it), __float_as_int(bnd));
    if (t == 0) a.L.icell[it] = 0;   // the particles moved a whole control step: the next P2G counts
    if (bad_any) atomicOr(a.flags + s, (int)FLAG_NONFINITE);
    if (cl_any) atomicOr(a.flags + s, (int)FLAG_CLAMPED);
    __syncthreads();
}

template <int B>
__global__ __launch_bounds__(WG) void k_sur_advance(StepArgs a, const float *grid0, const float *pred, int cp, int n_sub)
{
    constexpr int T = B + 4, T3 = T * T * T;
    __shared__ float vt[6 * T3];
    const int n_items = *a.L.n_items;
    const int G = active_wgs(n_items);
    if ((int)blockIdx.x >= G) return;
    for (int it = xcd_remap(blockIdx.x, G); it < n_items; it += G) {
        const Item item = a.L.items[it];
        sur_advance_item<B>(a, it, item, vt, grid0, pred, cp, n_sub);
    }
}

hipError_t launch_sur_advance(const StepArgs &a, const float *grid0, const float *pred, int cp, int n_sub, int n_wg,
                              hipStream_t st)
{
    n_wg = (n_wg + 7) & ~7;
    if (a.B == 4) k_sur_advance<4><<<n_wg, WG, 0, st>>>(a, grid0, pred, cp, n_sub);
    else k_sur_advance<8><<<n_wg, WG, 0, st>>>(a, grid0, pred, cp, n_sub);
    return hipGetLastError();
}

// Per-scene sums over the nodes of one block of 4096 nodes (all in one scene)
// that hold material at the start or after the re-splat:
// acc[s] += (sum |m_r - m_pred|, sum |m_r v_r - m_pred v_pred|_1, sum m_start,
// sum |m_start v_start|_1), with (m_r, v_r) the re-splat of the advanced
// particles and m_pred = m_start + dm, v_pred = v_start + dv the prediction.
static constexpr int RES_CHUNK = 4096;

__global__ __launch_bounds__(WG) void k_sur_residual(StepArgs a, int res, const float *grid0, const float *pred, int cp,
                                                     const float *gend, float *acc)
{
    __shared__ float red[4][WG / 64];
    const int s = blockIdx.y;
    const long long per = a.sur_org ? (long long)a.sur_box[0] * a.sur_box[1] * a.sur_box[2] : (long long)res * res * res;
    const long long base = a.sur_org ? (long long)s * per : a.cap_off[s];
    const long long l0 = (long long)blockIdx.x * RES_CHUNK, l1 = min(per, l0 + RES_CHUNK);
    const SceneDev &S = a.scenes[s];
    const float mu = S.mass / S.vol * S.dx * S.dx * S.dx * SUR_DM;   // mass unit of the prediction
    float sm = 0.0f, sp = 0.0f, m0 = 0.0f, p0 = 0.0f;
    for (long long l = l0 + threadIdx.x; l < l1; l += WG) {
        const long long c = base + l;
        const float4 g = *(const float4 *)(grid0 + 4 * c);
        const float4 r = *(const float4 *)(gend + 4 * c);
        if (g.x == 0.0f && r.x == 0.0f) continue;   // no material at this node before or after
        const float4 p = *(const float4 *)(pred + c * cp);
        const float mp = fmaf(p.w, mu, g.x);
        const float ve[3] = {fmaf(p.x, SUR_VEL, g.y), fmaf(p.y, SUR_VEL, g.z), fmaf(p.z, SUR_VEL, g.w)};
        sm += fabsf(r.x - mp);
        sp += fabsf(r.x * r.y - mp * ve[0]) + fabsf(r.x * r.z - mp * ve[1]) + fabsf(r.x * r.w - mp * ve[2]);
        m0 += g.x;
        p0 += g.x * (fabsf(g.y) + fabsf(g.z) + fabsf(g.w));
    }
    // re-splat mass outside the box has no prediction to match: all of it is mismatch
    if (blockIdx.x == 0 && threadIdx.x == 0 && a.out_mass) sm += a.out_mass[s];
    float v4[4] = {sm, sp, m0, p0};
    for (int k = 0; k < 4; k++) {
        float v = v4[k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0) red[k][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        float v = 0.0f;
        for (int w = 0; w < WG / 64; w++) v += red[threadIdx.x][w];
        atomicAdd(acc + 4 * s + threadIdx.x, v);
    }
}

hipError_t launch_sur_residual(const StepArgs &a, int res, const float *grid0, const float *pred, int cp,
                               const float *gend, float *acc, hipStream_t st)
{
    const long long per = a.sur_org ? (long long)a.sur_box[0] * a.sur_box[1] * a.sur_box[2] : (long long)res * res * res;
    const long long nb = (per + RES_CHUNK - 1) / RES_CHUNK;
    if (a.n_scenes > 0 && nb > 0) k_sur_residual<<<dim3((unsigned)nb, a.n_scenes), WG, 0, st>>>(a, res, grid0, pred, cp, gend, acc);
    return hipGetLastError();
}

// Residual per scene r = max(sum|dm| / sum m, sum|dp| / (sum m u_ref)), with
// u_ref = SUR_ERR_BAR dx / T the speed that crosses the per-block error bar in
// one control step, and the fallback decision r > threshold (a non-finite r
// falls back too).
__global__ void k_sur_decide(StepArgs a, const float *acc, int n_sub, float threshold, int fallback, float *residual,
                             int *active, int *n_fallback)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.n_scenes) return;
    const SceneDev &S = a.scenes[s];
    const float *q = acc + 4 * s;
    float r = 0.0f;
    if (q[2] > 0.0f) {
        const float u_ref = SUR_ERR_BAR * S.dx / ((float)n_sub * S.dt);
        r = fmaxf(q[0] / q[2], q[1] / (q[2] * u_ref));
    }
    if (!isfinite(r) || (a.flags[s] & FLAG_NONFINITE)) r = INFINITY;
    if (residual) residual[s] = r;
    const int fb = !(r <= threshold);
    active[s] = fallback ? fb : 0;
    if (fb && n_fallback) atomicAdd(n_fallback, 1);
}

hipError_t launch_sur_decide(const StepArgs &a, const float *acc, int n_sub, float threshold, int fallback,
                             float *residual, int *active, int *n_fallback, hipStream_t st)
{
    k_sur_decide<<<(a.n_scenes + 63) / 64, 64, 0, st>>>(a, acc, n_sub, threshold, fallback, residual, active, n_fallback);
    return hipGetLastError();
}

// Particles of the scenes marked active get their snapshot back.
__global__ __launch_bounds__(WG) void k_sur_restore(const float *Psnap, float *P, long long ps, const int *psc,
                                                    const int *active, int N)
{
    for (long long j = (long long)blockIdx.x * WG + threadIdx.x; j < N; j += (long long)gridDim.x * WG) {
        if (!active[psc[j]]) continue;
        for (int c = 0; c < NCOMP; c++) P[c * ps + j] = Psnap[c * ps + j];
    }
}

hipError_t launch_sur_restore(const float *Psnap, float *P, long long pstride, const int *psc, const int *active, int N,
                              hipStream_t st)
{
    if (N > 0) {
        const long long nb = (N + WG - 1) / WG;
        k_sur_restore<<<(unsigned)(nb < 8192 ? nb : 8192), WG, 0, st>>>(Psnap, P, pstride, psc, active, N);
    }
    return hipGetLastError();
}

// Training targets from the start grids of two consecutive control steps:
// target = ((v1 - v0) / vel unit, (m1 - m0) / mass-change unit), and a loss
// weight mask = min(1, max(m0, m1) / (rho dx^3)) where m0 > 0 or m1 > 0, else 0
// (the node's share of a filled cell's mass: the residual gate weighs
// velocity errors by mass).
__global__ __launch_bounds__(WG) void k_sur_targets(StepArgs a, int res, const float *g0, const float *g1, int ct,
                                                    float *target, float *mask)
{
    const long long R3 = (long long)res * res * res, total = R3 * a.n_scenes;
    for (long long e = (long long)blockIdx.x * WG + threadIdx.x; e < total; e += (long long)gridDim.x * WG) {
        const SceneDev &S = a.scenes[e / R3];
        const float inv_mu = S.vol / (S.mass * S.dx * S.dx * S.dx * SUR_DM);
        const float4 u = *(const float4 *)(g0 + 4 * e);
        const float4 w = *(const float4 *)(g1 + 4 * e);
        float *tp = target + e * ct;
        tp[0] = (w.y - u.y) * (1.0f / SUR_VEL);
        tp[1] = (w.z - u.z) * (1.0f / SUR_VEL);
        tp[2] = (w.w - u.w) * (1.0f / SUR_VEL);
        tp[3] = (w.x - u.x) * inv_mu;
        const float mfill = fmaxf(u.x, w.x) * (S.vol / (S.mass * S.dx * S.dx * S.dx));
        mask[e] = (u.x > 0.0f || w.x > 0.0f) ? fmaxf(fminf(mfill, 1.0f), 1e-30f) : 0.0f;
    }
}

hipError_t launch_sur_targets(const StepArgs &a, int res, const float *g0, const float *g1, int ct, float *target,
                              float *mask, hipStream_t st)
{
    const long long total = (long long)res * res * res * a.n_scenes;
    const long long nb = (total + WG - 1) / WG;
    k_sur_targets<<<(unsigned)(nb < 16384 ? nb : 16384), WG, 0, st>>>(a, res, g0, g1, ct, target, mask);
    return hipGetLastError();
}

}  // namespace mpm
