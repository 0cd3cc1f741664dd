// Launch interface of the HIP kernels (internal, host side).
#pragma once
#include <hip/hip_runtime.h>
#include "mpm_types.hpp"

namespace mpm {

// Everything a substep kernel needs, passed by value.
struct StepArgs {
    const SceneDev *scenes;
    int n_scenes;
    float *P;                 // current particle buffer: component c at P + c * pstride
    long long pstride;
    float *gm, *gpx, *gpy, *gpz;   // grid mass / momentum (zero between substeps)
    float *gvx, *gvy, *gvz;        // grid velocity
    float *cap;               // optional capture of (m, p) per scene, dense [res^3] x 4, or null
    const long long *cap_off; // per scene offset into cap (in nodes)
    const ColliderDev *cols;
    void *colnow;             // per collider: pose at the current substep (ColliderNow), left by the grid update
    Lists L;
    int *flags;               // per scene
    int substep;              // substep index within the current call
    int B;                    // block edge
    const int *active;        // per scene: 0 = leave this scene's particles as they are (P2G / G2P skip it)
    float *dense;             // optional grid-update output per scene on the surrogate box [box][4] = (m, v), or null
    float *feat;              // optional surrogate input channels 0-3 (m, p normalised) [box][cf], or null
    int cf;
    int keep_bound;           // 1: a P2G with no G2P after it (leave the per-item scatter bounds as they are)
    const int *sur_org;       // surrogate box of scene s: origin sur_org[3 s ..] (device), size sur_box;
    int sur_box[3];           //   null = the whole grid (res^3 per scene, offset cap_off[s])
    float *out_mass;          // per scene: P2G mass the grid update found outside the box (added), or null
    const float *sdf;         // samples of the SDF-volume colliders (ColliderNow::sdf_off into it)
    int contact;              // 0 grid-node projection, 1 particle penalty (in G2P), 2 both
    float *wrench;            // per collider (global index): [6] impulse and angular impulse about its centre
                              //   received from the material, summed over grid updates (or null)
    int nt;                   // threads per workgroup of P2G and G2P: 256 or 512
    int chain;                // 1: a P2G that starts a run of fused substeps (keeps the scatter bounds, stores
                              //   the per-cell count it takes for the fused G2P's scale)
};


struct SortArgs {
    const SceneDev *scenes;
    int n_scenes;
    const int *psc;           // scene of each particle slot
    const float *P;           // current buffer
    float *Pn;                // other buffer
    long long pstride;
    int N;                    // particle slots in use
    int T;                    // bins in total
    const int *scene_bin_off; // [n_scenes + 1]
    unsigned *keys;           // [N]
    int *count;               // [T] (zero on entry, zero again after scatter)
    int *pstart;              // [T]
    int *perm;                // [N]
    int *perm2;               // [N] perm with every item in bank order (k_gather reads this)
    int3 *tsum;               // per scan tile
    unsigned char *dil;       // [T] 1 = grid block of the dilated particle set (by linear block)
    Lists L;
    int B;
    int CH;                   // max particles per item
};

hipError_t launch_sort(const SortArgs &a, hipStream_t st);
// The next P2G / grid / G2P / G2P2G launch on this thread records start and
// stop into these events at the kernel's own start and end.
void time_next_launch(hipEvent_t start, hipEvent_t stop);
hipError_t launch_p2g(const StepArgs &a, int chunk, int n_wg, hipStream_t st);
hipError_t launch_grid(const StepArgs &a, int n_wg, hipStream_t st);
hipError_t launch_g2p(const StepArgs &a, int n_wg, hipStream_t st);
// G2P of substep a.substep and P2G of substep a.substep + 1 in one launch.
hipError_t launch_g2p2g(const StepArgs &a, int n_wg, hipStream_t st);
// One cooperative launch per substep (P2G, grid update, G2P separated by
// grid-wide barriers); cus = compute units of the device, per_cu_cap = most
// workgroups per CU to launch (fewer than fit when the work is small).
hipError_t launch_persistent(const StepArgs &a, int cus, int per_cu_cap, hipStream_t st);
hipError_t launch_collider_advance(ColliderDev *cols, int n_cols, const int *col_scene, const SceneDev *scenes,
                                   int n_substeps, hipStream_t st);

// Boundary conversions (creation order <-> sorted SoA).
// Bytes of one collider's per-substep pose record (the device array a.colnow).
size_t collider_now_bytes();
// Collider wrenches out as [n_scenes][max_col][6] (zero past a scene's colliders), accumulators cleared.
hipError_t launch_wrench_out(const SceneDev *scenes, int n_scenes, int max_col, float *acc, float *out, hipStream_t st);
hipError_t launch_init_particles(const SceneDev *scenes, int n_scenes, const int *psc, float *P, long long pstride,
                                 const float *x, const float *v, const float *C, const float *F, int begin, int end,
                                 int *flags, hipStream_t st);
hipError_t launch_get_state(const SceneDev *scenes, const int *psc, const float *P, long long pstride, int begin,
                            int end, float *x, float *v, float *C, float *F, hipStream_t st);
hipError_t launch_clear_f(float *p, long long n, hipStream_t st);
hipError_t launch_fill_i(int *p, long long n, int v, hipStream_t st);

// Grid surrogate support (all scenes share one resolution `res`).
hipError_t launch_colliders_now(const StepArgs &a, int n_cols, const int *col_scene, hipStream_t st);
hipError_t launch_sur_init(const StepArgs &a, int res, float *feat, int cf, float *grid0, hipStream_t st);
hipError_t launch_sur_bbox(const StepArgs &a, int res, int *box, hipStream_t st);
hipError_t launch_sur_advance(const StepArgs &a, const float *grid0, const float *pred, int cp, int n_sub, int n_wg,
                              hipStream_t st);
hipError_t launch_sur_residual(const StepArgs &a, int res, const float *grid0, const float *pred, int cp,
                               const float *gend, float *acc, hipStream_t st);
hipError_t launch_sur_decide(const StepArgs &a, const float *acc, int n_sub, float threshold, int fallback,
                             float *residual, int *active, int *n_fallback, hipStream_t st);
hipError_t launch_sur_restore(const float *Psnap, float *P, long long pstride, const int *psc, const int *active, int N,
                              hipStream_t st);
hipError_t launch_sur_targets(const StepArgs &a, int res, const float *g0, const float *g1, int ct, float *target,
                              float *mask, hipStream_t st);

}  // namespace mpm
