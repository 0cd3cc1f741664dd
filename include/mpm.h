/*
 * mpm.h -- C ABI of the MI355X MLS-MPM soft-body library (libmpm_hip.so).
 *
 * The calls follow the paper's statement of the soft-body problem
 * (Sec. 3 "Rigid-soft Coupling" and Algorithm 1 in App. D.1):
 *   - create a soft scene and copy the rigid collision shapes into it
 *     (Algorithm 1: "copy rigid body shapes ... to soft scene")      -> mpm_create
 *   - after each rigid step copy rigid poses and velocities into it
 *     (Sec. 3: poses and velocities are copied after each rigid step) -> mpm_set_colliders
 *   - run the soft steps: particle-to-grid, grid velocity, grid-to-particle,
 *     integrate (Algorithm 1, inner loop)                             -> mpm_step
 *   - hand particle positions to the consumer, ideally by one device-to-device
 *     copy (App. D.2)                                                  -> mpm_get_particles
 *   - read out the forces the soft body exerts on the rigid bodies
 *     (Algorithm 1 accumulates them for the rigid step)               -> mpm_get_collider_wrenches
 * The method of a substep is MLS-MPM with APIC transfers and quadratic
 * B-splines (Sec. 3 names MLS-MPM); colliders are analytic box / capsule
 * SDFs applied on grid nodes (Sec. 3: the grid-node variant the simulator
 * also supports), material is neo-Hookean or Hencky elasticity with a von
 * Mises return map (App. D.3, Table "tab:mpm_param": Young's modulus,
 * Poisson ratio, yield stress).
 *
 * Conventions shared by every call:
 *   - Every call returns mpm_status: 0 = MPM_OK, > 0 warning, < 0 error.
 *     No C++ exception crosses the ABI.  Arguments are validated before any
 *     device work is queued; on an argument error nothing is changed.
 *   - The context owns all device memory it allocates.  Pointers passed in
 *     are borrowed for the duration of the call only.
 *   - on_device = 1: pointers are device pointers on the context's device;
 *     copies are queued on the context stream and the call returns without
 *     waiting (synchronise that stream, or call mpm_sync, before reading).
 *     on_device = 0: pointers are host pointers; the call blocks until the
 *     copy is complete.
 *   - Layout at the ABI: positions / velocities [n][3] row-major float32,
 *     matrices [n][3][3] row-major float32, particles in the order they were
 *     given to mpm_create (scenes concatenated).  The library keeps its own
 *     sorted SoA layout internally.
 *   - World: grid node (i, j, k) sits at (i dx, j dx, k dx), i, j, k in
 *     [0, res); y is up.  Dense grid outputs are [res][res][res] with x
 *     slowest (index (i * res + j) * res + k).
 *   - Threading: a context is used by one host thread at a time.
 */
#ifndef MPM_H
#define MPM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mpm_ctx_s *mpm_ctx;

typedef enum {
    MPM_OK = 0,
    MPM_WARN_CLAMPED = 1,     /* a particle stencil touched the grid edge and was clamped */
    MPM_WARN_FALLBACK = 2,    /* mpm_step_blocks: at least one scene fell back to the plain substeps */
    MPM_ERR_ARG = -1,         /* invalid argument; nothing was changed */
    MPM_ERR_HIP = -2,         /* HIP runtime error; detail via mpm_last_error */
    MPM_ERR_OOM = -3,         /* device allocation failed */
    MPM_ERR_NONFINITE = -4,   /* NaN / Inf found in the particle state */
    MPM_ERR_STATE = -5        /* call not valid in the current state */
} mpm_status;

/* Materials (App. D.3 gives E, nu and the yield stress of the elastoplastic
 * bodies; the liquid of the Pour task (Sec. 2.1 "Heterogeneous Task Families",
 * and the soft-body task table of the appendix) has no printed law):
 *   MPM_NEO_HOOKEAN           tau = mu (F F^T - I) + lambda ln(J) I
 *   MPM_HENCKY_VON_MISES      Hencky elasticity, von Mises return map on the
 *                             principal log strain (yield_stress, yield_form)
 *   MPM_WEAKLY_COMPRESSIBLE_FLUID
 *                             tau = -J p(J) I, p(J) = (K / 7) (J^-7 - 1),
 *                             K = lambda + 2 mu / 3 from (E, nu); F is kept as
 *                             J^(1/3) I (volume change only, no shear) */
typedef enum { MPM_NEO_HOOKEAN = 0, MPM_HENCKY_VON_MISES = 1, MPM_WEAKLY_COMPRESSIBLE_FLUID = 2 } mpm_model;
typedef enum { MPM_BOX = 0, MPM_CAPSULE = 1, MPM_SDF_VOLUME = 2 } mpm_shape_type;

typedef struct {
    int model;             /* mpm_model */
    float E;               /* Young's modulus, Pa (> 0) */
    float nu;              /* Poisson ratio, in (-1, 0.5) */
    float rho;             /* density, kg/m^3 (> 0) */
    float yield_stress;    /* Pa; <= 0 or +inf disables plasticity (Hencky only) */
    int yield_form;        /* 0: |dev eps| <= sy/(2 mu); 1: sqrt(2/3) sy/(2 mu) */
} mpm_material;

typedef struct {
    int type;              /* mpm_shape_type */
    float half_extents[3]; /* box half sizes, body frame */
    float radius;          /* capsule radius */
    float half_length;     /* capsule half segment length along body y */
    float friction;        /* Coulomb coefficient >= 0; +inf = sticky */
    /* MPM_SDF_VOLUME: a mesh collider as a sampled signed distance (the paper
     * keeps mesh SDFs as 3D textures, Sec. 3): host samples [nx][ny][nz] of
     * the body-frame distance at sdf_origin + (i, j, k) sdf_cell, copied by
     * mpm_create.  The distance is their trilinear interpolant, the normal its
     * normalised gradient; outside the sampled box there is no contact, so
     * the brick must enclose the surface.  Each dimension >= 2, sdf_cell > 0,
     * samples finite.  Ignored by the other types (may be NULL / 0). */
    const float *sdf;
    int sdf_dims[3];
    float sdf_cell;
    float sdf_origin[3];
} mpm_collider_shape;

typedef struct {
    int n_particles;                 /* >= 0 */
    const float *x;                  /* host [n][3]; inside [0, res dx)^3 */
    const float *v;                  /* host [n][3] or NULL (zero) */
    float particle_volume;           /* m^3 (> 0); particle mass = rho * volume */
    int res;                         /* grid nodes per axis: 16, 32, 64 or 128 */
    float dx;                        /* node spacing, m (> 0) */
    float dt;                        /* substep, s (> 0) */
    float gravity[3];                /* m/s^2 */
    int bound;                       /* wall thickness in nodes, 0 <= bound < res/2 */
    mpm_material mat;
    int n_colliders;                 /* 0 .. MPM_MAX_COLLIDERS */
    const mpm_collider_shape *colliders;
} mpm_scene_desc;

#define MPM_MAX_COLLIDERS 4

/* Create a context holding n_scenes independent scenes (one batch).  Copies
 * the scenes to the device (C = 0, F = I), sorts the particles and allocates
 * every buffer a substep needs.  hip_stream: a hipStream_t to run on (for
 * example PyTorch's current stream), or NULL to create one owned by the
 * context.  Collider poses start at the origin with identity orientation and
 * zero velocity until mpm_set_colliders is called.  On success *out holds
 * the new context; on error *out is NULL.  MPM_ERR_OOM when the device
 * cannot hold the state. */
mpm_status mpm_create(const mpm_scene_desc *scenes, int n_scenes, void *hip_stream, mpm_ctx *out);

/* Release every resource of the context (waits for queued work). NULL is a no-op. */
mpm_status mpm_destroy(mpm_ctx ctx);

/* Hand over collider poses and velocities (Sec. 3: copied after each rigid
 * step).  poses [n_scenes][max_colliders][7] = centre xyz, quaternion wxyz
 * (body -> world, normalised by the caller); velocities
 * [n_scenes][max_colliders][6] = linear xyz (m/s), angular xyz (rad/s,
 * world frame), where max_colliders = mpm_max_colliders(ctx).  Entries past a
 * scene's own collider count are ignored.  Within the following mpm_step
 * calls each collider moves kinematically: substep k of a call uses
 * c + k dt v and exp(k dt w / 2) (x) q, the start-of-substep pose. */
mpm_status mpm_set_colliders(mpm_ctx ctx, const float *poses, const float *velocities, int on_device);

/* Two-way coupling read-out (Algorithm 1 accumulates the soft body's forces
 * on the rigid bodies over the soft steps and applies them in the rigid
 * step).  With contact on grid nodes, the impulse collider k receives in a
 * substep is minus the momentum its projection gives the material,
 * -sum_i m_i (v_i after - v_i before) over the nodes it touches, and its
 * angular impulse about its own centre (at that substep's pose) is
 * -sum_i (x_i - c_k) x m_i (v_i after - v_i before); with particle penalty
 * contact (MPM_OPT_CONTACT 1 or 2) the particles inside it add -m_p dv_p and
 * -(x_p - c_k) x m_p dv_p in the same way.  out
 * [n_scenes][max_colliders][6] = impulse xyz (N s), angular impulse xyz
 * (N m s), summed over every substep since the previous call (or since
 * mpm_create); entries past a scene's own collider count are zero.  Divide
 * by the elapsed time (substeps x dt) for the mean force and torque.  The
 * call resets the sums.  Only plain substeps contribute (a control step the
 * surrogate takes adds nothing; its fallback substeps do); mpm_autotune
 * leaves the sums as they were.  The sums use floating-point atomics, so
 * their last bits vary from run to run. */
mpm_status mpm_get_collider_wrenches(mpm_ctx ctx, float *out, int on_device);

/* Run n_substeps >= 0 substeps of every scene (Algorithm 1, inner loop).
 * Queued on the context stream; returns without waiting.  Warnings and
 * non-finite errors found by earlier substeps are reported by mpm_sync. */
mpm_status mpm_step(mpm_ctx ctx, int n_substeps);

/* Wait for queued work; returns MPM_ERR_NONFINITE / MPM_WARN_CLAMPED if the
 * device flagged them since the last mpm_sync, else MPM_OK. */
mpm_status mpm_sync(mpm_ctx ctx);

/* Particle positions (and optionally velocities and deformation gradients)
 * of one scene, or of all scenes concatenated (scene = -1), in creation
 * order.  x: [n][3]; v: [n][3] or NULL; F: [n][3][3] or NULL. */
mpm_status mpm_get_particles(mpm_ctx ctx, int scene, float *x, float *v, float *F, int on_device);

/* Zero-copy view of the particle positions for a consumer on the same GPU (a
 * renderer: App. D.2 hands the particles over on the GPU rather than through
 * the host).  *x, *y, *z receive device pointers to the current x, y and z
 * coordinates in the library's internal order (sorted by grid block, not
 * creation order); scene s holds slots [slot_begin[s], slot_begin[s + 1])
 * when slot_begin (host, n_scenes + 1 ints) is not NULL.  Read-only, and
 * valid only until the next call that steps or changes the state (mpm_step,
 * mpm_sur_block, mpm_set_state, mpm_autotune): a re-sort moves the
 * particles to the other buffer.  Synchronise the context stream before
 * reading. */
mpm_status mpm_particle_view(mpm_ctx ctx, const float **x, const float **y, const float **z, int *slot_begin);

/* Full particle state (checkpoint / teacher forcing): x, v [n][3]; affine
 * velocity C and deformation gradient F [n][3][3] of one scene or all
 * (scene = -1).  mpm_set_state replaces that state (all four arrays are
 * required) and re-sorts the particles.  Host arrays with a non-finite x or
 * v are refused (MPM_ERR_ARG); any other non-finite value (device arrays,
 * C, F, or an F without a defined stress) is reported by the next
 * mpm_sync as MPM_ERR_NONFINITE. */
mpm_status mpm_get_state(mpm_ctx ctx, int scene, float *x, float *v, float *C, float *F, int on_device);
mpm_status mpm_set_state(mpm_ctx ctx, int scene, const float *x, const float *v, const float *C,
                         const float *F, int on_device);

/* Grid mass [res^3] and momentum [res^3][3] written by the particle-to-grid
 * transfer of the most recent substep of one scene, before the grid update.
 * Only available when capture is on (mpm_set_option(ctx, MPM_OPT_CAPTURE_GRID, 1)
 * before stepping); MPM_ERR_STATE otherwise. */
mpm_status mpm_get_grid(mpm_ctx ctx, int scene, float *m, float *p, int on_device);

/* Tuning and debugging options. */
typedef enum {
    MPM_OPT_SORT_EVERY = 0,     /* substeps between particle re-sorts (>= 1), default 25 */
    MPM_OPT_BLOCK = 1,          /* grid block edge for binning: 4 or 8, default 4 */
    MPM_OPT_CHUNK = 2,          /* max particles per work item: 64 .. 8192, default 2048 */
    MPM_OPT_PERSISTENT = 3,     /* 1: one persistent launch per substep; 0: three launches */
    MPM_OPT_GRAPH = 4,          /* 1: replay a captured hipGraph for 25-substep blocks */
    MPM_OPT_CAPTURE_GRID = 5,   /* 1: keep the last P2G grid for mpm_get_grid (slow, debug) */
    MPM_OPT_TIMING = 6,         /* 1: time every kernel launch with HIP events (see mpm_get_timing) */
    MPM_OPT_CONTACT = 7,        /* collider contact, default 0 (Sec. 3 names both models):
                                 * 0: on grid nodes (separating projection with Coulomb friction);
                                 * 1: particle penalty: a particle inside a collider after its
                                 *    position update gets -phi n / (4 dt) (stiffness m / (4 dt^2));
                                 * 2: both.  Either reaction goes into mpm_get_collider_wrenches. */
    MPM_OPT_WG = 8,             /* threads per workgroup of the particle kernels (P2G, G2P): 256
                                 * (default) or 512 */
    MPM_OPT_FUSE = 9            /* 1: between two re-sorts, the G2P of a substep and the P2G of
                                 * the next run as one pass over the particles (each advanced
                                 * particle is scattered from registers into the fixed-point LDS
                                 * tile; only x and F are stored, and the last substep of the run,
                                 * or of the call, stores v and C too; the default); 0: separate
                                 * P2G and G2P launches.  Same results to FP32 reorder tolerance;
                                 * the fused launch does not read the particles a second time and
                                 * is the faster on every workload measured (mpm_autotune tries
                                 * both). */
} mpm_option;

/* Kernel classes reported by mpm_get_timing (MPM_K_G2P2G: the fused G2P +
 * next-substep P2G launch of MPM_OPT_FUSE). */
typedef enum {
    MPM_K_SORT = 0, MPM_K_P2G = 1, MPM_K_GRID = 2, MPM_K_G2P = 3, MPM_K_PERSISTENT = 4, MPM_K_G2P2G = 5,
    MPM_KCLASSES = 6
} mpm_kernel_class;

mpm_status mpm_set_option(mpm_ctx ctx, int option, int value);
mpm_status mpm_get_option(mpm_ctx ctx, int option, int *value);

/* Time the candidate tunings on the live scenes for `substeps` substeps each
 * (at least one re-sort period, after one untimed period): every block edge (4, 8) x chunk size (512,
 * 2048, 8192) x sort cadence (10, 25, 50, 100) x separate or fused launches
 * (MPM_OPT_FUSE) with 256-thread workgroups, then 512-thread workgroups and
 * the one-launch substep (MPM_OPT_PERSISTENT) at the fastest of those; keep
 * the fastest, and
 * restore the particle state, the collider table and the collider wrench
 * sums afterwards.  The result is cached per (GPU architecture, grid
 * resolutions, particle-count bucket, one or many scenes), for the process
 * and in a text file ($MPM_AUTOTUNE_CACHE, else
 * $XDG_CACHE_HOME/mpm_mi355x_autotune.txt, else
 * $HOME/.cache/mpm_mi355x_autotune.txt; unreadable or unwritable files are
 * ignored): a cached tuning is applied without trials.  Writes a one-line
 * JSON report to report[0 .. report_len) when report is non-NULL (cut at
 * report_len - 1 bytes; every trial is listed, 8 KB hold them all). */
mpm_status mpm_autotune(mpm_ctx ctx, int substeps, char *report, size_t report_len);

/* Accumulated GPU time (ms, from HIP events recorded on the context stream
 * around each launch while MPM_OPT_TIMING is on) and launch counts per
 * kernel class, arrays of MPM_KCLASSES entries (either may be NULL).  Waits
 * for the timed work.  reset = 1 clears the accumulators. */
mpm_status mpm_get_timing(mpm_ctx ctx, double *ms_total, long long *launches, int reset);

/* Work queued on the context stream since mpm_create or the last reset,
 * out[MPM_NCOUNTERS] (host):
 *   MPM_CNT_SUBSTEPS        substeps of every scene (plain; a surrogate
 *                           control step counts only its fallback substeps)
 *   MPM_CNT_GRAPH_LAUNCHES  25-substep control steps replayed from a
 *                           captured hipGraph
 *   MPM_CNT_HOST_SUBSTEPS   substeps whose kernels were launched one by one
 *                           from the host
 *   MPM_CNT_SORTS           particle re-sorts (those inside replayed graphs
 *                           included)
 * Autotuning trials are counted too.  reset = 1 zeroes the counters after
 * reading them.  Never waits. */
enum { MPM_CNT_SUBSTEPS = 0, MPM_CNT_GRAPH_LAUNCHES = 1, MPM_CNT_HOST_SUBSTEPS = 2, MPM_CNT_SORTS = 3,
       MPM_NCOUNTERS = 4 };
mpm_status mpm_get_counters(mpm_ctx ctx, long long *out, int reset);

/* Internal particle order (debugging and tests): pid_out[slot] = creation
 * index of the particle held in internal slot `slot`, for all particles
 * (length mpm_num_particles(ctx, -1)); host pointer; blocks.  Inside each
 * scene the slots are ordered by the Morton code of the particle's grid
 * block (block edge = MPM_OPT_BLOCK) as of the last re-sort. */
mpm_status mpm_get_order(mpm_ctx ctx, int *pid_out);

/* Per-scene stepping mask: active[s] = 0 leaves scene s untouched by the
 * following mpm_step calls (its particles neither scatter nor move; its
 * colliders still advance).  active = NULL (or all nonzero) steps every
 * scene again.  Host array of mpm_num_scenes(ctx) ints; blocks.  The
 * scenes are independent (Sec. 3 runs one soft scene per environment), so
 * stepping a subset gives those scenes exactly what stepping all would. */
mpm_status mpm_set_scene_mask(mpm_ctx ctx, const int *active);

/* ---- Grid surrogate for one control step ------------------------------
 * The paper has no learned component; these calls let a grid network stand
 * in for one control step of 25 substeps (App. E.3: 25 physics steps per
 * control step), with the plain substeps above as the per-scene fallback.
 * All scenes must share one grid resolution R; every pointer is a device
 * pointer on the context's device; work is queued on the context stream.
 * Units: velocities in 0.2 m/s, masses in rho dx^3 of the scene, predicted
 * mass changes in rho dx^3 / 32. */

/* Box: the surrogate arrays of the next calls cover, per scene s, either the
 * whole grid (origin = NULL; the box is R^3) or the box of D x H x W nodes
 * starting at node (origin[3 s], origin[3 s + 1], origin[3 s + 2]) (origin
 * a device array of 3 n_scenes ints; 1 <= D, H, W <= R; the caller keeps
 * the box inside the grid).  Array [n_scenes][box][c] below means
 * [n_scenes][D][H][W][c], node (i, j, k) at box index (i - o0, j - o1, k - o2).
 *
 * Per scene, the nodes the current particles' P2G stencils reach: box
 * [6 n_scenes] (device) = (lo i, lo j, lo k, hi i, hi j, hi k), inclusive;
 * all zero for a scene without particles.  A box around it with a margin
 * holds every node the features and the re-splat of a control step touch. */
mpm_status mpm_sur_bbox(mpm_ctx ctx, int *box);

/* Network input and start grid of the current state at the current
 * collider poses: a P2G and grid update (the state is not changed).
 * feat  [n_scenes][box][cf] (cf >= 8): 0 m, 1-3 p (P2G output), 4
 *       distance to the nearest collider in cells clipped to [-3, 3], 5-7
 *       that collider's velocity where it is closer than 3 cells (else 0),
 *       8.. zero;
 * grid0 [n_scenes][box][4]: (m, v = p / m) of that P2G, before gravity,
 *       colliders and walls (v = 0 where m = 0).  Node (i, j, k) is at
 *       (i dx, j dx, k dx).  Material outside the box is left out. */
mpm_status mpm_sur_features(mpm_ctx ctx, float *feat, int cf, float *grid0, const int *origin, int D, int H, int W);

/* One control step from a grid prediction.  pred [n_scenes][box][cp]
 * (cp >= 4, multiple of 4): 0-2 velocity change, 3 mass change over the
 * step, at the nodes of grid0 (from mpm_sur_features on this state, same
 * box; the prediction is zero outside the box).
 * Particles advance with T = 25 dt: x += T v_mid, F <- (I + T C_mid) F
 * then the return map (v_mid the mean of the start field and the end field
 * v_end = v_start + dv, C_mid its APIC gradient at the particle), and take
 * the predicted change: v += the interpolated dv, C += its APIC gradient.
 * A P2G of the advanced particles (m_r, p_r) is compared with the
 * prediction over the nodes holding material before or after:
 *   r = max(|m_r - m_pred|_1 / sum m, |p_r - m_pred v_end|_1 / (sum m u_ref)),
 * per scene, with u_ref = 0.02 dx / T, the speed that carries a particle
 * across the per-block error bar (2e-2 dx) in one control step (re-splat
 * mass outside the box counts in full in the first term).  Scenes with r > threshold (or non-finite state) are put back
 * to their state at the start of the step and run the 25 plain substeps
 * instead (flag MPM_SUR_NO_FALLBACK keeps every scene on the surrogate and
 * only reports r).  residual [n_scenes] (nullable) receives r; n_fallback
 * [1] (nullable) the number of scenes over the threshold.  MPM_SUR_SYNC
 * waits for the decision and skips the plain substeps when no scene fell
 * back.  Colliders advance by 25 substeps either way. */
enum { MPM_SUR_NO_FALLBACK = 1, MPM_SUR_SYNC = 2 };
mpm_status mpm_sur_block(mpm_ctx ctx, const float *pred, int cp, const float *grid0, const int *origin, int D, int H,
                         int W, float threshold, int flags, float *residual, int *n_fallback);

/* Library-owned surrogate (Algorithm 1's inner soft-step loop, one control
 * step of 25 substeps at a time, App. E.3, with the network in front of it).
 *
 * mpm_surrogate_load: copy a trained grid U-Net into the context (replacing
 * one loaded before).  weights: host blob of `bytes` bytes, little-endian:
 *   int32 header[8] = {0x554E504D, 1, cin, cout, width, 15, 0, 0}
 *   then for each of the 15 layers in order (e1a, e1b, d1, e2a, e2b, d2,
 *   e3a, e3b, u2, c2a, c2b, u1, c1a, c1b, head): FP32 weights
 *   [taps][ci][co] (taps 27 for 3^3 and upsampling layers, 8 for the
 *   stride-2 layers, 1 for the head; z-major) and FP32 bias [co].
 * Channels (ci -> co) at width 1: e1a ceil16(cin) -> 32 (weights of the
 * padding channels ignored), e1b 32 -> 32, d1 32 -> 64, e2a/e2b 64 -> 64,
 * d2 64 -> 128, e3a/e3b 128 -> 128, u2 128 -> 64, c2a 128 -> 64, c2b 64 -> 64,
 * u1 64 -> 32, c1a 64 -> 32, c1b 32 -> 32, head 32 -> cout; width 2 halves
 * every count but cin and cout.  cin <= 8 (the feature channels of
 * mpm_sur_features), cout a multiple of 4 (channels 0-3 as in mpm_sur_block).
 * The blob is borrowed for the call.  MPM_ERR_ARG for a malformed blob or a
 * batch without one common grid resolution.
 *
 * mpm_step_blocks: run n_blocks control steps of every scene.  use_surrogate
 * = 0: 25 plain substeps each (as mpm_step(ctx, 25 n_blocks)).
 * use_surrogate = 1: per block, the box of the material (mpm_sur_bbox, read
 * back to the host: the call waits once per block), the features on it, the
 * network's prediction, and mpm_sur_block's control step with its residual
 * gate at residual_threshold: scenes over it are put back and run the 25
 * plain substeps.  *fallback_count (host, nullable) receives the number of
 * scene-blocks that fell back; the call returns MPM_WARN_FALLBACK when any
 * did.  MPM_ERR_STATE when no network is loaded.  Colliders advance by 25
 * substeps per block either way. */
mpm_status mpm_surrogate_load(mpm_ctx ctx, const void *weights, size_t bytes);
mpm_status mpm_step_blocks(mpm_ctx ctx, int n_blocks, int use_surrogate, float residual_threshold,
                           int *fallback_count);

/* Residual of every scene in the last block mpm_step_blocks ran with the
 * surrogate: out [n_scenes] (host).  MPM_ERR_STATE before any such block. */
mpm_status mpm_surrogate_residuals(mpm_ctx ctx, float *out);

/* Training targets between the start grids g0, g1 of two consecutive
 * control steps (both from mpm_sur_features on the whole grid): target
 * [n][R^3][ct] (ct >= 4)
 * = ((v1 - v0) in 0.2 m/s, (m1 - m0) in rho dx^3 / 32), and a loss weight
 * mask [n][R^3] = min(1, max(m0, m1) / (rho dx^3)) where m0 > 0 or m1 > 0
 * (positive there), else 0: the node's share of a filled cell's mass, as
 * the residual gate weighs velocity errors by mass. */
mpm_status mpm_sur_targets(mpm_ctx ctx, const float *g0, const float *g1, float *target, int ct, float *mask);

/* Introspection. */
int mpm_num_scenes(mpm_ctx ctx);
int mpm_num_particles(mpm_ctx ctx, int scene);   /* scene = -1: total */
int mpm_max_colliders(mpm_ctx ctx);
int mpm_res(mpm_ctx ctx, int scene);
const char *mpm_status_string(mpm_status status);
const char *mpm_last_error(mpm_ctx ctx);          /* detail of the last error on ctx */

#ifdef __cplusplus
}
#endif
#endif /* MPM_H */
