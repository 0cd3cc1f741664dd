// Shared host/device layout of the MI355X MLS-MPM library (internal).
#pragma once
#include <stdint.h>

namespace mpm {

// Particle storage: one float array per component, struct-of-arrays, all
// scenes concatenated (scene s owns the fixed slot range [p_begin, p_end)).
// The particle order inside a scene changes at every re-sort; PID keeps the
// creation index (stored as int bits).
enum Comp : int {
    X0 = 0, X1, X2,                 // position (m)
    V0, V1, V2,                     // velocity (m/s)
    A00, A01, A02, A10, A11, A12, A20, A21, A22,   // affine momentum m C - dt V D tau(F), row-major
    G00, G01, G02, G10, G11, G12, G20, G21, G22,   // displacement gradient G = F - I, row-major
    PID,
    NCOMP
};

enum Flag : int { FLAG_CLAMPED = 1, FLAG_NONFINITE = 2, FLAG_OVERFLOW_FULL = 8 };

constexpr int MAX_COLLIDERS_PER_SCENE = 4;   // equals MPM_MAX_COLLIDERS of the public header

struct SceneDev {
    int p_begin, p_end;       // particle slots
    int res, nb;              // nodes per axis, blocks per axis
    long long grid_off;       // first node of this scene in the dense grid arrays
    int bin_off;              // first bin (nb^3 bins per scene)
    int col_off, n_col;       // colliders
    int bound;
    int model;                // 0 neo-Hookean, 1 Hencky
    int plastic;              // von Mises return map on/off
    float dx, inv_dx, dt;
    float g[3];
    float mu, la;             // Lame parameters
    float yield_eps;          // yield radius in deviatoric log strain
    float mass, vol;          // per particle
    float kstress;            // dt * vol * 4 / dx^2
    float D;                  // 4 / dx^2
};

struct ColliderDev {
    int type;                 // 0 box, 1 capsule, 2 sampled SDF volume
    float he[3];
    float radius, half_length, friction;
    float pos[3];             // centre at the start of the current mpm_step call
    float quat[4];            // w x y z at the start of the current call
    float vlin[3];
    float omega[3];
    int sdf_off;              // type 2: first sample in the context's SDF buffer
    int sdf_dims[3];          //   samples per axis, stored [nx][ny][nz]
    float sdf_cell;           //   spacing
    float sdf_origin[3];      //   body-frame position of sample (0, 0, 0)
};

// One unit of particle work: a chunk of the particles binned to one grid
// block of one scene (particles [start, start + count) in sorted order).
struct Item {
    int scene;
    int block;                // linear block index (bx * nb + by) * nb + bz
    int start;
    int count;
};

// Substep work lists and counters produced by the sort (device memory).
struct Lists {
    Item *items;              // particle items, scene-major
    int2 *gitems;             // grid blocks to update: (scene, linear block)
    int *n_items;             // [1]
    int *n_gitems;            // [1]
    int *scene_item_begin;    // [n_scenes + 1]
    int *scene_gitem_begin;   // [n_scenes + 1]
    int *bflag;               // per block (all scenes, linear order): 2 static grid block, 1 overflow, 0 none
    int2 *ovf;                // overflow grid blocks (scene, linear block)
    int *n_ovf;               // [2] overflow list length, by substep parity
    int ovf_cap;
    float *ibound;            // per item: max over its particles of m|v_c| + 1.5 dx sum_e |A_ce| (P2G scale)
    int *icell;               // per item: most particles sharing a base cell (P2G scale), 0 = not known
    unsigned char *touched;   // per block (all scenes, linear order): 1 = received mass in this substep's P2G
    int *order;               // [n_items] item indices, most particles first: the dispatch order of P2G / G2P
};

}  // namespace mpm
