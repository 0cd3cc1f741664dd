/*
 * FP64 CPU oracle for one MLS-MPM substep (TEST INFRASTRUCTURE ONLY).
 *
 * This file is the plain, slow reference that the HIP path is checked
 * against.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline load it; the product library never links or calls it, and it
 * shares no code, header, table or helper with the HIP sources.
 *
 * What it computes (the paper, Sec. 3 "Rigid-soft Coupling" and Algorithm 1
 * in App. D.1): the soft step is MLS-MPM (moving least squares MPM with APIC
 * transfers, the method the paper says its solver follows) with
 *   particle-to-grid transfer of mass and momentum including the stress term,
 *   a grid velocity update,
 *   grid-to-particle transfer of velocity and its gradient,
 *   particle integration (position, deformation gradient),
 * for elastoplastic material (App. D.3, Table "tab:mpm_param": Young's
 * modulus, Poisson ratio, yield stress), pushed by kinematic rigid shapes
 * given as analytic signed distance functions (Sec. 3: boxes and capsules,
 * applied on grid nodes, the PlasticineLab-style variant the paper also
 * supports).  The paper prints no equations for these steps; the readings
 * taken where it is silent are:
 *   - quadratic B-spline weights, APIC affine matrix C, D^-1 = 4/dx^2;
 *   - neo-Hookean:  tau = mu (F F^T - I) + lambda ln(J) I;
 *   - Hencky:       F = U S V^T, eps = ln S, tau = U (2 mu eps + lambda tr(eps) I) U^T;
 *   - von Mises return map on the principal log strain, applied after the
 *     F update; yield when |dev eps| > sy / (2 mu) (yield_form 0) or
 *     sqrt(2/3) sy / (2 mu) (yield_form 1);
 *   - grid order: v = p/m (0 when m == 0), gravity, colliders in index
 *     order (contact when phi < 0 and the relative normal velocity is
 *     negative; Coulomb friction), then walls of `bound` cells (separating);
 *   - collider pose for a substep is its start-of-substep pose; after G2P
 *     c <- c + dt v and q <- exp(dt w / 2) (x) q;
 *   - SVD: singular values sorted descending, U and V proper rotations, the
 *     last singular value negative when det F < 0; clamp at 1e-6 before ln.
 *   - weakly compressible fluid (model 2, for the liquid of the Pour task,
 *     Sec. 2.1; the paper prints no fluid law): Tait equation of state with exponent 7
 *     and the bulk modulus K = lambda + 2 mu / 3 of (E, nu),
 *     p(J) = (K / 7) (J^-7 - 1), Kirchhoff stress tau = -J p(J) I; after the
 *     F update F is replaced by J^(1/3) I (the fluid keeps its volume change
 *     and no shear).
 *   - a particle whose stencil leaves the grid is an error (return -2).
 *
 * Grid layout: node (i, j, k) sits at (i dx, j dx, k dx) and is stored at
 * index (i * res + j) * res + k.  Particle arrays are row-major [n][3] and
 * [n][3][3].  Parallel loops (OpenMP) are only over independent particles
 * or nodes; the particle-to-grid scatter runs serially in particle order.
 */
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int type;                 /* 0 box, 1 capsule, 2 sampled SDF volume */
    double half_extents[3];   /* box half sizes, body frame */
    double radius;            /* capsule radius */
    double half_length;       /* capsule half segment length along body y */
    double friction;          /* Coulomb coefficient; +inf = sticky */
    double pos[3];            /* centre (world) */
    double quat[4];           /* orientation w, x, y, z (body -> world) */
    double vlin[3];           /* linear velocity of the centre */
    double omega[3];          /* angular velocity (world frame) */
    /* type 2: samples of the body-frame signed distance at sdf_origin + (i, j, k) sdf_cell,
     * stored [nx][ny][nz]; the distance is their trilinear interpolant */
    const double *sdf;
    int sdf_dims[3];
    double sdf_cell;
    double sdf_origin[3];
} orc_collider;

typedef struct {
    int n;
    double *x, *v, *C, *F;    /* [n][3], [n][3], [n][3][3], [n][3][3] */
    int res;
    double dx, dt;
    double g[3];
    int bound;
    int model;                /* 0 neo-Hookean, 1 Hencky + von Mises, 2 weakly compressible fluid */
    double E, nu, rho, yield_stress;
    int yield_form;
    double p_vol;
    int n_col;
    orc_collider *col;
    double *wrench;           /* [n_col][6] or NULL: impulse on each collider and its
                                 angular impulse about the collider centre, summed */
    int contact;              /* 0 grid-node projection, 1 particle penalty, 2 both */
} orc_scene;

#define SIGMA_MIN 1e-6

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the parallel loops that follow (n >= 1); timing only. */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n < 1 ? 1 : n);
#else
    (void)n;
#endif
}

static void lame(const orc_scene *s, double *mu, double *la)
{
    *mu = s->E / (2.0 * (1.0 + s->nu));
    *la = s->E * s->nu / ((1.0 + s->nu) * (1.0 - 2.0 * s->nu));
}

static int is_plastic(const orc_scene *s)
{
    return s->model == 1 && s->yield_stress > 0.0 && isfinite(s->yield_stress);
}

/* Quadratic B-spline weights for the three nodes base, base+1, base+2 at
 * fractional offset f = x/dx - base, f in [0.5, 1.5). */
void orc_weights(double f, double w[3])
{
    w[0] = 0.5 * (1.5 - f) * (1.5 - f);
    w[1] = 0.75 - (f - 1.0) * (f - 1.0);
    w[2] = 0.5 * (f - 0.5) * (f - 0.5);
}

/* ---------------- 3x3 helpers (row-major) ---------------- */
static void matmul(const double *a, const double *b, double *c)
{
    double t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double acc = 0.0;
            for (int k = 0; k < 3; k++) acc += a[i * 3 + k] * b[k * 3 + j];
            t[i * 3 + j] = acc;
        }
    memcpy(c, t, sizeof t);
}

static double det3(const double *a)
{
    return a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6])
         + a[2] * (a[3] * a[7] - a[4] * a[6]);
}

static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* SVD of a 3x3 matrix by one-sided (Hestenes) Jacobi: rotate column pairs
 * of W = F V until all columns are orthogonal; singular values are the
 * column norms.  Output convention: S descending, U and V rotations,
 * S[2] < 0 when det F < 0.  Returns the number of sweeps used. */
int orc_svd3(const double *F, double *U, double *S, double *V)
{
    double W[9];
    memcpy(W, F, sizeof W);
    for (int i = 0; i < 9; i++) V[i] = (i % 4 == 0) ? 1.0 : 0.0;
    int sweep;
    for (sweep = 0; sweep < 100; sweep++) {
        int rotated = 0;
        for (int p = 0; p < 2; p++)
            for (int q = p + 1; q < 3; q++) {
                double a = 0, b = 0, g = 0;
                for (int k = 0; k < 3; k++) {
                    a += W[k * 3 + p] * W[k * 3 + p];
                    b += W[k * 3 + q] * W[k * 3 + q];
                    g += W[k * 3 + p] * W[k * 3 + q];
                }
                if (g == 0.0 || fabs(g) <= DBL_EPSILON * sqrt(a * b)) continue;
                rotated = 1;
                double zeta = (b - a) / (2.0 * g);
                double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                for (int k = 0; k < 3; k++) {
                    double wp = W[k * 3 + p], wq = W[k * 3 + q];
                    W[k * 3 + p] = c * wp - s * wq;
                    W[k * 3 + q] = s * wp + c * wq;
                    double vp = V[k * 3 + p], vq = V[k * 3 + q];
                    V[k * 3 + p] = c * vp - s * vq;
                    V[k * 3 + q] = s * vp + c * vq;
                }
            }
        if (!rotated) break;
    }
    double sig[3];
    for (int j = 0; j < 3; j++)
        sig[j] = sqrt(W[j] * W[j] + W[3 + j] * W[3 + j] + W[6 + j] * W[6 + j]);
    /* sort columns by singular value, descending */
    int ord[3] = {0, 1, 2};
    for (int i = 0; i < 3; i++)
        for (int j = i + 1; j < 3; j++)
            if (sig[ord[j]] > sig[ord[i]]) { int t = ord[i]; ord[i] = ord[j]; ord[j] = t; }
    double Ws[9], Vs[9];
    for (int j = 0; j < 3; j++) {
        S[j] = sig[ord[j]];
        for (int k = 0; k < 3; k++) {
            Ws[k * 3 + j] = W[k * 3 + ord[j]];
            Vs[k * 3 + j] = V[k * 3 + ord[j]];
        }
    }
    memcpy(V, Vs, sizeof Vs);
    /* U columns: normalised W columns; complete the basis where S is zero */
    double u[3][3];
    for (int j = 0; j < 3; j++)
        for (int k = 0; k < 3; k++) u[j][k] = S[j] > 0 ? Ws[k * 3 + j] / S[j] : 0.0;
    if (S[0] == 0.0) { u[0][0] = 1; u[0][1] = 0; u[0][2] = 0; }
    if (S[1] == 0.0) {
        double e[3] = {0, 0, 0};
        int a = fabs(u[0][0]) < 0.5 ? 0 : 1;
        e[a] = 1.0;
        double d = e[0] * u[0][0] + e[1] * u[0][1] + e[2] * u[0][2];
        double n = 0;
        for (int k = 0; k < 3; k++) { u[1][k] = e[k] - d * u[0][k]; n += u[1][k] * u[1][k]; }
        n = sqrt(n);
        for (int k = 0; k < 3; k++) u[1][k] /= n;
    }
    if (S[2] == 0.0) cross3(u[0], u[1], u[2]);
    for (int j = 0; j < 3; j++)
        for (int k = 0; k < 3; k++) U[k * 3 + j] = u[j][k];
    if (det3(U) < 0) { for (int k = 0; k < 3; k++) U[k * 3 + 2] = -U[k * 3 + 2]; S[2] = -S[2]; }
    if (det3(V) < 0) { for (int k = 0; k < 3; k++) V[k * 3 + 2] = -V[k * 3 + 2]; S[2] = -S[2]; }
    return sweep;
}

/* Kirchhoff stress tau(F). */
void orc_stress(const orc_scene *s, const double *F, double *tau)
{
    double mu, la;
    lame(s, &mu, &la);
    if (s->model == 2) {
        double J = det3(F);
        double K = la + 2.0 * mu / 3.0;
        double p = K / 7.0 * (pow(J, -7.0) - 1.0);
        for (int i = 0; i < 9; i++) tau[i] = i % 4 == 0 ? -J * p : 0.0;
        return;
    }
    if (s->model == 0) {
        double J = det3(F);
        double lnJ = log(J);
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                double ffT = 0;
                for (int k = 0; k < 3; k++) ffT += F[i * 3 + k] * F[j * 3 + k];
                tau[i * 3 + j] = mu * (ffT - (i == j)) + (i == j ? la * lnJ : 0.0);
            }
        return;
    }
    double U[9], S[3], V[9], eps[3];
    orc_svd3(F, U, S, V);
    for (int k = 0; k < 3; k++) eps[k] = log(S[k] > SIGMA_MIN ? S[k] : SIGMA_MIN);
    double tr = eps[0] + eps[1] + eps[2];
    double d[3];
    for (int k = 0; k < 3; k++) d[k] = 2.0 * mu * eps[k] + la * tr;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double acc = 0;
            for (int k = 0; k < 3; k++) acc += U[i * 3 + k] * d[k] * U[j * 3 + k];
            tau[i * 3 + j] = acc;
        }
}

/* von Mises return map in principal log strain; F is replaced in place.
 * Returns 1 when the particle yielded. */
int orc_return_map(const orc_scene *s, double *F)
{
    if (!is_plastic(s)) return 0;
    double mu, la;
    lame(s, &mu, &la);
    double U[9], S[3], V[9], eps[3];
    orc_svd3(F, U, S, V);
    for (int k = 0; k < 3; k++) eps[k] = log(S[k] > SIGMA_MIN ? S[k] : SIGMA_MIN);
    double mean = (eps[0] + eps[1] + eps[2]) / 3.0;
    double dev[3], nd = 0;
    for (int k = 0; k < 3; k++) { dev[k] = eps[k] - mean; nd += dev[k] * dev[k]; }
    nd = sqrt(nd);
    double ry = s->yield_stress / (2.0 * mu);
    if (s->yield_form == 1) ry *= sqrt(2.0 / 3.0);
    double dg = nd - ry;
    int yielded = dg > 0;
    if (yielded)
        for (int k = 0; k < 3; k++) eps[k] -= dg * dev[k] / nd;
    double e[3];
    for (int k = 0; k < 3; k++) e[k] = exp(eps[k]);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double acc = 0;
            for (int k = 0; k < 3; k++) acc += U[i * 3 + k] * e[k] * V[j * 3 + k];
            F[i * 3 + j] = acc;
        }
    return yielded;
}

/* ---------------- colliders ---------------- */
static void quat_rotate(const double *q, const double *v, double *out)
{
    /* out = R(q) v for unit q = (w, x, y, z) */
    double w = q[0], x = q[1], y = q[2], z = q[3];
    double R[9] = {
        1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
        2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
        2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
    for (int i = 0; i < 3; i++) out[i] = R[i * 3] * v[0] + R[i * 3 + 1] * v[1] + R[i * 3 + 2] * v[2];
}

static void quat_rotate_inv(const double *q, const double *v, double *out)
{
    double qc[4] = {q[0], -q[1], -q[2], -q[3]};
    quat_rotate(qc, v, out);
}

/* Sampled SDF volume (a mesh collider stored as a 3D grid of distances, as
 * the paper keeps its mesh SDFs in 3D textures, Sec. 3): the distance at a
 * body-frame point p is the trilinear interpolant of the eight samples of the
 * cell holding p, the normal the normalised gradient of that interpolant
 * (body +x where it vanishes).  Outside the sampled box there is no contact:
 * the distance is +DBL_MAX. */
static double sdf_volume(const orc_collider *c, const double *p, double *nb)
{
    double u[3], f[3];
    int i0[3];
    nb[0] = 1.0; nb[1] = 0.0; nb[2] = 0.0;
    for (int a = 0; a < 3; a++) {
        u[a] = (p[a] - c->sdf_origin[a]) / c->sdf_cell;
        if (!(u[a] >= 0.0 && u[a] <= c->sdf_dims[a] - 1)) return DBL_MAX;
        i0[a] = (int)floor(u[a]);
        if (i0[a] > c->sdf_dims[a] - 2) i0[a] = c->sdf_dims[a] - 2;
        f[a] = u[a] - i0[a];
    }
    int ny = c->sdf_dims[1], nz = c->sdf_dims[2];
    double phi = 0.0, g[3] = {0.0, 0.0, 0.0};
    for (int dx_ = 0; dx_ < 2; dx_++)
        for (int dy = 0; dy < 2; dy++)
            for (int dz = 0; dz < 2; dz++) {
                double s = c->sdf[((size_t)(i0[0] + dx_) * ny + (i0[1] + dy)) * nz + (i0[2] + dz)];
                double wx = dx_ ? f[0] : 1.0 - f[0], wy = dy ? f[1] : 1.0 - f[1], wz = dz ? f[2] : 1.0 - f[2];
                phi += wx * wy * wz * s;
                g[0] += (dx_ ? 1.0 : -1.0) * wy * wz * s;
                g[1] += (dy ? 1.0 : -1.0) * wx * wz * s;
                g[2] += (dz ? 1.0 : -1.0) * wx * wy * s;
            }
    double len = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    if (len > 0.0)
        for (int a = 0; a < 3; a++) nb[a] = g[a] / len;
    return phi;
}

/* Signed distance of world point x to the collider and the outward unit
 * normal (world frame).  Box inside: nearest face, ties to the lowest axis,
 * + before -.  Capsule on its axis: body +x. */
double orc_sdf(const orc_collider *c, const double *x, double *n)
{
    double r[3] = {x[0] - c->pos[0], x[1] - c->pos[1], x[2] - c->pos[2]};
    double p[3], nb[3] = {0, 0, 0}, phi;
    quat_rotate_inv(c->quat, r, p);
    if (c->type == 2) {
        phi = sdf_volume(c, p, nb);
    } else if (c->type == 0) {
        double q[3], outside = 0;
        for (int a = 0; a < 3; a++) {
            q[a] = fabs(p[a]) - c->half_extents[a];
            if (q[a] > 0) outside += q[a] * q[a];
        }
        if (outside > 0) {
            phi = sqrt(outside);
            for (int a = 0; a < 3; a++)
                nb[a] = q[a] > 0 ? (p[a] >= 0 ? 1.0 : -1.0) * q[a] / phi : 0.0;
        } else {
            int best = 0;
            for (int a = 1; a < 3; a++)
                if (q[a] > q[best]) best = a;
            phi = q[best];
            nb[best] = p[best] >= 0 ? 1.0 : -1.0;
        }
    } else {
        double t = p[1];
        if (t > c->half_length) t = c->half_length;
        if (t < -c->half_length) t = -c->half_length;
        double d[3] = {p[0], p[1] - t, p[2]};
        double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        phi = len - c->radius;
        if (len > 0) { nb[0] = d[0] / len; nb[1] = d[1] / len; nb[2] = d[2] / len; }
        else nb[0] = 1.0;
    }
    quat_rotate(c->quat, nb, n);
    return phi;
}

/* Project one grid velocity against one collider (in place).  Returns 1 if
 * the contact branch was taken. */
int orc_collide(const orc_collider *c, const double *xi, double *v)
{
    double n[3];
    double phi = orc_sdf(c, xi, n);
    double r[3] = {xi[0] - c->pos[0], xi[1] - c->pos[1], xi[2] - c->pos[2]};
    double wr[3];
    cross3(c->omega, r, wr);
    double vc[3] = {c->vlin[0] + wr[0], c->vlin[1] + wr[1], c->vlin[2] + wr[2]};
    double u[3] = {v[0] - vc[0], v[1] - vc[1], v[2] - vc[2]};
    double un = u[0] * n[0] + u[1] * n[1] + u[2] * n[2];
    if (!(phi < 0 && un < 0)) return 0;
    double ut[3] = {u[0] - un * n[0], u[1] - un * n[1], u[2] - un * n[2]};
    double lt = sqrt(ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2]);
    double scale;
    if (isinf(c->friction) || lt == 0.0) scale = 0.0;
    else {
        scale = 1.0 + c->friction * un / lt;
        if (scale < 0) scale = 0;
    }
    for (int a = 0; a < 3; a++) v[a] = vc[a] + scale * ut[a];
    return 1;
}

void orc_advance_colliders(orc_scene *s)
{
    for (int k = 0; k < s->n_col; k++) {
        orc_collider *c = &s->col[k];
        for (int a = 0; a < 3; a++) c->pos[a] += s->dt * c->vlin[a];
        double wn = sqrt(c->omega[0] * c->omega[0] + c->omega[1] * c->omega[1] + c->omega[2] * c->omega[2]);
        if (wn == 0.0) continue;
        double h = 0.5 * s->dt * wn;
        double dq[4] = {cos(h), sin(h) * c->omega[0] / wn, sin(h) * c->omega[1] / wn, sin(h) * c->omega[2] / wn};
        double *q = c->quat;
        double nq[4] = {
            dq[0] * q[0] - dq[1] * q[1] - dq[2] * q[2] - dq[3] * q[3],
            dq[0] * q[1] + dq[1] * q[0] + dq[2] * q[3] - dq[3] * q[2],
            dq[0] * q[2] - dq[1] * q[3] + dq[2] * q[0] + dq[3] * q[1],
            dq[0] * q[3] + dq[1] * q[2] - dq[2] * q[1] + dq[3] * q[0]};
        memcpy(q, nq, sizeof nq);
    }
}

/* ---------------- transfers ---------------- */
static int particle_base(const orc_scene *s, const double *x, int base[3], double f[3])
{
    for (int a = 0; a < 3; a++) {
        double xi = x[a] / s->dx;
        double b = floor(xi - 0.5);
        if (!(b >= 0 && b <= s->res - 3)) return -2;
        base[a] = (int)b;
        f[a] = xi - b;
    }
    return 0;
}

/* Affine momentum matrix A_p = m C_p - dt V (4/dx^2) tau(F_p) for every
 * particle (row-major [n][3][3]). */
void orc_affine(const orc_scene *s, double *A)
{
    double m = s->rho * s->p_vol;
    double k = s->dt * s->p_vol * 4.0 / (s->dx * s->dx);
#pragma omp parallel for schedule(static)
    for (int p = 0; p < s->n; p++) {
        double tau[9];
        orc_stress(s, s->F + 9 * p, tau);
        for (int i = 0; i < 9; i++) A[9 * p + i] = m * s->C[9 * p + i] - k * tau[i];
    }
}

/* Particle to grid.  m: [res^3], p: [res^3][3]; both are overwritten. */
int orc_p2g(const orc_scene *s, double *gm, double *gp)
{
    size_t nn = (size_t)s->res * s->res * s->res;
    memset(gm, 0, nn * sizeof(double));
    memset(gp, 0, 3 * nn * sizeof(double));
    double *A = (double *)malloc(sizeof(double) * 9 * (size_t)(s->n > 0 ? s->n : 1));
    if (!A) return -3;
    orc_affine(s, A);
    double m = s->rho * s->p_vol;
    int err = 0;
    for (int p = 0; p < s->n && !err; p++) {
        int base[3];
        double f[3], w[3][3];
        if (particle_base(s, s->x + 3 * p, base, f)) { err = -2; break; }
        for (int a = 0; a < 3; a++) orc_weights(f[a], w[a]);
        const double *v = s->v + 3 * p, *Ap = A + 9 * p;
        for (int ox = 0; ox < 3; ox++)
            for (int oy = 0; oy < 3; oy++)
                for (int oz = 0; oz < 3; oz++) {
                    double wt = w[0][ox] * w[1][oy] * w[2][oz];
                    double d[3] = {(ox - f[0]) * s->dx, (oy - f[1]) * s->dx, (oz - f[2]) * s->dx};
                    size_t idx = ((size_t)(base[0] + ox) * s->res + (base[1] + oy)) * s->res + (base[2] + oz);
                    gm[idx] += wt * m;
                    for (int i = 0; i < 3; i++)
                        gp[3 * idx + i] += wt * (m * v[i] + Ap[3 * i] * d[0] + Ap[3 * i + 1] * d[1] + Ap[3 * i + 2] * d[2]);
                }
    }
    free(A);
    return err;
}

/* Grid velocity update: vg[res^3][3] from m, p.
 *
 * Two-way coupling (Algorithm 1 accumulates the soft body's forces on the
 * rigid bodies during the soft steps): with contact on grid nodes, what
 * collider c exerts on the material in this substep is the momentum its
 * projection adds at the nodes it touches, m_i (v_after - v_before); by
 * Newton's third law the collider receives the opposite impulse, and the
 * opposite angular impulse (x_i - c) x m_i (v_after - v_before) about its
 * centre c at this substep's pose.  With s->wrench set they are summed into
 * s->wrench (then the node loop runs serially, in node order). */
void orc_grid_op(const orc_scene *s, const double *gm, const double *gp, double *vg)
{
    int R = s->res;
#pragma omp parallel for schedule(static) if (s->wrench == NULL)
    for (int i = 0; i < R; i++)
        for (int j = 0; j < R; j++)
            for (int k = 0; k < R; k++) {
                size_t idx = ((size_t)i * R + j) * R + k;
                double v[3];
                for (int a = 0; a < 3; a++) v[a] = gm[idx] > 0 ? gp[3 * idx + a] / gm[idx] : 0.0;
                for (int a = 0; a < 3; a++) v[a] += s->dt * s->g[a];
                double xi[3] = {i * s->dx, j * s->dx, k * s->dx};
                for (int c = 0; c < s->n_col && s->contact != 1; c++) {
                    double v0[3] = {v[0], v[1], v[2]};
                    if (!orc_collide(&s->col[c], xi, v) || !s->wrench) continue;
                    double dp[3], r[3], t[3];
                    for (int a = 0; a < 3; a++) {
                        dp[a] = gm[idx] * (v[a] - v0[a]);
                        r[a] = xi[a] - s->col[c].pos[a];
                    }
                    cross3(r, dp, t);
                    for (int a = 0; a < 3; a++) {
                        s->wrench[6 * c + a] -= dp[a];
                        s->wrench[6 * c + 3 + a] -= t[a];
                    }
                }
                int ii[3] = {i, j, k};
                for (int a = 0; a < 3; a++) {
                    if (ii[a] < s->bound && v[a] < 0) v[a] = 0;
                    if (ii[a] >= R - s->bound && v[a] > 0) v[a] = 0;
                }
                for (int a = 0; a < 3; a++) vg[3 * idx + a] = v[a];
            }
}

/* Particle penalty contact (the paper's default contact model, Sec. 3; its
 * stiffness is not printed): a particle found inside collider c after its
 * position update (phi < 0 at the substep's pose) receives the velocity
 * change -phi n / (4 dt), a spring of stiffness m / (4 dt^2) along the
 * outward normal that removes a quarter of the penetration per substep; the
 * collider receives the opposite impulse and angular impulse about its
 * centre (summed into s->wrench when set). */
static void penalty(orc_scene *s, const double *x, double *v)
{
    double m = s->rho * s->p_vol;
    for (int c = 0; c < s->n_col; c++) {
        double n[3];
        double phi = orc_sdf(&s->col[c], x, n);
        if (!(phi < 0.0)) continue;
        double dp[3], r[3], t[3];
        for (int a = 0; a < 3; a++) {
            double dv = -phi * n[a] / (4.0 * s->dt);
            v[a] += dv;
            dp[a] = m * dv;
            r[a] = x[a] - s->col[c].pos[a];
        }
        if (!s->wrench) continue;
        cross3(r, dp, t);
        for (int a = 0; a < 3; a++) {
            s->wrench[6 * c + a] -= dp[a];
            s->wrench[6 * c + 3 + a] -= t[a];
        }
    }
}

/* Grid to particle, particle integration and return map. */
int orc_g2p(orc_scene *s, const double *vg)
{
    int err = 0;
    double D = 4.0 / (s->dx * s->dx);
    /* with penalty wrenches summed, particles run in order (one accumulator) */
#pragma omp parallel for schedule(static) reduction(min : err) if (!(s->wrench && s->contact != 0))
    for (int p = 0; p < s->n; p++) {
        int base[3];
        double f[3], w[3][3];
        double *x = s->x + 3 * p, *v = s->v + 3 * p, *C = s->C + 9 * p, *F = s->F + 9 * p;
        if (particle_base(s, x, base, f)) { err = -2; continue; }
        for (int a = 0; a < 3; a++) orc_weights(f[a], w[a]);
        double nv[3] = {0, 0, 0}, B[9] = {0};
        for (int ox = 0; ox < 3; ox++)
            for (int oy = 0; oy < 3; oy++)
                for (int oz = 0; oz < 3; oz++) {
                    double wt = w[0][ox] * w[1][oy] * w[2][oz];
                    double d[3] = {(ox - f[0]) * s->dx, (oy - f[1]) * s->dx, (oz - f[2]) * s->dx};
                    size_t idx = ((size_t)(base[0] + ox) * s->res + (base[1] + oy)) * s->res + (base[2] + oz);
                    const double *vi = vg + 3 * idx;
                    for (int i = 0; i < 3; i++) {
                        nv[i] += wt * vi[i];
                        for (int j = 0; j < 3; j++) B[3 * i + j] += wt * vi[i] * d[j];
                    }
                }
        for (int i = 0; i < 3; i++) v[i] = nv[i];
        for (int i = 0; i < 9; i++) C[i] = D * B[i];
        for (int i = 0; i < 3; i++) x[i] += s->dt * v[i];
        if (s->contact != 0) penalty(s, x, v);
        double M[9];
        for (int i = 0; i < 9; i++) M[i] = (i % 4 == 0 ? 1.0 : 0.0) + s->dt * C[i];
        matmul(M, F, F);
        if (s->model == 2) {   /* fluid: only the volume change is kept */
            double c = cbrt(det3(F));
            for (int i = 0; i < 9; i++) F[i] = i % 4 == 0 ? c : 0.0;
        } else {
            orc_return_map(s, F);
        }
    }
    return err;
}

/* Surrogate control step from a grid prediction (the paper has no learned
 * part; a grid model stands in for one control step of n_sub substeps).
 * vs [res^3][3]: the start grid velocity (P2G momentum / mass of the current
 * state, 0 where the mass is 0); dv [res^3][3]: the predicted change of that
 * velocity over the step.  With T = n_sub dt, mid field u = vs + dv / 2 and
 * end field e = vs + dv, every particle, with its weights at its start
 * position:
 *   v_mid = sum w u_i,   C_mid = (4/dx^2) sum w u_i (x_i - x_p)^T,
 *   x    <- x + T v_mid,
 *   F    <- (I + T C_mid) F, then the return map (or the fluid's volume-only
 *           projection), as after a plain substep;
 *   mode 1: v <- v + sum w dv_i,  C <- C + (4/dx^2) sum w dv_i (x_i - x_p)^T
 *           (the particles take the predicted change: the surrogate's
 *           particle update);
 *   mode 0: v <- sum w e_i,  C <- (4/dx^2) sum w e_i (x_i - x_p)^T
 *           (the particles take the end field; kept to measure how far this
 *           simpler form lands from a plain control step).
 * Returns -2 when a stencil leaves the grid. */
int orc_sur_advance(orc_scene *s, const double *vs, const double *dv, int n_sub, int mode)
{
    int err = 0;
    double D = 4.0 / (s->dx * s->dx), T = n_sub * s->dt;
#pragma omp parallel for schedule(static) reduction(min : err)
    for (int p = 0; p < s->n; p++) {
        int base[3];
        double f[3], w[3][3];
        double *x = s->x + 3 * p, *v = s->v + 3 * p, *C = s->C + 9 * p, *F = s->F + 9 * p;
        if (particle_base(s, x, base, f)) { err = -2; continue; }
        for (int a = 0; a < 3; a++) orc_weights(f[a], w[a]);
        double vm[3] = {0, 0, 0}, ve[3] = {0, 0, 0}, vd[3] = {0, 0, 0};
        double Bm[9] = {0}, Be[9] = {0}, Bd[9] = {0};
        for (int ox = 0; ox < 3; ox++)
            for (int oy = 0; oy < 3; oy++)
                for (int oz = 0; oz < 3; oz++) {
                    double wt = w[0][ox] * w[1][oy] * w[2][oz];
                    double d[3] = {(ox - f[0]) * s->dx, (oy - f[1]) * s->dx, (oz - f[2]) * s->dx};
                    size_t idx = ((size_t)(base[0] + ox) * s->res + (base[1] + oy)) * s->res + (base[2] + oz);
                    for (int i = 0; i < 3; i++) {
                        double u = vs[3 * idx + i] + 0.5 * dv[3 * idx + i];
                        double e = vs[3 * idx + i] + dv[3 * idx + i];
                        vm[i] += wt * u;
                        ve[i] += wt * e;
                        vd[i] += wt * dv[3 * idx + i];
                        for (int j = 0; j < 3; j++) {
                            Bm[3 * i + j] += wt * u * d[j];
                            Be[3 * i + j] += wt * e * d[j];
                            Bd[3 * i + j] += wt * dv[3 * idx + i] * d[j];
                        }
                    }
                }
        for (int i = 0; i < 3; i++) x[i] += T * vm[i];
        double M[9];
        for (int i = 0; i < 9; i++) M[i] = (i % 4 == 0 ? 1.0 : 0.0) + T * D * Bm[i];
        matmul(M, F, F);
        if (s->model == 2) {
            double c = cbrt(det3(F));
            for (int i = 0; i < 9; i++) F[i] = i % 4 == 0 ? c : 0.0;
        } else {
            orc_return_map(s, F);
        }
        if (mode == 0) {
            for (int i = 0; i < 3; i++) v[i] = ve[i];
            for (int i = 0; i < 9; i++) C[i] = D * Be[i];
        } else {
            for (int i = 0; i < 3; i++) v[i] += vd[i];
            for (int i = 0; i < 9; i++) C[i] += D * Bd[i];
        }
    }
    return err;
}

/* n full substeps.  Work arrays: m [res^3], p and vg [res^3][3]. */
int orc_step(orc_scene *s, int n, double *gm, double *gp, double *vg)
{
    for (int it = 0; it < n; it++) {
        int e = orc_p2g(s, gm, gp);
        if (e) return e;
        orc_grid_op(s, gm, gp, vg);
        e = orc_g2p(s, vg);
        if (e) return e;
        orc_advance_colliders(s);
    }
    return 0;
}
