// Device math of the MLS-MPM substep for gfx950 (FP32).
//
// Quadratic B-spline weights and APIC transfer (MLS-MPM, the method the
// paper's soft-body solver follows, Sec. 3), neo-Hookean and Hencky
// elasticity with a von Mises return map (App. D.3, Table "tab:mpm_param"),
// analytic box / capsule SDFs (Sec. 3).
//
// Numerical design: the deformation gradient is carried as G = F - I and the
// Hencky model is evaluated from the eigen-decomposition of F^T F - I =
// G + G^T + G^T G, so log strains come from log1p of small numbers and keep
// their relative precision near F = I (an FP32 SVD of F itself loses it).
// With F^T F = V S^2 V^T and U = F V S^-1 (S signed, last value negative when
// det F < 0):
//   tau   = U diag(d) U^T            = F V diag(d_k / S_k^2) V^T F^T
//   F_new = U exp(eps_new) V^T        = F V diag(exp(eps_new,k) / S_k) V^T
// so neither U nor an SVD of F is formed.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include "mpm_types.hpp"

namespace mpm {

#define MPM_HD __host__ __device__ __forceinline__

MPM_HD float frcp(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}

MPM_HD float frsqrt(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rsqf(x);
#else
    return 1.0f / sqrtf(x);
#endif
}

MPM_HD float fsqrt(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_sqrtf(x);
#else
    return sqrtf(x);
#endif
}

// ln(1 + x) for x > -1.  |x| <= 1/4: 2 atanh(s), s = x / (2 + x), odd series
// to s^9 (truncation < 3e-11); otherwise the hardware log2.  Relative error
// stays at a few ulp near x = 0, where the log strains live.
MPM_HD float flog1p(float x)
{
    if (fabsf(x) <= 0.25f) {
        float s = x * frcp(2.0f + x);
        s = fmaf(fmaf(-s, 2.0f + x, x), frcp(2.0f + x), s);   // one Newton correction of the quotient
        float s2 = s * s;
        float p = fmaf(s2, 1.0f / 9.0f, 1.0f / 7.0f);
        p = fmaf(s2, p, 1.0f / 5.0f);
        p = fmaf(s2, p, 1.0f / 3.0f);
        p = fmaf(s2, p, 1.0f);
        return 2.0f * s * p;
    }
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_logf(1.0f + x) * 0.6931471805599453f;
#else
    return logf(1.0f + x);
#endif
}

// e^x - 1.  |x| <= 1/4: Taylor series to x^8 (truncation < 1e-11); otherwise
// the hardware exp2.
MPM_HD float fexpm1(float x)
{
    if (fabsf(x) <= 0.25f) {
        float p = fmaf(x, 1.0f / 40320.0f, 1.0f / 5040.0f);
        p = fmaf(x, p, 1.0f / 720.0f);
        p = fmaf(x, p, 1.0f / 120.0f);
        p = fmaf(x, p, 1.0f / 24.0f);
        p = fmaf(x, p, 1.0f / 6.0f);
        p = fmaf(x, p, 0.5f);
        p = fmaf(x, p, 1.0f);
        return x * p;
    }
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_exp2f(x * 1.4426950408889634f) - 1.0f;
#else
    return expf(x) - 1.0f;
#endif
}

// ---------------------------------------------------------------- Morton order
MPM_HD uint32_t spread3(uint32_t x)
{
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000FFu;
    x = (x | (x << 8)) & 0x0300F00Fu;
    x = (x | (x << 4)) & 0x030C30C3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

MPM_HD uint32_t compact3(uint32_t x)
{
    x &= 0x09249249u;
    x = (x ^ (x >> 2)) & 0x030C30C3u;
    x = (x ^ (x >> 4)) & 0x0300F00Fu;
    x = (x ^ (x >> 8)) & 0x030000FFu;
    x = (x ^ (x >> 16)) & 0x000003FFu;
    return x;
}

MPM_HD uint32_t morton3(uint32_t x, uint32_t y, uint32_t z)
{
    return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

// ---------------------------------------------------------------- B-spline
// Weights of nodes base, base+1, base+2 for fractional offset f in [0.5, 1.5).
MPM_HD void bspline_w(float f, float w[3])
{
    float a = 1.5f - f, b = f - 1.0f, c = f - 0.5f;
    w[0] = 0.5f * a * a;
    w[1] = 0.75f - b * b;
    w[2] = 0.5f * c * c;
}

// ---------------------------------------------------------------- 3x3 symmetric eigen
// Cyclic Jacobi on a symmetric matrix held as (a00, a11, a22, a01, a02, a12).
// On return the diagonal holds the eigenvalues and V (row-major, columns =
// eigenvectors) the rotation.  Three sweeps of three rotations give the
// Hencky stress to ~4e-6 relative (four: ~8e-7) for log strains up to 0.3.
#ifndef MPM_JACOBI_SWEEPS
#define MPM_JACOBI_SWEEPS 3
#endif
#ifndef MPM_JACOBI_APPROX
#define MPM_JACOBI_APPROX 0
#endif
struct Sym3 {
    float a00, a11, a22, a01, a02, a12;
};

MPM_HD void jacobi_rot(float &app, float &aqq, float &apq, float &arp, float &arq, float *V, int p, int q)
{
#if MPM_JACOBI_APPROX
    // Approximate Givens rotation (quaternion half-angle form, one rsqrt):
    // the half-angle (ch, sh) comes from the 2x2 block, clamped to pi/8 where
    // the first-order estimate is poor; c = ch^2 - sh^2, s = 2 ch sh.
    float ch = 2.0f * (app - aqq), sh = apq;
    const bool use = 5.8284271f * sh * sh < ch * ch;     // tan^2(pi/8) bound, 1/0.1716
    const float om = frsqrt(fmaf(ch, ch, sh * sh));
    ch = use ? om * ch : 0.92387953f;
    sh = use ? om * sh : 0.38268343f;
    float c = fmaf(ch, ch, -sh * sh), s = 2.0f * ch * sh;
    // rotation J with J_pp = c, J_pq = -s ... written as the same update as below
    s = -s;
    const float a_pp = app, a_qq = aqq, a_pq = apq;
    app = c * c * a_pp - 2.0f * c * s * a_pq + s * s * a_qq;
    aqq = s * s * a_pp + 2.0f * c * s * a_pq + c * c * a_qq;
    apq = (c * c - s * s) * a_pq + c * s * (a_pp - a_qq);
#else
    // t = tan of the rotation angle, the root of t^2 + 2 zeta t - 1 = 0 of
    // smaller magnitude, zeta = (aqq - app) / (2 apq), written with d = aqq - app
    // as t = sgn(d) 2 apq / (|d| + sqrt(d^2 + 4 apq^2)): one square root and
    // one reciprocal.
    float t = 0.0f;
    if (apq != 0.0f) {
        const float d = aqq - app;
        const float ad = fabsf(d);
        const float den = ad + fsqrt(fmaf(d, d, 4.0f * apq * apq));
        t = den > 0.0f ? 2.0f * apq * frcp(den) : copysignf(1.0f, apq);   // den = 0: d = 0 and apq^2 underflows
        if (d < 0.0f) t = -t;
    }
    float c = frsqrt(fmaf(t, t, 1.0f));
    float s = t * c;
    app = fmaf(-t, apq, app);
    aqq = fmaf(t, apq, aqq);
    apq = 0.0f;
#endif
    float rp = arp, rq = arq;
    arp = c * rp - s * rq;
    arq = s * rp + c * rq;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        float vp = V[3 * k + p], vq = V[3 * k + q];
        V[3 * k + p] = c * vp - s * vq;
        V[3 * k + q] = s * vp + c * vq;
    }
}

MPM_HD void sym_eig(Sym3 &a, float V[9])
{
#pragma unroll
    for (int i = 0; i < 9; i++) V[i] = (i % 4 == 0) ? 1.0f : 0.0f;
#pragma unroll
    for (int sweep = 0; sweep < MPM_JACOBI_SWEEPS; sweep++) {
        jacobi_rot(a.a00, a.a11, a.a01, a.a02, a.a12, V, 0, 1);   // r = 2: a20 = a02, a21 = a12
        jacobi_rot(a.a00, a.a22, a.a02, a.a01, a.a12, V, 0, 2);   // r = 1: a10 = a01, a12
        jacobi_rot(a.a11, a.a22, a.a12, a.a01, a.a02, V, 1, 2);   // r = 0: a01, a02
    }
}

// ---------------------------------------------------------------- constitutive models
// All matrices row-major [9].  G = F - I.

MPM_HD float det_minus_one(const float *G)
{
    // det(I + G) - 1 = tr G + (tr G^2 ... ) expanded to keep precision near G = 0
    float tr = G[0] + G[4] + G[8];
    float m2 = (G[0] * G[4] - G[1] * G[3]) + (G[0] * G[8] - G[2] * G[6]) + (G[4] * G[8] - G[5] * G[7]);
    float d3 = G[0] * (G[4] * G[8] - G[5] * G[7]) - G[1] * (G[3] * G[8] - G[5] * G[6]) +
               G[2] * (G[3] * G[7] - G[4] * G[6]);
    return tr + m2 + d3;
}

// Neo-Hookean Kirchhoff stress: mu (F F^T - I) + lambda ln(J) I.
MPM_HD void tau_neo_hookean(const float *G, float mu, float la, float tau[9], int &bad)
{
    float jm1 = det_minus_one(G);
    bad |= !(jm1 > -1.0f);
    float lnJ = flog1p(jm1);
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = i; j < 3; j++) {
            // F F^T - I = G + G^T + G G^T
            float ggt = G[3 * i] * G[3 * j] + G[3 * i + 1] * G[3 * j + 1] + G[3 * i + 2] * G[3 * j + 2];
            float v = mu * (G[3 * i + j] + G[3 * j + i] + ggt) + (i == j ? la * lnJ : 0.0f);
            tau[3 * i + j] = v;
            tau[3 * j + i] = v;
        }
}

struct Material {
    int model, plastic;
    float mu, la, yield_eps;
};

// tau = F M F^T for symmetric M, F = I + G (row-major).
MPM_HD void tau_from_M(const float *G, const float *M, float tau[9])
{
    float FM[9];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            float acc = M[3 * i + j];
#pragma unroll
            for (int k = 0; k < 3; k++) acc = fmaf(G[3 * i + k], M[3 * k + j], acc);
            FM[3 * i + j] = acc;
        }
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = i; j < 3; j++) {
            float acc = FM[3 * i + j];
#pragma unroll
            for (int k = 0; k < 3; k++) acc = fmaf(FM[3 * i + k], G[3 * j + k], acc);
            tau[3 * i + j] = acc;
            tau[3 * j + i] = acc;
        }
}

// Hencky elasticity with an optional von Mises return map through the
// eigen-decomposition of F^T F (any state).  Gt is the trial displacement
// gradient; Gout receives the projected one, tau the Kirchhoff stress of Gout.
// Returns 1 if the particle yielded.
MPM_HD int hencky_eigen(const float *Gt, const Material &mat, float *Gout, float tau[9], int &bad)
{
    const float SMIN = 1e-6f;
    Sym3 s;   // C - I = G + G^T + G^T G
    s.a00 = 2.0f * Gt[0] + (Gt[0] * Gt[0] + Gt[3] * Gt[3] + Gt[6] * Gt[6]);
    s.a11 = 2.0f * Gt[4] + (Gt[1] * Gt[1] + Gt[4] * Gt[4] + Gt[7] * Gt[7]);
    s.a22 = 2.0f * Gt[8] + (Gt[2] * Gt[2] + Gt[5] * Gt[5] + Gt[8] * Gt[8]);
    s.a01 = Gt[1] + Gt[3] + (Gt[0] * Gt[1] + Gt[3] * Gt[4] + Gt[6] * Gt[7]);
    s.a02 = Gt[2] + Gt[6] + (Gt[0] * Gt[2] + Gt[3] * Gt[5] + Gt[6] * Gt[8]);
    s.a12 = Gt[5] + Gt[7] + (Gt[1] * Gt[2] + Gt[4] * Gt[5] + Gt[7] * Gt[8]);
    float V[9];
    sym_eig(s, V);
    float lam[3] = {s.a00, s.a11, s.a22};
    float jm1 = det_minus_one(Gt);
    bad |= !(jm1 == jm1);
    // the smallest singular value carries the sign of det F
    int kmin = lam[0] <= lam[1] ? (lam[0] <= lam[2] ? 0 : 2) : (lam[1] <= lam[2] ? 1 : 2);
    float sig2[3], eps[3], sgn[3];
    int clamp[3];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        sig2[k] = 1.0f + lam[k];
        sgn[k] = (k == kmin && jm1 < -1.0f) ? -1.0f : 1.0f;
        clamp[k] = (sgn[k] < 0.0f) || !(sig2[k] >= SMIN * SMIN);
        eps[k] = clamp[k] ? -13.815510557964274f : 0.5f * flog1p(lam[k]);   // ln(1e-6)
    }
    float tr = eps[0] + eps[1] + eps[2];
    float mean = tr * (1.0f / 3.0f);
    float dv[3] = {eps[0] - mean, eps[1] - mean, eps[2] - mean};
    float nd = fsqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    float dg = nd - mat.yield_eps;
    int yielded = mat.plastic && dg > 0.0f;
    float en[3] = {eps[0], eps[1], eps[2]};
#pragma unroll
    for (int i = 0; i < 9; i++) Gout[i] = Gt[i];
    if (yielded) {
        float r = dg * frcp(nd);
        float q[3];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            en[k] = eps[k] - r * dv[k];
            float sk = sgn[k] * fsqrt(fmaxf(sig2[k], 0.0f));
            q[k] = clamp[k] ? (fexpm1(en[k]) + 1.0f) * frcp(sk) - 1.0f : fexpm1(en[k] - eps[k]);
        }
        // F_new = F (I + Q), Q = V diag(q) V^T  ->  G_new = G + Q + G Q
        float Q[9];
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++)
                Q[3 * i + j] = V[3 * i] * q[0] * V[3 * j] + V[3 * i + 1] * q[1] * V[3 * j + 1] +
                               V[3 * i + 2] * q[2] * V[3 * j + 2];
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++)
                Gout[3 * i + j] = Gt[3 * i + j] + Q[3 * i + j] +
                                  (Gt[3 * i] * Q[j] + Gt[3 * i + 1] * Q[3 + j] + Gt[3 * i + 2] * Q[6 + j]);
    }
    // tau = U diag(d) U^T with U = F V S^-1 of the trial F (the return map
    // keeps U and V): tau = F M F^T, M = V diag(d_k / S_k^2) V^T.
    float trn = en[0] + en[1] + en[2];
    float dk[3];
#pragma unroll
    for (int k = 0; k < 3; k++) dk[k] = (2.0f * mat.mu * en[k] + mat.la * trn) * frcp(fmaxf(sig2[k], SMIN * SMIN));
    float M[9];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++)
            M[3 * i + j] = V[3 * i] * dk[0] * V[3 * j] + V[3 * i + 1] * dk[1] * V[3 * j + 1] +
                           V[3 * i + 2] * dk[2] * V[3 * j + 2];
    tau_from_M(Gt, M, tau);
    return yielded;
}

// Symmetric 3x3 matrices as (00, 11, 22, 01, 02, 12).  The product of two
// that commute (functions of one symmetric matrix) is symmetric: its six
// entries.
MPM_HD void sym_mul(const float a[6], const float b[6], float c[6])
{
    c[0] = fmaf(a[0], b[0], fmaf(a[3], b[3], a[4] * b[4]));
    c[1] = fmaf(a[3], b[3], fmaf(a[1], b[1], a[5] * b[5]));
    c[2] = fmaf(a[4], b[4], fmaf(a[5], b[5], a[2] * b[2]));
    c[3] = fmaf(a[0], b[3], fmaf(a[3], b[1], a[4] * b[5]));
    c[4] = fmaf(a[0], b[4], fmaf(a[3], b[5], a[4] * b[2]));
    c[5] = fmaf(a[3], b[4], fmaf(a[1], b[5], a[5] * b[2]));
}

#ifndef MPM_HENCKY_SERIES
#define MPM_HENCKY_SERIES 1
#endif

// Hencky stress of a state that stays elastic, without an eigen-decomposition.
// With b = F F^T and the spatial log strain e = ln(b) / 2, the Kirchhoff
// stress is tau = 2 mu e + lambda tr(e) I (the eigen path's U diag(d) U^T).
// ln b = 2 atanh(Z) with Z = (b - I)(b + I)^-1 (functions of b, so they
// commute), hence e = Z + Z^3/3 + Z^5/5 + Z^7/7 + Z^9/9 + ...; while
// |b - I|_F <= 0.35 the eigenvalues of Z stay within 0.35 / 1.65 and the first
// term left out is below 4e-9.  The deviatoric norm of e is that of the
// principal log strains, so the yield test is the eigen path's.
// hencky_series_strain: e (symmetric, as sym_mul's six entries) and 1 when
// the series applies (det F > 1/2, |b - I|_F <= 0.35, no yield), else 0.
MPM_HD int hencky_series_strain(const float *G, const Material &mat, float e[6])
{
    // b - I = G + G^T + G G^T
    float s[6];
    s[0] = 2.0f * G[0] + (G[0] * G[0] + G[1] * G[1] + G[2] * G[2]);
    s[1] = 2.0f * G[4] + (G[3] * G[3] + G[4] * G[4] + G[5] * G[5]);
    s[2] = 2.0f * G[8] + (G[6] * G[6] + G[7] * G[7] + G[8] * G[8]);
    s[3] = G[1] + G[3] + (G[0] * G[3] + G[1] * G[4] + G[2] * G[5]);
    s[4] = G[2] + G[6] + (G[0] * G[6] + G[1] * G[7] + G[2] * G[8]);
    s[5] = G[5] + G[7] + (G[3] * G[6] + G[4] * G[7] + G[5] * G[8]);
    const float nb2 = s[0] * s[0] + s[1] * s[1] + s[2] * s[2] + 2.0f * (s[3] * s[3] + s[4] * s[4] + s[5] * s[5]);
    // (b + I)^-1 = (2 I + s)^-1 by its adjugate
    const float a = 2.0f + s[0], d = 2.0f + s[1], f = 2.0f + s[2];
    float inv[6];
    inv[0] = d * f - s[5] * s[5];
    inv[1] = a * f - s[4] * s[4];
    inv[2] = a * d - s[3] * s[3];
    inv[3] = s[4] * s[5] - s[3] * f;
    inv[4] = s[3] * s[5] - s[4] * d;
    inv[5] = s[3] * s[4] - a * s[5];
    const float idet = frcp(a * inv[0] + s[3] * inv[3] + s[4] * inv[4]);
#pragma unroll
    for (int k = 0; k < 6; k++) inv[k] *= idet;
    float z[6], z2[6], p[6], q[6];
    sym_mul(s, inv, z);
    sym_mul(z, z, z2);
    // p = I + z2/3 + z2^2/5 + z2^3/7 + z2^4/9 (Horner in z2)
#pragma unroll
    for (int k = 0; k < 6; k++) p[k] = z2[k] * (1.0f / 9.0f) + (k < 3 ? 1.0f / 7.0f : 0.0f);
    sym_mul(z2, p, q);
#pragma unroll
    for (int k = 0; k < 6; k++) p[k] = q[k] + (k < 3 ? 1.0f / 5.0f : 0.0f);
    sym_mul(z2, p, q);
#pragma unroll
    for (int k = 0; k < 6; k++) p[k] = q[k] + (k < 3 ? 1.0f / 3.0f : 0.0f);
    sym_mul(z2, p, q);
#pragma unroll
    for (int k = 0; k < 6; k++) p[k] = q[k] + (k < 3 ? 1.0f : 0.0f);
    sym_mul(z, p, e);
    const float mean = (e[0] + e[1] + e[2]) * (1.0f / 3.0f);
    const float d0 = e[0] - mean, d1 = e[1] - mean, d2 = e[2] - mean;
    const float nd2 = d0 * d0 + d1 * d1 + d2 * d2 + 2.0f * (e[3] * e[3] + e[4] * e[4] + e[5] * e[5]);
    return nb2 <= 0.1225f && det_minus_one(G) > -0.5f && !(mat.plastic && nd2 > mat.yield_eps * mat.yield_eps);
}

// tau = 2 mu e + lambda tr(e) I.
MPM_HD void hencky_tau_of_strain(const float e[6], const Material &mat, float tau[9])
{
    const float tm = 2.0f * mat.mu, tl = mat.la * (e[0] + e[1] + e[2]);
    tau[0] = fmaf(tm, e[0], tl);
    tau[4] = fmaf(tm, e[1], tl);
    tau[8] = fmaf(tm, e[2], tl);
    tau[1] = tau[3] = tm * e[3];
    tau[2] = tau[6] = tm * e[4];
    tau[5] = tau[7] = tm * e[5];
}

// The series path of one state (host tests): 1 and tau if it applies.
MPM_HD int hencky_elastic_series(const float *G, const Material &mat, float *Gout, float tau[9])
{
    float e[6];
    if (!hencky_series_strain(G, mat, e)) return 0;
    hencky_tau_of_strain(e, mat, tau);
#pragma unroll
    for (int i = 0; i < 9; i++) Gout[i] = G[i];
    return 1;
}

// Hencky elasticity with an optional von Mises return map.  Gt is the trial
// displacement gradient; Gout receives the projected one (may alias Gt only
// through a copy made by the caller), tau the Kirchhoff stress of Gout.
// Returns 1 if the particle yielded.  States near the identity that stay
// elastic take the series above, on the GPU when every lane of the wave
// qualifies (one path per wave); the rest the eigen-decomposition of F^T F.
MPM_HD int hencky_update(const float *Gt, const Material &mat, float *Gout, float tau[9], int &bad)
{
#if MPM_HENCKY_SERIES
    float e[6];
    int ok = hencky_series_strain(Gt, mat, e);
#if defined(__HIP_DEVICE_COMPILE__)
    ok = __ballot(ok) == __ballot(1);
#endif
    // both paths fill the same locals, written out once (stores of the two
    // branches merged into one would keep the arrays out of registers)
    float tv[9], gv[9];
    int yielded = 0;
    if (ok) {
        hencky_tau_of_strain(e, mat, tv);
#pragma unroll
        for (int i = 0; i < 9; i++) gv[i] = Gt[i];
    } else {
        yielded = hencky_eigen(Gt, mat, gv, tv, bad);
    }
#pragma unroll
    for (int i = 0; i < 9; i++) {
        tau[i] = tv[i];
        Gout[i] = gv[i];
    }
    return yielded;
#else
    return hencky_eigen(Gt, mat, Gout, tau, bad);
#endif
}

// Weakly compressible fluid: Tait pressure p(J) = (K / 7) (J^-7 - 1) with the
// bulk modulus K = lambda + 2 mu / 3, Kirchhoff stress tau = -J p(J) I, and the
// state reduced to J^(1/3) I (volume change only).  With L = ln J from
// log1p(J - 1): J^(1/3) - 1 = expm1(L / 3) and J^-7 - 1 = expm1(-7 L), so
// small volume changes keep their relative precision.
MPM_HD void fluid_update(const float *Gt, const Material &mat, float *Gout, float tau[9], int &bad)
{
    const float jm1 = det_minus_one(Gt);
    bad |= !(jm1 > -1.0f);
    const float L = flog1p(jm1);
    const float g = fexpm1(L * (1.0f / 3.0f));
    const float K = mat.la + (2.0f / 3.0f) * mat.mu;
    const float t = -(1.0f + jm1) * (K * (1.0f / 7.0f)) * fexpm1(-7.0f * L);
#pragma unroll
    for (int i = 0; i < 9; i++) {
        Gout[i] = (i % 4 == 0) ? g : 0.0f;
        tau[i] = (i % 4 == 0) ? t : 0.0f;
    }
}

// Stress of a state without any return map (a state handed in from outside).
MPM_HD void stress_of(const float *G, const Material &mat, float tau[9], int &bad)
{
    if (mat.model == 0) {
        tau_neo_hookean(G, mat.mu, mat.la, tau, bad);
        return;
    }
    if (mat.model == 2) {
        float Gc[9];
        fluid_update(G, mat, Gc, tau, bad);   // the stress depends on det F only
        return;
    }
    Material m2 = mat;
    m2.plastic = 0;
    float Gc[9];
    hencky_update(G, m2, Gc, tau, bad);
}

// ---------------------------------------------------------------- rotations and SDFs
MPM_HD void quat_to_mat(const float q[4], float R[9])
{
    float w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z); R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z); R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y); R[7] = 2 * (y * z + w * x); R[8] = 1 - 2 * (x * x + y * y);
}

// q_k = exp(k dt w / 2) (x) q0
MPM_HD void quat_advance(const float q0[4], const float w[3], float tk, float q[4])
{
    float wn = sqrtf(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    if (wn == 0.0f) {
        q[0] = q0[0]; q[1] = q0[1]; q[2] = q0[2]; q[3] = q0[3];
        return;
    }
    float h = 0.5f * tk * wn;
    float sh = sinf(h) / wn, ch = cosf(h);
    float d[4] = {ch, sh * w[0], sh * w[1], sh * w[2]};
    q[0] = d[0] * q0[0] - d[1] * q0[1] - d[2] * q0[2] - d[3] * q0[3];
    q[1] = d[0] * q0[1] + d[1] * q0[0] + d[2] * q0[3] - d[3] * q0[2];
    q[2] = d[0] * q0[2] - d[1] * q0[3] + d[2] * q0[0] + d[3] * q0[1];
    q[3] = d[0] * q0[3] + d[1] * q0[2] - d[2] * q0[1] + d[3] * q0[0];
}

// Collider at one substep: world pose + rotation matrix.
struct ColliderNow {
    int type;
    float he[3], radius, half_length, friction;
    float c[3], R[9], v[3], w[3];
    int sdf_off, sdf_dims[3];
    float sdf_cell, sdf_origin[3];
};

MPM_HD void collider_at(const ColliderDev &cd, float tk, ColliderNow &cn)
{
    cn.type = cd.type;
    for (int a = 0; a < 3; a++) {
        cn.he[a] = cd.he[a];
        cn.c[a] = fmaf(tk, cd.vlin[a], cd.pos[a]);
        cn.v[a] = cd.vlin[a];
        cn.w[a] = cd.omega[a];
    }
    cn.radius = cd.radius;
    cn.half_length = cd.half_length;
    cn.friction = cd.friction;
    cn.sdf_off = cd.sdf_off;
    cn.sdf_cell = cd.sdf_cell;
    for (int a = 0; a < 3; a++) {
        cn.sdf_dims[a] = cd.sdf_dims[a];
        cn.sdf_origin[a] = cd.sdf_origin[a];
    }
    float q[4];
    quat_advance(cd.quat, cd.omega, tk, q);
    quat_to_mat(q, cn.R);
}

// Sampled SDF volume at body-frame point p: trilinear interpolant of the
// eight samples of the cell holding p, normal = normalised gradient of that
// interpolant (body +x where it vanishes); outside the brick no contact
// (a large positive distance).
MPM_HD float sdf_volume(const ColliderNow &c, const float *sdf, const float p[3], float nb[3])
{
    float f[3];
    int i0[3];
    nb[0] = 1.0f;
    nb[1] = 0.0f;
    nb[2] = 0.0f;
    const float ic = 1.0f / c.sdf_cell;
    for (int a = 0; a < 3; a++) {
        const float u = (p[a] - c.sdf_origin[a]) * ic;
        if (!(u >= 0.0f && u <= (float)(c.sdf_dims[a] - 1))) return 3.0e38f;
        i0[a] = (int)floorf(u);
        if (i0[a] > c.sdf_dims[a] - 2) i0[a] = c.sdf_dims[a] - 2;
        f[a] = u - (float)i0[a];
    }
    const int ny = c.sdf_dims[1], nz = c.sdf_dims[2];
    const float *s0 = sdf + c.sdf_off + ((long long)i0[0] * ny + i0[1]) * nz + i0[2];
    const long long sx = (long long)ny * nz, sy = nz;
    const float s000 = s0[0], s001 = s0[1], s010 = s0[sy], s011 = s0[sy + 1];
    const float s100 = s0[sx], s101 = s0[sx + 1], s110 = s0[sx + sy], s111 = s0[sx + sy + 1];
    // interpolate along z, then y, then x; the gradient from the same partial sums
    const float a00 = s000 + f[2] * (s001 - s000), a01 = s010 + f[2] * (s011 - s010);
    const float a10 = s100 + f[2] * (s101 - s100), a11 = s110 + f[2] * (s111 - s110);
    const float b0 = a00 + f[1] * (a01 - a00), b1 = a10 + f[1] * (a11 - a10);
    const float phi = b0 + f[0] * (b1 - b0);
    const float gx = b1 - b0;
    const float gy = (a01 - a00) + f[0] * ((a11 - a10) - (a01 - a00));
    const float dz0 = (s001 - s000) + f[1] * ((s011 - s010) - (s001 - s000));
    const float dz1 = (s101 - s100) + f[1] * ((s111 - s110) - (s101 - s100));
    const float gz = dz0 + f[0] * (dz1 - dz0);
    const float len2 = gx * gx + gy * gy + gz * gz;
    if (len2 > 0.0f) {
        const float il = 1.0f / sqrtf(len2);
        nb[0] = gx * il;
        nb[1] = gy * il;
        nb[2] = gz * il;
    }
    return phi;
}

// Signed distance and outward unit normal (world).  Box interior: nearest
// face, ties to the lowest axis, + before -.  Capsule on its axis: body +x.
// sdf: the context's buffer of SDF-volume samples (read by type 2 only).
MPM_HD float sdf_eval(const ColliderNow &c, const float x[3], float n[3], const float *sdf)
{
    float r[3] = {x[0] - c.c[0], x[1] - c.c[1], x[2] - c.c[2]};
    float p[3];
    for (int a = 0; a < 3; a++) p[a] = c.R[a] * r[0] + c.R[3 + a] * r[1] + c.R[6 + a] * r[2];   // R^T r
    float nb[3] = {0.0f, 0.0f, 0.0f};
    float phi;
    if (c.type == 2) {
        phi = sdf_volume(c, sdf, p, nb);
    } else if (c.type == 0) {
        float q[3], out = 0.0f;
        for (int a = 0; a < 3; a++) {
            q[a] = fabsf(p[a]) - c.he[a];
            if (q[a] > 0.0f) out += q[a] * q[a];
        }
        if (out > 0.0f) {
            phi = sqrtf(out);
            float ip = 1.0f / phi;
            for (int a = 0; a < 3; a++) nb[a] = q[a] > 0.0f ? copysignf(q[a] * ip, p[a] >= 0.0f ? 1.0f : -1.0f) : 0.0f;
        } else {
            int best = 0;
            if (q[1] > q[best]) best = 1;
            if (q[2] > q[best]) best = 2;
            phi = q[best];
            nb[best] = p[best] >= 0.0f ? 1.0f : -1.0f;
        }
    } else {
        float t = fminf(fmaxf(p[1], -c.half_length), c.half_length);
        float d[3] = {p[0], p[1] - t, p[2]};
        float len = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        phi = len - c.radius;
        if (len > 0.0f) {
            float il = 1.0f / len;
            nb[0] = d[0] * il; nb[1] = d[1] * il; nb[2] = d[2] * il;
        } else {
            nb[0] = 1.0f;
        }
    }
    for (int a = 0; a < 3; a++) n[a] = c.R[3 * a] * nb[0] + c.R[3 * a + 1] * nb[1] + c.R[3 * a + 2] * nb[2];
    return phi;
}

// Grid-node contact: separating test and Coulomb friction (in place).
MPM_HD int collide_node(const ColliderNow &c, const float xi[3], float v[3], const float *sdf)
{
    float n[3];
    float phi = sdf_eval(c, xi, n, sdf);
    float r[3] = {xi[0] - c.c[0], xi[1] - c.c[1], xi[2] - c.c[2]};
    float vc[3] = {c.v[0] + (c.w[1] * r[2] - c.w[2] * r[1]),
                   c.v[1] + (c.w[2] * r[0] - c.w[0] * r[2]),
                   c.v[2] + (c.w[0] * r[1] - c.w[1] * r[0])};
    float u[3] = {v[0] - vc[0], v[1] - vc[1], v[2] - vc[2]};
    float un = u[0] * n[0] + u[1] * n[1] + u[2] * n[2];
    if (!(phi < 0.0f && un < 0.0f)) return 0;
    float ut[3] = {u[0] - un * n[0], u[1] - un * n[1], u[2] - un * n[2]};
    float lt = sqrtf(ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2]);
    float scale = 0.0f;
    if (!isinf(c.friction) && lt > 0.0f) scale = fmaxf(0.0f, 1.0f + c.friction * un / lt);
    for (int a = 0; a < 3; a++) v[a] = vc[a] + scale * ut[a];
    return 1;
}

}  // namespace mpm
