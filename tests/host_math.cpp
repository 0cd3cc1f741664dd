// Host build of the HIP path's FP32 material routines (test harness only):
// exposes the stress, return-map and fluid updates of mpm_math.hpp to the
// CPU tests, which compare them with the FP64 oracle on random deformation
// gradients.  Built with hipcc for the host only (no device code).
#include "../paper_2302_04659_amd/csrc/mpm_math.hpp"

extern "C" void host_material(const float *F, int n, int model, int plastic, float mu, float la, float yield_eps,
                              float *Fout, float *tau, int *bad)
{
    mpm::Material m{model, plastic, mu, la, yield_eps};
    for (int p = 0; p < n; p++) {
        float G[9], Gn[9];
        for (int e = 0; e < 9; e++) G[e] = F[9 * p + e] - (e % 4 == 0 ? 1.0f : 0.0f);
        int b = 0;
        if (model == 0) {
            mpm::tau_neo_hookean(G, mu, la, tau + 9 * p, b);
            for (int e = 0; e < 9; e++) Gn[e] = G[e];
        } else if (model == 2) {
            mpm::fluid_update(G, m, Gn, tau + 9 * p, b);
        } else {
            mpm::hencky_update(G, m, Gn, tau + 9 * p, b);
        }
        for (int e = 0; e < 9; e++) Fout[9 * p + e] = Gn[e] + (e % 4 == 0 ? 1.0f : 0.0f);
        bad[p] = b;
    }
}

// Both Hencky paths on the same states: the elastic series (applied[p] = 1
// when it took the state) and the eigen-decomposition.
extern "C" void host_hencky_paths(const float *F, int n, int plastic, float mu, float la, float yield_eps,
                                  float *tau_series, float *tau_eigen, int *applied)
{
    mpm::Material m{1, plastic, mu, la, yield_eps};
    for (int p = 0; p < n; p++) {
        float G[9], Gn[9];
        for (int e = 0; e < 9; e++) G[e] = F[9 * p + e] - (e % 4 == 0 ? 1.0f : 0.0f);
        int b = 0;
        for (int e = 0; e < 9; e++) tau_series[9 * p + e] = 0.0f;
        applied[p] = mpm::hencky_elastic_series(G, m, Gn, tau_series + 9 * p);
        mpm::hencky_eigen(G, m, Gn, tau_eigen + 9 * p, b);
    }
}
