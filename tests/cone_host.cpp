// Host build of the solver's FP64 cone polish (the header the GPU kernels
// use), for CPU tests: solve one grasp's QPs from an ADMM-form start state.
#include <cmath>
#include <cstring>

#include "../paper_2412_16490_amd/csrc/bodex_cone.h"

using namespace bodex;

namespace {

template <int MM, bool GAM>
int solve_one(const double* G, const double* mu, const double* bt, int m, double fmax, double gamma, double eps,
              const float* z0, double pull, double t0, double gap, double growth, double loose, int max_newton, double* x_out,
              int* newton) {
    constexpr int NV = 3 * MM;
    ConeData<MM, const double*, GAM> D;
    D.G = G;
    D.mu = mu;
    for (int r = 0; r < 6; ++r) D.bt[r] = bt[r];
    D.m = m;
    D.fmax = fmax;
    D.gamma = gamma;
    D.eps = eps;
    double fb[NV] = {}, db[NV] = {}, tb[NV] = {}, rb[NV] = {};
    const ConeWork<LaneVec> W(LaneVec{fb, 1}, LaneVec{db, 1}, LaneVec{tb, 1}, LaneVec{rb, 1});
    cone_start<MM>(D, [&](int r) { return double(z0[r]); }, pull, W);
    const ConePolishOut po = cone_polish<MM>(D, t0, gap, growth, loose, max_newton, W);
    for (int c = 0; c < NV; ++c) x_out[c] = c < 3 * m ? fb[c] : 0.0;
    *newton = po.newton;
    return po.status;
}

}  // namespace

extern "C" {

// Projection of one contact force onto the truncated cone as the solver
// computes it; returns the region.
int host_cone_project(double a, double t2, double t3, double mu, double fmax, double* z) {
    return cone_project<double>(a, t2, t3, mu, fmax, z);
}

// Solve s QPs of one grasp with m <= 5 contacts from ADMM-form points.
// p, n: [m][3]; mu: [m]; t: [s][6]; z0: [s][16] cone ADMM-form z (rows
// 3i..3i+2); x: [s][15].  Returns the number of QPs not accepted.
int host_cone_polish_grasp(int m, const double* p, const double* n, const double* mu, const double* t, int s,
                           double kappa, double beta, double eps, double fmax, double gamma, const float* z0,
                           double pull, double t0, double gap, double growth, double loose, int max_newton, double* x,
                           int* status, int* newton) {
    constexpr int MM = 5, NV = 15;
    double G[6 * NV] = {};
    double muv[MM] = {};
    for (int i = 0; i < m; ++i) {
        grasp_columns<double, NV>(p + 3 * i, n + 3 * i, kappa, i, G);
        muv[i] = mu[i];
    }
    int bad = 0;
    for (int j = 0; j < s; ++j) {
        double bt[6];
        for (int r = 0; r < 6; ++r) bt[r] = beta * t[6 * j + r];
        status[j] = gamma > 0.0 ? solve_one<MM, true>(G, muv, bt, m, fmax, gamma, eps, z0 + 16 * j, pull, t0, gap,
                                                       growth, loose, max_newton, x + NV * j, newton + j)
                                : solve_one<MM, false>(G, muv, bt, m, fmax, gamma, eps, z0 + 16 * j, pull, t0, gap,
                                                        growth, loose, max_newton, x + NV * j, newton + j);
        bad += status[j] != 0;
    }
    return bad;
}

}  // extern "C"
