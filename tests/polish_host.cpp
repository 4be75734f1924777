// Host build of the solver's FP64 polish (the header the GPU kernels use),
// for CPU tests: solve one grasp's QPs from a given ADMM-form dual guess.
#include <cmath>
#include <cstring>

#include "../paper_2412_16490_amd/csrc/bodex_math.h"

using namespace bodex;

namespace {

template <int MM, bool GAM>
int solve_one(const double* G, const double* muc, const double* bt, int m, double fmax, double gamma, double eps,
              const float* y0, int max_steps, double* x_out, int* steps_out) {
    constexpr int NV = 3 * MM;
    PolishData<MM, const double*, GAM> D;
    D.G = G;
    D.muc = muc;
    for (int r = 0; r < 6; ++r) D.bt[r] = bt[r];
    D.m = m;
    D.fmax = fmax;
    D.gamma = gamma;
    D.eps = eps;
    double xb[NV] = {}, zb[NV] = {}, pcb[3 * MM] = {};
    PolishWork<LaneVec> W{{xb, 1}, {zb, 1}};
    PolishState<MM> PS;
    PS.S.pc = LaneVec{pcb, 1};
    const PolishOut po = polish_qp<MM>(D, y0, max_steps, W, PS);
    for (int c = 0; c < NV; ++c) x_out[c] = c < 3 * m ? xb[c] : 0.0;
    *steps_out = po.steps;
    return po.status;
}

}  // namespace

extern "C" {

// Row coefficients of facet k as the solver computes them.
void host_facet_cs(int k, double* c, double* s) { facet_cs(k, c, s); }

// Solve s QPs of one grasp with m <= 5 contacts.  p, n: [m][3]; mu: [m];
// t: [s][6]; y0: [s][46] ADMM-form duals (the warm guess); x: [s][15].
// Returns the number of QPs whose polish was not accepted.
int host_polish_grasp(int m, const double* p, const double* n, const double* mu, const double* t, int s,
                      double kappa, double beta, double eps, double fmax, double gamma, const float* y0,
                      int max_steps, double* x, int* status, int* steps) {
    constexpr int MM = 5, NV = 15;
    double G[6 * NV] = {};
    double muc[MM] = {};
    for (int i = 0; i < m; ++i) {
        grasp_columns<double, NV>(p + 3 * i, n + 3 * i, kappa, i, G);
        muc[i] = mu[i] * kC8;
    }
    int bad = 0;
    for (int j = 0; j < s; ++j) {
        double bt[6];
        for (int r = 0; r < 6; ++r) bt[r] = beta * t[6 * j + r];
        status[j] = gamma > 0.0 ? solve_one<MM, true>(G, muc, bt, m, fmax, gamma, eps, y0 + 46 * j, max_steps,
                                                       x + NV * j, steps + j)
                                : solve_one<MM, false>(G, muc, bt, m, fmax, gamma, eps, y0 + 46 * j, max_steps,
                                                        x + NV * j, steps + j);
        bad += status[j] != 0;
    }
    return bad;
}

}  // extern "C"
