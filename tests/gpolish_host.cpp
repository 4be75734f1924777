// Host build of the chunked FP64 polish (the headers the GPU kernels use),
// for CPU tests: the one-lane polish runs a budget of factorisations and
// saves its state into a spill record, then the contact-parallel polish
// continues from the record with GS threads standing in for the GS lanes of
// a group (each group operation is a barrier plus a reduction in lane order,
// the same value in every thread).
#include <cstring>
#include <thread>
#include <type_traits>
#include <vector>

#include "../paper_2412_16490_amd/csrc/bodex_gpolish.h"
#include "host_team.h"

using namespace bodex;

namespace {

constexpr int MM = 5, NV = 15, GS = 8;

}  // namespace

extern "C" {

// Chunked polish of the s QPs of one grasp with m <= 5 contacts (beta = 1,
// fmax = 1, gamma = 0): the one-lane polish from the ADMM-form dual guess
// y0 [s][46] with a budget of `budget` factorisations; a QP not finished by
// then is saved to a record and finished by the contact-parallel polish.
// Outputs x [s][15], status [s], handed [s] (1 if the group finished it),
// counts [s][4] (factorisations, of which one-row changes, equality solves,
// one-row steps).  force_break: the first ratio test (in whichever kernel
// runs it) reports a breakdown.  shared_factor: the group keeps its 6x6
// factor and each lane its block of G in the memory-backed forms the GPU
// kernel uses (LdsStore; here each thread has its own copy of the factor,
// since host threads do not run in lockstep).
// Returns the number of QPs whose polish was not accepted.
int host_chunked_polish(int m, const double* p, const double* n, const double* mu, const double* t, int s,
                        double kappa, double eps, const float* y0, int budget, double* x, int* status,
                        int* handed, int* counts, int force_break, int shared_factor) {
    double G[6 * NV] = {};
    double muc[MM] = {};
    for (int i = 0; i < m; ++i) {
        grasp_columns<double, NV>(p + 3 * i, n + 3 * i, kappa, i, G);
        muc[i] = mu[i] * kC8;
    }
    int bad = 0;
    std::vector<double> dsp((3 * MM + 3) * 1);
    std::vector<int> isp(kSpInts * 1);
    SpillPtrs sp{dsp.data(), isp.data(), 1};
    for (int j = 0; j < s; ++j) {
        PolishData<MM, const double*, false> D;
        D.G = G;
        D.muc = muc;
        for (int r = 0; r < 6; ++r) D.bt[r] = t[6 * j + r];
        D.m = m;
        D.fmax = 1.0;
        D.gamma = 0.0;
        D.eps = eps;
        double xb[NV] = {}, zb[NV] = {};
        PolishWork<LaneVec> W{{xb, 1}, {zb, 1}};
        PolishState<MM> PS;
        PS.S.pc = LaneVec{nullptr, 1};
        polish_begin<MM>(D, y0 + 46 * j, PS);
        PS.budget = budget;
        if (force_break) PS.chg |= kChgBreakAny;
        do {
            while (!polish_advance<MM, decltype(D), LaneVec, true>(D, 200, W, PS)) {
            }
        } while (!polish_finish<MM>(D, W, PS));
        PolishOut po = PS.out;
        handed[j] = po.status == kPolishSuspended;
        if (handed[j]) {
            polish_save<MM>(PS, W.x, m, sp, 0, j, 0);
            Shared sh(GS);
            std::vector<std::thread> th;
            auto lane = [&](int l, auto tag) {
                using LS = decltype(tag);
                    HostTeam<GS> team{l, &sh};
                    GQP<MM, LS> Q;
                    double lbuf[21], gbuf[18];
                    if constexpr (std::is_same<LS, LdsStore>::value) {
                        Q.L.a.p = lbuf;
                        Q.L.a.stride = 1;
                        Q.G.p = gbuf;
                        Q.G.stride = 1;
                    }
                    Q.sub = l;
                    double p3[3] = {0.0, 0.0, 0.0}, n3[3] = {0.0, 0.0, 1.0}, mu1 = 0.5;
                    if (l < m) {
                        for (int q = 0; q < 3; ++q) {
                            p3[q] = p[3 * l + q];
                            n3[q] = n[3 * l + q];
                        }
                        mu1 = mu[l];
                    }
                    gpolish_load<MM>(team, Q, sp, 0, m, p3, n3, mu1, kappa, t + 6 * j, 1.0, eps);
                    do {
                        while (!gpolish_advance<MM>(team, Q, 200)) {
                        }
                    } while (!gpolish_finish<MM>(team, Q));
                    gpolish_store<MM>(team, Q, sp, 0);
            };
            for (int l = 0; l < GS; ++l) {
                if (shared_factor)
                    th.emplace_back([&, l] { lane(l, LdsStore{}); });
                else
                    th.emplace_back([&, l] { lane(l, RegStore{}); });
            }
            for (auto& h : th) h.join();
            for (int c = 0; c < NV; ++c) xb[c] = c < 3 * m ? sp.dv(c, 0) : 0.0;
            po.status = sp.iv(kSpStatus, 0);
            po.steps = sp.iv(kSpSteps, 0);
            po.updates = sp.iv(kSpUpdates, 0);
            po.eqps = sp.iv(kSpEqps, 0);
            po.moves = sp.iv(kSpMoves, 0);
            // the saved active set, reassembled by the group, equals each
            // contact's rows at the end
        }
        for (int c = 0; c < NV; ++c) x[NV * j + c] = c < 3 * m ? xb[c] : 0.0;
        status[j] = po.status;
        counts[4 * j] = po.steps;
        counts[4 * j + 1] = po.updates;
        counts[4 * j + 2] = po.eqps;
        counts[4 * j + 3] = po.moves;
        bad += po.status != 0;
    }
    return bad;
}

}  // extern "C"
