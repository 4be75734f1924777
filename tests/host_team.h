// A group of GS lanes stood in for by GS host threads, for the CPU tests of
// the group-shaped polishes: every group operation is a barrier plus a
// reduction in lane order, so every thread gets the same value (the GPU's
// butterfly reductions also give every lane the same value, though summed in
// another order).
#pragma once

#include <atomic>
#include <cmath>
#include <thread>

namespace {

// GS threads of one group: shared slots and a spinning barrier with a
// generation count (acquire/release: what a thread wrote before the barrier
// is visible to every thread after it).
struct Shared {
    int n;
    std::atomic<int> waiting{0};
    std::atomic<long> gen{0};
    double d[8][32];
    int i[8][4];
    explicit Shared(int n_) : n(n_) {}
    void barrier() {
        const long g = gen.load(std::memory_order_acquire);
        if (waiting.fetch_add(1, std::memory_order_acq_rel) + 1 == n) {
            waiting.store(0, std::memory_order_relaxed);
            gen.store(g + 1, std::memory_order_release);
        } else {
            int spins = 0;
            while (gen.load(std::memory_order_acquire) == g)
                if (++spins > 256) std::this_thread::yield();
        }
    }
};

template <int GS>
struct HostTeam {
    int sub;
    Shared* S;
    double sum(double v) const {
        S->d[sub][0] = v;
        S->barrier();
        double r = 0.0;
        for (int l = 0; l < GS; ++l) r += S->d[l][0];
        S->barrier();
        return r;
    }
    template <int N>
    void sum(double (&v)[N]) const {
        static_assert(N <= 32, "slot size");
        for (int j = 0; j < N; ++j) S->d[sub][j] = v[j];
        S->barrier();
        for (int j = 0; j < N; ++j) {
            double r = 0.0;
            for (int l = 0; l < GS; ++l) r += S->d[l][j];
            v[j] = r;
        }
        S->barrier();
    }
    double max(double v) const {
        S->d[sub][0] = v;
        S->barrier();
        double r = S->d[0][0];
        for (int l = 1; l < GS; ++l) r = fmax(r, S->d[l][0]);
        S->barrier();
        return r;
    }
    void argmax(double& v, int& idx) const {
        S->d[sub][0] = v;
        S->i[sub][0] = idx;
        S->barrier();
        for (int l = 0; l < GS; ++l) {
            const double ov = S->d[l][0];
            const int oi = S->i[l][0];
            if (ov > v || (ov == v && unsigned(oi) < unsigned(idx))) {
                v = ov;
                idx = oi;
            }
        }
        S->barrier();
    }
    void argmin_frac(double& tn, double& td, int& idx) const {
        S->d[sub][0] = tn;
        S->d[sub][1] = td;
        S->i[sub][0] = idx;
        S->barrier();
        for (int l = 0; l < GS; ++l) {
            const double on = S->d[l][0], od = S->d[l][1];
            const int oi = S->i[l][0];
            const double a = on * td, b = tn * od;
            if (a < b || (a == b && unsigned(oi) < unsigned(idx))) {
                tn = on;
                td = od;
                idx = oi;
            }
        }
        S->barrier();
    }
    double bcast(double v, int src) const {
        S->d[sub][0] = v;
        S->barrier();
        const double r = S->d[src][0];
        S->barrier();
        return r;
    }
    int bcast(int v, int src) const {
        S->i[sub][0] = v;
        S->barrier();
        const int r = S->i[src][0];
        S->barrier();
        return r;
    }
    unsigned bor(unsigned v) const {
        S->i[sub][0] = int(v);
        S->barrier();
        unsigned r = 0u;
        for (int l = 0; l < GS; ++l) r |= unsigned(S->i[l][0]);
        S->barrier();
        return r;
    }
};

}  // namespace
