// bodex_gpolish.h -- the FP64 polish of one QP by a group of lanes, one lane
// per contact (contact-parallel), and the record that carries a polish from
// the one-lane kernel to this one.
//
// The method is the one-lane polish's (bodex_math.h: Goldfarb-Idnani dual
// active-set steps with per-contact closed-form null-space projectors and the
// 6x6 Woodbury factor of eps I6 + G Pi G^T, one-row changes of that factor,
// a KKT acceptance check and one retry on fresh factorisations), for the
// problem without the normal-sum row (gamma = 0).  What changes is the
// mapping: lane `sub` of a group of GS lanes owns contact `sub` -- its three
// force components, its nine rows, its active rows and its projector -- so
// every per-contact loop of the one-lane polish becomes one pass of the
// group, and every sum over contacts (G x, G Pi v, the 6x6 matrix, the most
// violated row, the ratio test, the acceptance check) a butterfly reduction
// over the group.  The 6x6 factor and the step's scalars are replicated in
// the group's lanes; butterfly sums are commutative pairwise additions, so
// every lane gets the same bits and the group's control flow stays uniform.
//
// It exists for latency: a lane-per-QP polish runs a QP's steps one contact
// after another, and the hardest QPs of a batch (several times the mean
// number of steps) set the time of the whole launch.  The solver runs the
// one-lane polish for a budget of factorisations and hands the QPs still
// unfinished to this kernel (polish_save / gpolish_load).
#pragma once

#include "bodex_math.h"

namespace bodex {

// ---------------------------------------------------------------------------
// Record of a suspended polish: structure of arrays over the record index k
// (capacity K).  Saved at a point where a factorisation is due, so neither
// the factor nor the step vector needs saving.
//   dsp [3 MM + 3][K]  x (FP64), then up, mup, lg
//   isp [kSpInts][K]   the fields below
// ---------------------------------------------------------------------------
enum SpillInt {
    kSpW = 0,     // QP index
    kSpG,         // its grasp
    kSpPpi,       // pending row
    kSpPpk,
    kSpMpi,       // row of the multipliers still to compute
    kSpMpk,
    kSpPhase,
    kSpMode,
    kSpNeedMult,
    kSpChg,
    kSpStep0,
    kSpStatus,
    kSpSteps,
    kSpUpdates,
    kSpEqps,
    kSpMoves,
    kSpPicks,
    kSpMask0,     // active rows, 4 x 32 bits (9 per contact)
    kSpMask1,
    kSpMask2,
    kSpMask3,
    kSpInts
};

struct SpillPtrs {
    double* d;
    int* i;
    int K;
    BODEX_FI double& dv(int f, int k) const { return d[size_t(f) * K + k]; }
    BODEX_FI int& iv(int f, int k) const { return i[size_t(f) * K + k]; }
};

template <class Mask>
BODEX_FI void mask_to_words(Mask m, unsigned w[4]) {
    w[0] = unsigned(m);
    w[1] = unsigned(m >> 32);
    if constexpr (sizeof(Mask) > 8) {
        w[2] = unsigned(m >> 64);
        w[3] = unsigned(m >> 96);
    } else {
        w[2] = w[3] = 0u;
    }
}

template <class Mask>
BODEX_FI Mask mask_from_words(const unsigned w[4]) {
    Mask m = Mask(w[0]) | (Mask(w[1]) << 32);
    if constexpr (sizeof(Mask) > 8) m |= (Mask(w[2]) << 64) | (Mask(w[3]) << 96);
    return m;
}

// One lane's suspended polish (the one-lane kernel) into record k.
template <int MM, class V>
BODEX_FI void polish_save(const PolishState<MM>& PS, const V& x, int m, const SpillPtrs& sp, int k, int w, int g) {
#pragma unroll 1
    for (int c = 0; c < 3 * MM; ++c) sp.dv(c, k) = c < 3 * m ? x[c] : 0.0;
    sp.dv(3 * MM, k) = PS.up;
    sp.dv(3 * MM + 1, k) = PS.mup;
    sp.dv(3 * MM + 2, k) = PS.lg;
    unsigned mw[4];
    mask_to_words(PS.S.mask, mw);
    sp.iv(kSpW, k) = w;
    sp.iv(kSpG, k) = g;
    sp.iv(kSpPpi, k) = PS.p.pi;
    sp.iv(kSpPpk, k) = PS.p.pk;
    sp.iv(kSpMpi, k) = PS.mp.pi;
    sp.iv(kSpMpk, k) = PS.mp.pk;
    sp.iv(kSpPhase, k) = PS.phase;
    sp.iv(kSpMode, k) = PS.mode;
    sp.iv(kSpNeedMult, k) = PS.need_mult ? 1 : 0;
    sp.iv(kSpChg, k) = PS.chg;
    sp.iv(kSpStep0, k) = PS.step0;
    sp.iv(kSpStatus, k) = PS.out.status;
    sp.iv(kSpSteps, k) = PS.out.steps;
    sp.iv(kSpUpdates, k) = PS.out.updates;
    sp.iv(kSpEqps, k) = PS.out.eqps;
    sp.iv(kSpMoves, k) = PS.out.moves;
    sp.iv(kSpPicks, k) = PS.out.picks;
#pragma unroll
    for (int q = 0; q < 4; ++q) sp.iv(kSpMask0 + q, k) = int(mw[q]);
}

// The pending row (pi, pk) with its coefficients (pk < 0: none).
BODEX_FI PendingRow pending_row(int pi, int pk, double muc, double fm) {
    PendingRow r = {pi, pk, {0.0, 0.0, 0.0}, 0.0};
    if (pk >= 0 && pk < 9) row3(pk, muc, fm, r.c, &r.b);
    return r;
}

// ---------------------------------------------------------------------------
// Group operations.  ShflTeam: the GS lanes of an aligned group of a
// wavefront (cross-lane shuffles); the host tests provide another Team with
// the same interface.
// ---------------------------------------------------------------------------
#if defined(__HIPCC__)
// Value of lane (lane ^ O) within aligned groups of 8 lanes, by DPP moves
// (no LDS traffic): quad permutations for O = 1, 2; for O = 4 the lower
// half of each group reads 4 lanes up (row_shl:4), the upper half 4 lanes
// down (row_shr:4).  Every lane of the group must be active.
template <int O>
__device__ inline int xor_lane(int v) {
    static_assert(O == 1 || O == 2 || O == 4, "xor distance within a group of 8");
    if constexpr (O == 1) return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
    if constexpr (O == 2) return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
    const int up = __builtin_amdgcn_update_dpp(0, v, 0x104, 0xF, 0xF, false);    // row_shl:4
    const int down = __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false);  // row_shr:4
    return (threadIdx.x & 4) ? down : up;
}
template <int O>
__device__ inline double xor_lane(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = xor_lane<O>(int(b)), hi = xor_lane<O>(int(b >> 32));
    return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

template <int GS>
struct ShflTeam {
    static_assert(GS == 4 || GS == 8, "groups of 4 or 8 lanes");
    int sub;
    template <class F>
    __device__ static void each(F f) {
        f(std::integral_constant<int, 1>{});
        f(std::integral_constant<int, 2>{});
        if constexpr (GS == 8) f(std::integral_constant<int, 4>{});
    }
    __device__ double sum(double v) const {
        each([&](auto o) { v += xor_lane<decltype(o)::value>(v); });
        return v;
    }
    template <int N>
    __device__ void sum(double (&v)[N]) const {
        each([&](auto o) {
#pragma unroll
            for (int j = 0; j < N; ++j) v[j] += xor_lane<decltype(o)::value>(v[j]);
        });
    }
    __device__ double max(double v) const {
        each([&](auto o) { v = fmax(v, xor_lane<decltype(o)::value>(v)); });
        return v;
    }
    // the largest v, the lowest index among equals (index -1 loses)
    __device__ void argmax(double& v, int& idx) const {
        each([&](auto o) {
            const double ov = xor_lane<decltype(o)::value>(v);
            const int oi = xor_lane<decltype(o)::value>(idx);
            if (ov > v || (ov == v && unsigned(oi) < unsigned(idx))) {
                v = ov;
                idx = oi;
            }
        });
    }
    // the smallest fraction tn / td (td > 0), the lowest index among equals
    __device__ void argmin_frac(double& tn, double& td, int& idx) const {
        each([&](auto o) {
            constexpr int O = decltype(o)::value;
            const double on = xor_lane<O>(tn), od = xor_lane<O>(td);
            const int oi = xor_lane<O>(idx);
            const double a = on * td, b = tn * od;
            if (a < b || (a == b && unsigned(oi) < unsigned(idx))) {
                tn = on;
                td = od;
                idx = oi;
            }
        });
    }
    __device__ double bcast(double v, int src) const { return __shfl(v, src, GS); }
    __device__ int bcast(int v, int src) const { return __shfl(v, src, GS); }
    __device__ unsigned bor(unsigned v) const {
        each([&](auto o) { v |= unsigned(xor_lane<decltype(o)::value>(int(v))); });
        return v;
    }
};
#endif

// ---------------------------------------------------------------------------
// One QP as one lane of its group sees it.  The storage policy SP names
// where the lane's block of G and the group's 6x6 factor live: RegStore
// keeps both in the lane (registers); LdsStore keeps the block in memory
// shared by the lanes (lane-interleaved) and the factor once per group
// (every lane of the group computes it to the same bits in lockstep).
// ---------------------------------------------------------------------------
// A lane's 6x3 block of G in memory: entry (k, t) at p[(3 k + t) * stride].
struct GBlockShared {
    double* p;
    int stride;
    struct Row {
        double* p;
        int stride;
        BODEX_FI double& operator[](int t) const { return p[t * stride]; }
    };
    BODEX_FI Row operator[](int k) const { return Row{p + 3 * k * stride, stride}; }
};
struct RegStore {
    using Block = double[6][3];
    using Factor = Sym6;
};
struct LdsStore {
    using Block = GBlockShared;
    using Factor = Sym6Shared;
};

template <int MM, class LS = RegStore>
struct GQP {
    // the lane's contact (zeros when sub >= m)
    typename LS::Block G;
    double muc;
    bool live;
    unsigned mk;  // its active rows (9 bits)
    double x[3], z[3];
    ContactProj P;  // its projector at the last factorisation
    // replicated in the group
    double bt[6];
    int m, sub;
    double fmax, eps;
    typename LS::Factor L;  // the factor (one copy per lane or per group)
    PendingRow p, mp;
    double up, mup;
    int phase, mode, chg, step0;
    bool refactor, need_mult;
    PolishOut out;
};

template <int MM, class LS>
BODEX_FI bool gp_on(const GQP<MM, LS>& Q, const PendingRow& p) {
    return p.pk >= 0 && p.pk < 9 && p.pi == Q.sub;
}

// r6 = G v (minus beta t when with_t), v the lanes' 3-vectors.
template <int MM, class T, class LS>
BODEX_FI void gp_gtimes(const T& team, const GQP<MM, LS>& Q, const double* v, bool with_t, double (&r6)[6]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) r6[k] = Q.G[k][0] * v[0] + Q.G[k][1] * v[1] + Q.G[k][2] * v[2];
    team.sum(r6);
    if (with_t) {
#pragma unroll
        for (int k = 0; k < 6; ++k) r6[k] -= Q.bt[k];
    }
}

// The lane's part of 2 (G^T r6 + eps v).
template <int MM, class LS>
BODEX_FI void gp_grad(const GQP<MM, LS>& Q, const double (&r6)[6], const double* v, double* g) {
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        double s = Q.eps * v[t];
#pragma unroll
        for (int k = 0; k < 6; ++k) s += Q.G[k][t] * r6[k];
        g[t] = 2.0 * s;
    }
}

template <int MM, class LS>
BODEX_FI void gp_rows(const GQP<MM, LS>& Q, unsigned mk, ContactRows& R) {
    contact_rows(mk, Q.muc, Q.fmax, R);
}

template <int MM, class LS>
BODEX_FI void gp_refresh_proj(GQP<MM, LS>& Q) {
    ContactRows R;
    gp_rows(Q, Q.mk, R);
    contact_proj(R, Q.P);
}

// v <- H v (v: the lane's 3-vector).
template <int MM, class T, class LS>
BODEX_FI void gp_apply_h(const T& team, const GQP<MM, LS>& Q, double* v) {
    double f[3] = {v[0], v[1], v[2]};
    proj_apply(Q.P, f);
    double gv[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) gv[k] = Q.G[k][0] * f[0] + Q.G[k][1] * f[1] + Q.G[k][2] * f[2];
    team.sum(gv);
    chol6_solve(Q.L, gv);
    double t3[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 6; ++k) s += Q.G[k][t] * gv[k];
        t3[t] = s;
    }
    proj_apply(Q.P, t3);
    const double s2 = 0.5 / Q.eps;
#pragma unroll
    for (int t = 0; t < 3; ++t) v[t] = s2 * (f[t] - t3[t]);
}

// eps I6 + G Pi G^T from every contact (into Q.L, to be factored).
template <int MM, class T, class LS>
BODEX_FI void gp_set_matrix(const T& team, GQP<MM, LS>& Q) {
    double b[6][3];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
#pragma unroll
        for (int t = 0; t < 3; ++t) b[k][t] = Q.G[k][t];
        proj_apply(Q.P, b[k]);
    }
    // the 21 sums in three batches of 7 (bounds the registers the
    // reductions hold at once)
#pragma unroll
    for (int h = 0; h < 3; ++h) {
        double a[7];
#pragma unroll
        for (int e = 0; e < 7; ++e) {
            const int q = 7 * h + e;
            int r = 0;
            while (lo_idx(r + 1, 0) <= q) ++r;
            const int c = q - lo_idx(r, 0);
            a[e] = dot3(b[r], b[c]);
        }
        team.sum(a);
#pragma unroll
        for (int e = 0; e < 7; ++e) Q.L.a[7 * h + e] = a[e];
        BODEX_SPLIT();
    }
#pragma unroll
    for (int r = 0; r < 6; ++r) Q.L.a[lo_idx(r, r)] += Q.eps;
}

// Row kk of contact ci has joined (sgn = -1) or left (+1); the lanes' masks
// hold the new set and Q.L the factor of the old one: the new matrix from
// the old factor and the rank-one term of the changed contact (see
// matrix_row_change).  Returns false if the row has no component outside the
// contact's other rows.
template <int MM, class T, class LS>
BODEX_FI bool gp_row_change(const T& team, GQP<MM, LS>& Q, int ci, int kk, double sgn) {
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, s = 0.0;
    if (Q.sub == ci) {
        ContactRows R;
        ContactProj W;
        gp_rows(Q, Q.mk & ~(1u << kk), R);
        contact_proj(R, W);
        double c[3], bb;
        row3(kk, Q.muc, Q.fmax, c, &bb);
        proj_apply(W, c);
        const double n2 = dot3(c, c);
        s = n2 > 0.0 ? sgn / n2 : 0.0;
#pragma unroll
        for (int k = 0; k < 6; ++k) v[k] = Q.G[k][0] * c[0] + Q.G[k][1] * c[1] + Q.G[k][2] * c[2];
    }
    s = team.bcast(s, ci);
    if (!(s != 0.0)) return false;
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = team.bcast(v[k], ci);
    chol6_product(Q.L);
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c) Q.L.a[lo_idx(r, c)] += s * v[r] * v[c];
    return true;
}

// Multipliers of the lane's active rows at x with the partial multiplier up
// on the pending row (stationarity, closed form per contact).
template <int MM, class LS>
BODEX_FI void gp_multipliers(const GQP<MM, LS>& Q, const ContactRows& R, const double (&r6)[6], const PendingRow& p,
                             double up, double* lam) {
    double h[3];
    gp_grad(Q, r6, Q.x, h);
    const bool on = gp_on(Q, p);
#pragma unroll
    for (int t = 0; t < 3; ++t) h[t] = -h[t] - (on ? up * p.c[t] : 0.0);
    rows_coeffs(R, h, lam);
}

template <int MM, class T, class LS>
BODEX_FI bool gpolish_accept(const T& team, GQP<MM, LS>& Q) {
    double r6[6];
    gp_gtimes(team, Q, Q.x, true, r6);
    double gs = 0.0, stat = 0.0, lneg = 0.0, lmax = 0.0, viol = 0.0, vin = 0.0;
    if (Q.live) {
        double g[3];
        gp_grad(Q, r6, Q.x, g);
        gs = fmax(fabs(g[0]), fmax(fabs(g[1]), fabs(g[2])));
        ContactRows R;
        gp_rows(Q, Q.mk, R);
        double lam[3];
        const PendingRow none = {-1, -1, {0.0, 0.0, 0.0}, 0.0};
        gp_multipliers(Q, R, r6, none, 0.0, lam);
        double st[3] = {g[0], g[1], g[2]};
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            if (j >= R.n) continue;
#pragma unroll
            for (int t = 0; t < 3; ++t) st[t] += lam[j] * R.c[j][t];
            lneg = fmax(lneg, -lam[j]);
            lmax = fmax(lmax, fabs(lam[j]));
        }
        stat = fmax(fabs(st[0]), fmax(fabs(st[1]), fabs(st[2])));
#pragma unroll
        for (int kk = 0; kk < 9; ++kk) {
            double c[3], b;
            row3(kk, Q.muc, Q.fmax, c, &b);
            const double v = dot3(c, Q.x) - b;
            viol = fmax(viol, v);
            if (!((Q.mk >> kk) & 1u)) vin = fmax(vin, v);
        }
    }
    // a NaN anywhere must reject: carry it through the maxima as +inf
    auto nanmax = [](double v) { return v == v ? v : INFINITY; };
    gs = team.max(nanmax(gs));
    stat = team.max(nanmax(stat));
    lneg = team.max(nanmax(lneg));
    lmax = team.max(nanmax(lmax));
    viol = team.max(nanmax(viol));
    vin = team.max(nanmax(vin));
    const bool kkt = stat <= 1e-9 * (1.0 + gs + lmax) && lneg <= 1e-9 * (1.0 + lmax) && isfinite(stat) &&
                     isfinite(gs);
    const double vb = 1e-9 * (1.0 + Q.fmax);
    // violated only outside the active set: more steps (see kPolishViolated)
    Q.out.status = kkt && viol <= vb ? 0 : (kkt && vin > vb && viol == vin ? kPolishViolated : 1);
    return true;
}

// One step of the polish (see polish_advance, whose order and decisions
// this follows); returns true once the QP has reached its acceptance check
// or failed.
template <int MM, class T, class LS>
BODEX_FI bool gpolish_advance(const T& team, GQP<MM, LS>& Q, int max_steps) {
    PolishOut& out = Q.out;
    const double tol_add = 1e-12 * (1.0 + Q.fmax);
    const PendingRow none = {-1, -1, {0.0, 0.0, 0.0}, 0.0};
    if (Q.mode == kAccept) return true;
    if (Q.refactor) {
        if (++out.steps - Q.step0 > max_steps) {
            out.status = 2;
            return true;
        }
        const int row = Q.chg & kNoChange;
        bool quick = (Q.chg & kChgAllowed) && row != kNoChange;
        bool ok = false;
#pragma unroll 1
        for (;;) {
            gp_refresh_proj(Q);
            if (quick) {
                const int ci = row / 9;
                ok = gp_row_change(team, Q, ci, row - 9 * ci, (Q.chg & kChgJoin) ? -1.0 : 1.0);
            } else {
                gp_set_matrix(team, Q);
                ok = true;
            }
            ok = ok && chol6(Q.L);
            if (ok || !quick) break;
            quick = false;
        }
        if (!ok) {
            out.status = 3;
            return true;
        }
        if (quick) {
            ++out.updates;
            Q.chg |= kChgUsed;
        }
        Q.chg = with_change(Q.chg, kNoChange, false);
        Q.refactor = false;
    }
    if (Q.need_mult) Q.need_mult = false;  // no normal-sum multiplier without the sum row
    if (Q.mode == kCheck) {
        if (Q.phase == kFinal) {
            Q.mode = kAccept;
            return true;
        }
        if (Q.phase == kWarm) {
            // the most negative multiplier of the active rows
            double r6[6];
            gp_gtimes(team, Q, Q.x, true, r6);
            double wv = -1e-14;
            int wbit = -1;
            if (Q.live) {
                ContactRows R;
                gp_rows(Q, Q.mk, R);
                double lam[3];
                gp_multipliers(Q, R, r6, Q.mp, Q.mup, lam);
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    if (j < R.n && lam[j] < wv) {
                        wv = lam[j];
                        wbit = 9 * Q.sub + R.id[j];
                    }
                }
            }
            double nv = -wv;  // most negative = largest -lam
            team.argmax(nv, wbit);
            if (wbit >= 0) {
                if (Q.sub == wbit / 9) Q.mk &= ~(1u << (wbit % 9));
                Q.chg = with_change(Q.chg, wbit, false);
                Q.refactor = true;
                Q.mode = kEqp0;
                return false;
            }
            Q.phase = kSteps;
        }
        Q.mode = kPick;
    }
    if (Q.mode == kPick) {
        // the most violated inactive row
        double wv = tol_add;
        int wi = -1;
        if (Q.live) {
#pragma unroll
            for (int kk = 0; kk < 9; ++kk) {
                double c[3], b;
                row3(kk, Q.muc, Q.fmax, c, &b);
                const double s = dot3(c, Q.x) - b;
                if (!((Q.mk >> kk) & 1u) && s > wv) {
                    wv = s;
                    wi = 9 * Q.sub + kk;
                }
            }
        }
        team.argmax(wv, wi);
        ++out.picks;
        if (wi < 0) {
            Q.p = none;
            if (Q.phase != kFinal) {
                Q.mode = kAccept;
                return true;
            }
            Q.mode = kEqp0;
        } else {
            Q.p = pending_row(wi / 9, wi % 9, team.bcast(Q.muc, wi / 9), Q.fmax);
            Q.phase = kSteps;
            Q.up = 0.0;
            Q.mode = kStep;
        }
    }
    bool dep = false;
    double sp = -Q.p.b;
    if (Q.mode == kEqp0) {
        ContactRows R;
        gp_rows(Q, Q.mk, R);
        double f[3];
        rows_point(R, f);
#pragma unroll
        for (int t = 0; t < 3; ++t) Q.x[t] = Q.live ? f[t] : 0.0;
        ++out.eqps;
    }
    if (Q.mode != kStep) {
        double r6[6];
        gp_gtimes(team, Q, Q.x, true, r6);
        gp_grad(Q, r6, Q.x, Q.z);
        if (!Q.live) Q.z[0] = Q.z[1] = Q.z[2] = 0.0;
    } else {
        // c_p into z; is it in the span of the active rows?
        const bool on = gp_on(Q, Q.p);
        double v[3] = {on ? Q.p.c[0] : 0.0, on ? Q.p.c[1] : 0.0, on ? Q.p.c[2] : 0.0};
        double loc[3];
        loc[0] = dot3(v, Q.x);
        loc[1] = dot3(v, v);
#pragma unroll
        for (int t = 0; t < 3; ++t) Q.z[t] = v[t];
        proj_apply(Q.P, v);
        loc[2] = dot3(v, v);
        team.sum(loc);
        sp += loc[0];
        dep = !(loc[2] > 1e-12 * loc[1]);
    }
    if (dep) {
        Q.z[0] = Q.z[1] = Q.z[2] = 0.0;
    } else {
        gp_apply_h(team, Q, Q.z);
    }
    if (Q.mode != kStep) {
        // equality solve pass: x <- x - H grad(x)
#pragma unroll
        for (int t = 0; t < 3; ++t) Q.x[t] -= Q.z[t];
        if (Q.mode == kEqp0) {
            Q.mode = kEqp1;
        } else {
            Q.mp = none;
            Q.mup = 0.0;
            Q.need_mult = true;
            Q.mode = kCheck;
        }
        return false;
    }
    // one-row step: the largest step keeping the multipliers nonnegative
    // (t1) against the step that satisfies p (t2)
    ++out.moves;
    double gz[6], r6x[6];
    gp_gtimes(team, Q, Q.z, false, gz);
    gp_gtimes(team, Q, Q.x, true, r6x);
    double tn = INFINITY, td = 1.0, cz = 0.0;
    int lbit = -1;
    if (Q.live) {
        const bool on = gp_on(Q, Q.p);
        if (on) cz = dot3(Q.p.c, Q.z);
        ContactRows R;
        gp_rows(Q, Q.mk, R);
        double w[3], h[3], r[3], lam[3];
        gp_grad(Q, gz, Q.z, w);
#pragma unroll
        for (int t = 0; t < 3; ++t) w[t] = (on ? Q.p.c[t] : 0.0) - w[t];
        gp_grad(Q, r6x, Q.x, h);
        const bool mon = gp_on(Q, Q.mp);
#pragma unroll
        for (int t = 0; t < 3; ++t) h[t] = -h[t] - (mon ? Q.mup * Q.mp.c[t] : 0.0);
        rows_coeffs2(R, w, h, r, lam);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            if (j < R.n && r[j] > 0.0 && lam[j] * td < tn * r[j]) {
                tn = lam[j];
                td = r[j];
                lbit = 9 * Q.sub + R.id[j];
            }
        }
    }
    cz = team.sum(cz);
    team.argmin_frac(tn, td, lbit);
    const double t1 = tn / td;
    const double t2 = (dep || !(cz > 0.0)) ? INFINITY : sp / cz;
    const double st = t2 < t1 ? t2 : t1;
    if (!(st < INFINITY) || !(st >= 0.0) || (Q.chg & kChgBreakAny)) {
        Q.chg &= ~int(kChgBreakAny);
        out.status = 3;  // infeasible or broken down
        return true;
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) Q.x[t] -= st * Q.z[t];
    Q.up += st;
    Q.refactor = true;
    Q.need_mult = true;
    if (t2 <= t1) {
        // p joins the active set; an exact re-solve follows the last step
        if (Q.sub == Q.p.pi) Q.mk |= 1u << Q.p.pk;
        Q.chg = with_change(Q.chg, 9 * Q.p.pi + Q.p.pk, true);
        Q.phase = kFinal;
        Q.mp = none;
        Q.mup = 0.0;
        Q.mode = kPick;
    } else {
        // drop the row whose multiplier reached zero, continue with p
        if (Q.sub == lbit / 9) Q.mk &= ~(1u << (lbit % 9));
        Q.chg = with_change(Q.chg, lbit, false);
        Q.mp = Q.p;
        Q.mup = Q.up;
        Q.mode = kStep;
    }
    return false;
}

// See polish_finish: false when the QP is taken once more on fresh
// factorisations.
template <int MM, class T, class LS>
BODEX_FI bool gpolish_finish(const T& team, GQP<MM, LS>& Q) {
    const bool reached = Q.mode == kAccept;
    if (reached) gpolish_accept(team, Q);
    if (Q.out.status == kPolishViolated) {
        Q.out.status = 0;
        Q.phase = kSteps;
        Q.mode = kPick;
        return false;
    }
    if (Q.out.status != 0 && (Q.chg & kChgUsed)) {
        Q.out.status = 0;
        Q.chg = kNoChange | (Q.chg & kChgCold);
        Q.step0 = Q.out.steps;
        Q.refactor = true;
        Q.phase = kWarm;
        Q.mode = kEqp0;
        return false;
    }
    // as polish_finish: once more from the empty active set
    if (Q.out.status != 0 && !(Q.chg & kChgCold)) {
        const PendingRow none = {-1, -1, {0.0, 0.0, 0.0}, 0.0};
        Q.out.status = 0;
        Q.chg = kNoChange | kChgCold;
        Q.step0 = Q.out.steps;
        Q.mk = 0u;
        Q.p = none;
        Q.mp = none;
        Q.up = 0.0;
        Q.mup = 0.0;
        Q.need_mult = false;
        Q.refactor = true;
        Q.phase = kWarm;
        Q.mode = kEqp0;
        return false;
    }
    return true;
}

// The lane's view of record k: its contact's G (FP64, from the FP32
// inputs), mu_i cos(pi/8) of every contact, beta t, and the saved state.
template <int MM, class T, class LS>
BODEX_FI void gpolish_load(const T& team, GQP<MM, LS>& Q, const SpillPtrs& sp, int k, int m, const double* p3,
                           const double* n3, double mu_own, double kappa, const double* bt, double fmax, double eps) {
    Q.m = m;
    Q.live = Q.sub < m;
    Q.fmax = fmax;
    Q.eps = eps;
#pragma unroll
    for (int r = 0; r < 6; ++r) Q.bt[r] = bt[r];
    double Gc[6 * 3];
#pragma unroll
    for (int e = 0; e < 18; ++e) Gc[e] = 0.0;
    if (Q.live) grasp_columns<double, 3>(p3, n3, kappa, 0, Gc);
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int t = 0; t < 3; ++t) Q.G[r][t] = Gc[r * 3 + t];
    Q.muc = Q.live ? mu_own * kC8 : 0.5;
#pragma unroll
    for (int t = 0; t < 3; ++t) Q.x[t] = Q.live ? sp.dv(3 * Q.sub + t, k) : 0.0;
    Q.up = sp.dv(3 * MM, k);
    Q.mup = sp.dv(3 * MM + 1, k);
    unsigned mw[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) mw[j] = unsigned(sp.iv(kSpMask0 + j, k));
    const RowMask<MM> mask = mask_from_words<RowMask<MM>>(mw);
    Q.mk = Q.live ? contact_mask(mask, Q.sub) : 0u;
    const int ppi = sp.iv(kSpPpi, k), ppk = sp.iv(kSpPpk, k);
    const int mpi = sp.iv(kSpMpi, k), mpk = sp.iv(kSpMpk, k);
    const double pmuc = team.bcast(Q.muc, ppk >= 0 ? ppi : 0);
    const double mmuc = team.bcast(Q.muc, mpk >= 0 ? mpi : 0);
    Q.p = pending_row(ppi, ppk, pmuc, fmax);
    Q.mp = pending_row(mpi, mpk, mmuc, fmax);
    Q.phase = sp.iv(kSpPhase, k);
    Q.mode = sp.iv(kSpMode, k);
    Q.need_mult = sp.iv(kSpNeedMult, k) != 0;
    // the old factor was not saved: the next factorisation is a fresh one
    Q.chg = with_change(sp.iv(kSpChg, k), kNoChange, false);
    Q.step0 = sp.iv(kSpStep0, k);
    Q.out.status = 0;
    Q.out.steps = sp.iv(kSpSteps, k);
    Q.out.updates = sp.iv(kSpUpdates, k);
    Q.out.eqps = sp.iv(kSpEqps, k);
    Q.out.moves = sp.iv(kSpMoves, k);
    Q.out.picks = sp.iv(kSpPicks, k);
    Q.refactor = true;
#pragma unroll
    for (int t = 0; t < 3; ++t) Q.z[t] = 0.0;
}

// The finished polish back into record k: x, the active set and the counts
// (the tail of the finalize kernel forms the outputs from them).
template <int MM, class T, class LS>
BODEX_FI void gpolish_store(const T& team, const GQP<MM, LS>& Q, const SpillPtrs& sp, int k) {
    if (Q.live) {
#pragma unroll
        for (int t = 0; t < 3; ++t) sp.dv(3 * Q.sub + t, k) = Q.x[t];
    }
    // the contacts' 9-bit masks into the four 32-bit words
    unsigned mw[4] = {0u, 0u, 0u, 0u};
    const int bit = 9 * Q.sub;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int lo = 32 * j;
        unsigned wv = 0u;
        if (bit < lo + 32 && bit + 9 > lo) wv = bit >= lo ? (Q.mk << (bit - lo)) : (Q.mk >> (lo - bit));
        mw[j] = team.bor(wv);
    }
    if (Q.sub == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) sp.iv(kSpMask0 + j, k) = int(mw[j]);
        sp.dv(3 * MM + 2, k) = 0.0;
        sp.iv(kSpStatus, k) = Q.out.status;
        sp.iv(kSpSteps, k) = Q.out.steps;
        sp.iv(kSpUpdates, k) = Q.out.updates;
        sp.iv(kSpEqps, k) = Q.out.eqps;
        sp.iv(kSpMoves, k) = Q.out.moves;
        sp.iv(kSpPicks, k) = Q.out.picks;
    }
}

}  // namespace bodex
