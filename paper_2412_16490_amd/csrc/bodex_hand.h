// bodex_hand.h -- FP64 arithmetic of the coarse-stage contact query on an
// analytic object (arXiv 2412.16490, Sec. IV-C): nearest point of an
// ellipsoid, its Jacobian-transposed products and the Rodrigues exponential.
// Host and device: the GPU kernels use it, and a host build is checked against
// the oracle on the CPU.  The method is described in k_hand.hip.
#pragma once

#include <math.h>

#include "bodex_math.h"

namespace bodex {

struct Near {
    double p[3], n[3], d;
    double M[3];   // 1 / (a_k^2 + t), valid when jac
    double gh[3];  // g / |g| = -n
    double gn;     // |g|
    bool jac;      // a derivative exists (not on the ridge, not the centre)
};

BODEX_FI void nearest(const double c[3], const double a[3], Near& q) {
    int k0 = 0;
    for (int k = 1; k < 3; ++k)
        if (a[k] < a[k0] || (a[k] == a[k0] && fabs(c[k]) > fabs(c[k0]))) k0 = k;
    double a2[3], off[3];
    for (int k = 0; k < 3; ++k) a2[k] = a[k] * a[k];
    for (int k = 0; k < 3; ++k) off[k] = a2[k] - a2[k0];
    q.jac = false;
    if (c[0] == 0.0 && c[1] == 0.0 && c[2] == 0.0) {
        for (int k = 0; k < 3; ++k) {
            q.p[k] = k == k0 ? a[k0] : 0.0;
            q.n[k] = k == k0 ? -1.0 : 0.0;
        }
        q.d = -a[k0];
        return;
    }
    // S(u) and S1(u) = sum_k (a_k c_k)^2 / den_k^3
    auto eval = [&](double u, double& S1) {
        double S = 0.0;
        S1 = 0.0;
        for (int k = 0; k < 3; ++k) {
            if (c[k] == 0.0) continue;
            const double den = off[k] + u;
            const double r = a[k] * c[k] / den;
            S += r * r;
            S1 += r * r / den;
        }
        return S;
    };
    double u = a[k0] * fabs(c[k0]);
    bool ridge = false;
    if (c[k0] == 0.0) {
        // no pole at u = 0 (every axis as small as axis 0 has c_k = 0)
        double S1;
        ridge = eval(0.0, S1) <= 1.0;
        u = 0.0;
    }
    if (!ridge) {
        for (int it = 0; it < 100; ++it) {
            double S1;
            const double S = eval(u, S1);
            const double h = 1.0 / sqrt(S);
            if (!(h < 1.0)) break;  // at the root (to rounding)
            const double un = u + (1.0 - h) * S / (h * S1);
            if (!(un > u)) break;
            u = un;
        }
    }
    const double t = u - a2[k0];
    if (ridge) {
        double rest = 0.0;
        for (int k = 0; k < 3; ++k) {
            q.p[k] = k == k0 ? 0.0 : a2[k] * c[k] / (off[k] + u);
            rest += (q.p[k] / a[k]) * (q.p[k] / a[k]);
        }
        q.p[k0] = a[k0] * sqrt(fmax(0.0, 1.0 - rest));
        double gp[3], gpn = 0.0, dd = 0.0;
        for (int k = 0; k < 3; ++k) {
            gp[k] = q.p[k] / a2[k];
            gpn += gp[k] * gp[k];
            dd += (c[k] - q.p[k]) * (c[k] - q.p[k]);
        }
        gpn = sqrt(gpn);
        for (int k = 0; k < 3; ++k) q.n[k] = -gp[k] / gpn;
        q.d = -sqrt(dd);
        return;
    }
    double g[3], gn = 0.0;
    for (int k = 0; k < 3; ++k) {
        q.M[k] = 1.0 / (off[k] + u);
        g[k] = c[k] * q.M[k];
        q.p[k] = a2[k] * g[k];
        gn += g[k] * g[k];
    }
    gn = sqrt(gn);
    q.gn = gn;
    for (int k = 0; k < 3; ++k) {
        q.gh[k] = g[k] / gn;
        q.n[k] = -q.gh[k];
    }
    q.d = t * gn;  // c - p = t g
    q.jac = true;
}

// v^T dp/dc + vn^T dn/dc (a row vector; dp/dc is symmetric)
BODEX_FI void chain(const double c[3], const double a[3], const Near& q, const double* vp,
                             const double* vn, double out[3]) {
    double w[3], s = 0.0;
    for (int k = 0; k < 3; ++k) {
        w[k] = a[k] * a[k] * q.M[k] * q.M[k] * c[k];
        s += w[k] * c[k] * q.M[k];
    }
    double dt[3];
    for (int k = 0; k < 3; ++k) dt[k] = w[k] / s;
    for (int k = 0; k < 3; ++k) out[k] = 0.0;
    if (vp) {
        double wv = 0.0;
        for (int k = 0; k < 3; ++k) wv += w[k] * vp[k];
        for (int k = 0; k < 3; ++k) out[k] += a[k] * a[k] * q.M[k] * vp[k] - w[k] * wv / s;
    }
    if (vn) {
        // y = -(I - gh gh^T) vn / |g|;  dg/dc^T y = M o y - dt (M^2 c . y)
        double gv = 0.0;
        for (int k = 0; k < 3; ++k) gv += q.gh[k] * vn[k];
        double y[3], m2cy = 0.0;
        for (int k = 0; k < 3; ++k) {
            y[k] = -(vn[k] - q.gh[k] * gv) / q.gn;
            m2cy += q.M[k] * q.M[k] * c[k] * y[k];
        }
        for (int k = 0; k < 3; ++k) out[k] += q.M[k] * y[k] - dt[k] * m2cy;
    }
}

// Rodrigues: E = I + A K + B K^2 for K = [w]x, A = sin(th)/th, B = (1 - cos th)/th^2.
BODEX_FI void rodrigues(const double w[3], double E[9]) {
    const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    const double th = sqrt(th2);
    double A, B;
    if (th < 1e-6) {
        A = 1.0 - th2 / 6.0;
        B = 0.5 - th2 / 24.0;
    } else {
        const double sh = sin(0.5 * th);
        A = sin(th) / th;
        B = 2.0 * sh * sh / th2;
    }
    const double K[9] = {0.0, -w[2], w[1], w[2], 0.0, -w[0], -w[1], w[0], 0.0};
    for (int r = 0; r < 3; ++r)
        for (int col = 0; col < 3; ++col) {
            double k2 = 0.0;
            for (int j = 0; j < 3; ++j) k2 += K[3 * r + j] * K[3 * j + col];
            E[3 * r + col] = (r == col ? 1.0 : 0.0) + A * K[3 * r + col] + B * k2;
        }
}

}  // namespace bodex
