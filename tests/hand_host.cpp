// Host build of the solver's coarse-stage query arithmetic (the header the GPU
// kernels use), for CPU tests against the oracle.
#include "../paper_2412_16490_amd/csrc/bodex_hand.h"

using namespace bodex;

extern "C" {

// Nearest point, inward normal, signed distance; returns 1 where a Jacobian exists.
int host_nearest(const double* c, const double* a, double* p, double* n, double* d) {
    Near q;
    nearest(c, a, q);
    for (int k = 0; k < 3; ++k) {
        p[k] = q.p[k];
        n[k] = q.n[k];
    }
    *d = q.d;
    return q.jac ? 1 : 0;
}

// vp^T dp/dc + vn^T dn/dc + ws dd/dc at c (zero where no Jacobian exists).
void host_chain(const double* c, const double* a, const double* vp, const double* vn, double ws, double* out) {
    Near q;
    nearest(c, a, q);
    for (int k = 0; k < 3; ++k) out[k] = 0.0;
    if (!q.jac) return;
    chain(c, a, q, vp, vn, out);
    for (int k = 0; k < 3; ++k) out[k] += ws * q.gh[k];
}

void host_rodrigues(const double* w, double* E) { rodrigues(w, E); }

}  // extern "C"
