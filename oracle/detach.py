"""FP64 oracle of the fine-stage surrogate energies with the Detach trick
(arXiv 2412.16490, Sec. IV-C, Eq. 10-11).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.

For contact i of a grasp, with the link transform (R_i, T_i) of the finger
that carries it, the fine-stage nearest points c^f_{i,w} (fingertip, world
frame) and p^f_i (object), and the object point p^c_i kept from the end of
the coarse stage:

    c^f_{i,l}  = R_i^{-1} (c^f_{i,w} - T_i)        (the point in the link frame)
    c'_{i,w}   = R_i Detach(c^f_{i,l}) + T_i        (Eq. 11)
    E^f_d      = sum_i || c'_{i,w} - p^f_i ||^2     (Eq. 10)
    Q'         = sum_i || c'_{i,w} - p^c_i ||^2     (Eq. 10)

Detach makes c^f_{i,l} a constant of the differentiation, so c'_{i,w} depends
on (R_i, T_i) only through the affine map: for L = wq Q' + we E^f_d,

    g_i      = dL/dc'_{i,w} = 2 wq (c'_{i,w} - p^c_i) + 2 we (c'_{i,w} - p^f_i)
    dL/dR_i  = g_i (c^f_{i,l})^T,      dL/dT_i = g_i.

The forward values equal the plain distances of c^f_{i,w} (c' = c^f in exact
arithmetic); only the gradient path changes.  Contacts i >= count of a grasp
are padding: they add nothing and their gradients are zero.
"""
from __future__ import annotations

import numpy as np


def detach_energy(R, T, cw, pf, pc, counts=None, wq=None, we=None):
    """Eq. 10-11 in FP64.

    R [G][M][3][3], T, cw, pf, pc [G][M][3]; counts [G] (None: all M);
    wq, we [G] loss weights of Q' and E^f_d (None: zero).
    Returns (Qp [G], Ed [G], dR [G][M][3][3], dT [G][M][3]).
    """
    R = np.asarray(R, np.float64)
    T = np.asarray(T, np.float64)
    cw = np.asarray(cw, np.float64)
    pf = np.asarray(pf, np.float64)
    pc = np.asarray(pc, np.float64)
    G, M = T.shape[0], T.shape[1]
    counts = np.full(G, M) if counts is None else np.asarray(counts)
    wq = np.zeros(G) if wq is None else np.asarray(wq, np.float64)
    we = np.zeros(G) if we is None else np.asarray(we, np.float64)
    Qp = np.zeros(G)
    Ed = np.zeros(G)
    dR = np.zeros((G, M, 3, 3))
    dT = np.zeros((G, M, 3))
    for g in range(G):
        for i in range(int(counts[g])):
            # Eq. 11: the fingertip point in its link frame, held constant
            c_l = np.linalg.solve(R[g, i], cw[g, i] - T[g, i])
            c_w = R[g, i] @ c_l + T[g, i]
            d_c = c_w - pc[g, i]
            d_f = c_w - pf[g, i]
            # Eq. 10
            Qp[g] += d_c @ d_c
            Ed[g] += d_f @ d_f
            gi = 2.0 * wq[g] * d_c + 2.0 * we[g] * d_f
            dR[g, i] = np.outer(gi, c_l)
            dT[g, i] = gi
    return Qp, Ed, dR, dT
