"""Writes aed_rejection_window.txt: an 8 x 8 upper Hessenberg AED window whose
Schur form holds adjacent blocks too ill-conditioned to exchange (a cluster of
nearly defective 2x2 blocks with large coupling, hidden by a random orthogonal
similarity and a Hessenberg reduction).  Inputs only: numpy and scipy build
it from a fixed seed; no expected value is stored.  The seed was picked from
a seeded sweep as the first whose window makes the Bai-Demmel stability test
of an AED reordering (Sec. 2.5; swap failures in Sec. 3.5) reject a swap.

    python tests/golden/make_rejection_window.py
"""
import os

import numpy as np
import scipy.linalg as sla

SEED = 1545
HERE = os.path.dirname(os.path.abspath(__file__))


def std_block(a, w, r):
    return np.array([[a, w * r], [-w / r, a]])


def window(seed=SEED, m=8):
    g = np.random.default_rng(seed)
    T = np.triu(g.standard_normal((m, m))) * 10 ** g.uniform(0, 8)
    a = g.uniform(-1, 1)
    for k in range(0, m, 2):
        T[k:k + 2, k:k + 2] = std_block(a + 10 ** g.uniform(-12, -3) * g.standard_normal(),
                                        10 ** g.uniform(-10, 0), 10 ** g.uniform(-4, 4))
    G = np.linalg.qr(g.standard_normal((m, m)))[0]
    return sla.hessenberg(G @ T @ G.T)


if __name__ == "__main__":
    W = window()
    np.savetxt(os.path.join(HERE, "aed_rejection_window.txt"), W, fmt="%.17g",
               header=f"8x8 Hessenberg AED window (seed {SEED}); written by make_rejection_window.py")
