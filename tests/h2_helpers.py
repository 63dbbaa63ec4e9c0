"""Exactly H2 test matrices shared by the oracle pins and the GPU parity tests."""
import numpy as np


def exact_h2(t, r, seed=3):
    """A = blockdiag over leaves (Gaussian + m I) + U V^T with U, V of rank r.

    Every box's far-field interaction has rank <= 2r, and after an exact ID the
    couplings between eliminated indices and the neighbours vanish, so the
    structure survives each level (Sec. 3.1, Remark 2)."""
    rng = np.random.default_rng(seed)
    N = t.n
    A = np.zeros((N, N))
    for b in np.nonzero(t.is_leaf)[0]:
        idx = t.perm[t.pt_begin[b]:t.pt_end[b]]
        m = len(idx)
        A[np.ix_(idx, idx)] = rng.standard_normal((m, m)) + m * np.eye(m)
    U = rng.standard_normal((N, r))
    V = rng.standard_normal((N, r))
    return A + U @ V.T
