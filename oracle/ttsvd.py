"""Deterministic TT-rounding (the paper's Algorithm "TT-Rounding", Sec. 2.2).

Steps, in the paper's order:
  1. right-to-left orthogonalization of X;
  2. tau = eps * ||Y_1|| / sqrt(d-1) (fixed-precision mode);
  3. for k = 1..d-1: [V(Y_k), R] = QR(V(Y_k)); [U, S, V^T] = SVD(R) truncated
     by tau or to the target rank l_k; V(Y_k) = V(Y_k) U;
     H(Y_{k+1}) = S V^T H(Y_{k+1}).

Truncation rule (the paper says "tau truncated SVD" without a formula): keep
the smallest t >= 1 with sqrt(sum_{j>t} s_j^2) <= tau.  With per-bond
threshold eps*||X||/sqrt(d-1) the total error is at most eps*||X||.
"""

import math

import numpy as np

from .tt import h_unf, v_unf, orthogonalize_rl


def truncation_rank(s, tau):
    """Smallest t >= 1 whose discarded tail sqrt(sum_{j>=t} s_j^2) <= tau."""
    s = np.asarray(s, dtype=np.float64)
    m = s.size
    tail2 = np.concatenate([np.cumsum((s ** 2)[::-1])[::-1], [0.0]])  # tail2[t] = sum_{j>=t}
    for t in range(1, m + 1):
        if math.sqrt(tail2[t]) <= tau:
            return t
    return m


def bond_threshold(tol, norm, d):
    """Algorithm TT-Rounding (Sec. 2.3): tau = ||Y|| eps / sqrt(d-1), so
    that d-1 truncations of tail at most tau keep the total error within
    eps ||Y||."""
    return tol * norm / math.sqrt(d - 1)


def tt_svd_round(cores, tol=None, ranks=None):
    """Round X by TT-SVD.  Give tol (relative accuracy) or ranks (list of
    d+1 target ranks, ends 1).  Returns (cores, info)."""
    if (tol is None) == (ranks is None):
        raise ValueError("give exactly one of tol or ranks")
    ys = orthogonalize_rl(cores)
    d = len(ys)
    nrm = float(np.linalg.norm(ys[0]))
    tau = bond_threshold(tol, nrm, d) if tol is not None else None
    svals = []
    for k in range(d - 1):
        r0, n, _ = ys[k].shape
        q, r = np.linalg.qr(v_unf(ys[k]))
        u, s, vt = np.linalg.svd(r)
        svals.append(s)
        if tol is not None:
            t = truncation_rank(s, tau)
        else:
            t = max(1, min(int(ranks[k + 1]), s.size))
        ys[k] = (q @ u[:, :t]).reshape(r0, n, t)
        _, n1, r2 = ys[k + 1].shape
        nxt = (s[:t, None] * vt[:t, :]) @ h_unf(ys[k + 1])
        ys[k + 1] = nxt.reshape(t, n1, r2)
    return ys, {"tau": tau, "norm": nrm, "svals": svals,
                "ranks": [1] + [int(c.shape[2]) for c in ys]}
