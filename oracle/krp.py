"""KRP-sketched randomized TT-rounding, oracle side (CPU FP64).

Follows the paper step by step:
  * partial contractions with a Khatri-Rao sketch, Eq. (6)-(8) and the
    Algorithm "Right-to-Left Contraction with KRP Structured Matrix" (Sec. 3.1),
    and the left-to-right order the same section describes;
  * fixed-rank Randomize-then-Orthogonalize with KRP (Sec. 3.2);
  * residual sketching for basis expansion (Sec. 3.3) and the adaptive-rank
    Randomize-then-Orthogonalize with KRP (Sec. 3.3);
  * the norm estimate of Remark 1 and the recompression pass of Remark 2.

Readings taken where the paper is silent or ambiguous:
  * Index order of the KRP.  The paper writes W_k = H(X_k)[W_{k+1} (.) Omega_k]
    for MATLAB's column-major H.  In row-major storage the column index of
    H(X_k) is i*r_k + b, so the same product is H(X_k)[Omega_k (.) W_{k+1}];
    both equal W_k(a,j) = sum_{i,b} X_k(a,i,b) Omega_k(i,j) W_{k+1}(b,j).
  * Gaussian source: counter-based (oracle.philox), column-addressable, so a
    regenerated column is identical whatever chunk it is drawn in.
  * Regeneration size in the residual sketch: when W_{k+1} has fewer than
    col(Q)+b columns, exactly col(Q)+b-col(W_{k+1}) new columns are drawn
    for modes k+1..d (the printed size can be negative).
  * Sketch sizes are capped: fixed rank uses l_k = min(ell, rows, cols) of
    V(Y_k); the adaptive block is clamped to rbar_k - col(Q) and the
    estimate divides by the block actually used; the loop also stops when
    col(Q) reaches rbar_k.  "est == tau" stops (the test is est > tau).
  * ell_block replaces b_inc = ceil(f_inc * rbar_k); ell_block <= 0 means
    f_inc = 0.05.  f_init = 0.1 sets r0 and b_init as in the paper.
  * nrmx: given by the caller, else the Remark 1 estimate from all r0
    initial columns of W_2.
  * QR is Householder with the sign fixed so that diag(R) >= 0.
  * Oversampling (ell larger than the target ranks) and Remark 2 use a
    right-to-left pass: H(Y_k)^T = QR, SVD of R^T, truncate by tau (tail
    rule) or to the target rank, fold U*S into core k-1.
  * Sums of TT tensors (the remark on sums): the result is defined as the
    rounding of the formal sum sum_i w_i X^(i) (first cores side by side with
    the weights, block-diagonal middle cores, stacked last cores) with the
    same Gaussian factors.  Sketching the summands separately changes only
    the order of floating-point operations: the partial contractions of the
    formal sum are the summands' partial contractions stacked by rows.
"""

import math

import numpy as np

from .philox import gaussian_factor
from .tt import h_unf, v_unf
from .ttsvd import truncation_rank


def khatri_rao(a, b):
    """Column-wise Kronecker product: column j is kron(a[:, j], b[:, j])."""
    assert a.shape[1] == b.shape[1]
    return (a[:, None, :] * b[None, :, :]).reshape(a.shape[0] * b.shape[0], a.shape[1])


def partial_contractions_rl(cores, omegas, t):
    """W_d = H(X_d) Omega_d; W_k = H(X_k) [Omega_k (.) W_{k+1}] for k=d-1..t.

    cores: list of d cores; omegas: dict 1-based mode -> (n_mode x l).
    Returns dict 1-based k -> W_k of shape (r_{k-1} x l), k = t..d.
    """
    d = len(cores)
    w = {d: h_unf(cores[d - 1]) @ omegas[d]}
    for k in range(d - 1, t - 1, -1):
        w[k] = h_unf(cores[k - 1]) @ khatri_rao(omegas[k], w[k + 1])
    return w


def partial_contractions_lr(cores, omegas, t):
    """Left-to-right partial contractions (Sec. 3.1: the recurrence of the
    right-to-left algorithm run in the other order), for k = 1..t:
    WL_1 = V(X_1)^T Omega_1 and WL_k = V(X_k)^T [WL_{k-1} (.) Omega_k], i.e.
    WL_k(b, j) = sum_{a,i} X_k(a,i,b) WL_{k-1}(a,j) Omega_k(i,j).

    cores: list of d cores; omegas: dict 1-based mode -> (n_mode x l).
    Returns dict 1-based k -> WL_k of shape (r_k x l), k = 1..t.
    """
    w = {1: v_unf(cores[0]).T @ omegas[1]}
    for k in range(2, t + 1):
        # the row (a, i) of V(X_k) pairs with WL_{k-1}(a, :) * Omega_k(i, :)
        w[k] = v_unf(cores[k - 1]).T @ khatri_rao(w[k - 1], omegas[k])
    return w


def qr_pos(s):
    """Reduced Householder QR with diag(R) >= 0; returns Q."""
    q, r = np.linalg.qr(s)
    sgn = np.sign(np.diag(r))
    sgn[sgn == 0] = 1.0
    return q * sgn[None, :]


def draw_omegas(seed, dims, modes, col0, ncols):
    return {j: gaussian_factor(seed, j, dims[j - 1], col0, ncols) for j in modes}


def recompress_rl(cores, tau=None, ranks=None):
    """Right-to-left truncation pass (Remark 2): for k = d..2,
    H(Y_k)^T = QR; R^T = U S V^T; keep t columns (tail rule with tau, or the
    target rank); H(Y_k) = V_t^T Q^T; V(Y_{k-1}) = V(Y_{k-1}) U_t S_t.
    ranks: list of d+1 target ranks.  Output is right-orthonormal."""
    ys = [np.array(c, copy=True) for c in cores]
    d = len(ys)
    for k in range(d - 1, 0, -1):
        r0, n, r1 = ys[k].shape
        q, r = np.linalg.qr(h_unf(ys[k]).T)       # (n r1) x m, m x r0
        u, s, vt = np.linalg.svd(r.T)             # r^T: r0 x m
        if tau is not None:
            t = truncation_rank(s, tau)
        else:
            t = max(1, min(int(ranks[k]), s.size))
        ys[k] = (vt[:t, :] @ q.T).reshape(t, n, r1)
        p0, pn, _ = ys[k - 1].shape
        ys[k - 1] = (v_unf(ys[k - 1]) @ (u[:, :t] * s[None, :t])).reshape(p0, pn, t)
    return ys


def round_fixed(cores, ell, seed, target_ranks=None):
    """Fixed-rank Rand-Orth-KRP (Sec. 3.2) with sketch size ell, then, if
    target_ranks (d+1 list) asks for less, the right-to-left truncation.
    Returns (cores, info)."""
    d = len(cores)
    dims = [c.shape[1] for c in cores]
    om = draw_omegas(seed, dims, range(2, d + 1), 0, ell)
    w = partial_contractions_rl(cores, om, 2)
    ys = [None] * d
    y = np.array(cores[0], copy=True)
    sk_ranks = [1]
    for k in range(1, d):                      # k is 1-based mode
        z = v_unf(y)
        lk = min(ell, z.shape[0], z.shape[1])
        s = z @ w[k + 1][:, :lk]
        q = qr_pos(s)
        m = q.T @ z
        ys[k - 1] = q.reshape(y.shape[0], y.shape[1], lk)
        _, n1, r2 = cores[k].shape
        y = (m @ h_unf(cores[k])).reshape(lk, n1, r2)
        sk_ranks.append(lk)
    ys[d - 1] = y
    sk_ranks.append(1)
    info = {"sketch_ranks": sk_ranks, "W": w}
    if target_ranks is not None and any(int(target_ranks[k]) < sk_ranks[k] for k in range(1, d)):
        ys = recompress_rl(ys, ranks=target_ranks)
    info["ranks"] = [1] + [int(c.shape[2]) for c in ys]
    return ys, info


class _Sketches:
    """Partial contractions W_j (j = 2..d) whose columns grow on demand; all
    W_j that are still needed share one column count."""

    def __init__(self, cores, seed, ncols):
        self.cores = cores
        self.seed = seed
        self.dims = [c.shape[1] for c in cores]
        self.d = len(cores)
        om = draw_omegas(seed, self.dims, range(2, self.d + 1), 0, ncols)
        self.w = partial_contractions_rl(cores, om, 2)
        self.passes = 1

    def ncols(self, k):
        return self.w[k].shape[1]

    def extend(self, k, extra):
        """Append `extra` new columns to W_k..W_d (a partial contraction
        pass over cores k..d with freshly drawn Omega columns)."""
        c0 = self.ncols(k)
        om = draw_omegas(self.seed, self.dims, range(k, self.d + 1), c0, extra)
        new = partial_contractions_rl(self.cores, om, k)
        for j in range(k, self.d + 1):
            self.w[j] = np.concatenate([self.w[j], new[j]], axis=1)
        self.passes += 1


def generate_residual_sketch(sk, z, q, k, b):
    """Residual sketching (Sec. 3.3): make sure W_{k+1} has col(Q)+b
    columns, then S = Z W_{k+1}(:, col(Q):col(Q)+b) and S -= Q (Q^T S)."""
    need = q.shape[1] + b
    have = sk.ncols(k + 1)
    if have < need:
        sk.extend(k + 1, need - have)
    s = z @ sk.w[k + 1][:, q.shape[1]:need]
    s = s - q @ (q.T @ s)
    return s


def norm_estimate(core1, w2):
    """Remark 1: ||X|| ~ ||V(X_1) W_2||_F / sqrt(r), r = columns of W_2."""
    return float(np.linalg.norm(v_unf(core1) @ w2) / math.sqrt(w2.shape[1]))


def initial_sketch_columns(cores, f_init):
    """Sec. 3.3, first step of the adaptive algorithm: the Gaussian factors
    start with r = ceil(f_init * max_j r_j) columns, the maximum taken over
    the interior ranks r_1 .. r_{d-1} of X."""
    rmax = max(c.shape[2] for c in cores[:-1])
    return int(math.ceil(f_init * rmax))


def modewise_threshold(tol, nrmx, d):
    """Sec. 3.3: the accuracy eps is spread evenly over the d-1 bonds, so
    each mode's residual must fall below tau = eps * ||X|| / sqrt(d-1)
    (the allocation the paper justifies with its Theorem 8.6 reference)."""
    return tol * nrmx / math.sqrt(d - 1)


def round_adaptive(cores, tol, ell_block, seed, nrmx=None, f_init=0.1,
                   recompress=0, keep=False):
    """Adaptive-rank Rand-Orth-KRP (Sec. 3.3) with residual sketching.

    Returns (cores, info); the output is left-orthonormal unless recompress
    is 1 (Remark 2 pass with the same tau), then right-orthonormal.
    """
    d = len(cores)
    r0 = initial_sketch_columns(cores, f_init)
    sk = _Sketches(cores, seed, r0)
    if nrmx is None or nrmx <= 0:
        nrmx = norm_estimate(cores[0], sk.w[2])
    tau = modewise_threshold(tol, nrmx, d)
    ys = [None] * d
    y = np.array(cores[0], copy=True)
    ests, margins, kept = [], [], []
    for k in range(1, d):
        z = v_unf(y)
        rbar = min(z.shape)
        binit = max(1, min(rbar, int(math.ceil(f_init * rbar))))
        s = z @ sk.w[k + 1][:, :binit]
        q = qr_pos(s)
        m = q.T @ z
        hnext = m @ h_unf(cores[k])
        b = int(ell_block) if ell_block and ell_block > 0 else int(math.ceil(0.05 * rbar))
        mode_ests = []
        while q.shape[1] < rbar:
            bb = min(b, rbar - q.shape[1])
            s = generate_residual_sketch(sk, z, q, k, bb)
            est = float(np.linalg.norm(s) / math.sqrt(bb))
            mode_ests.append(est)
            margins.append(abs(est - tau) / tau if tau > 0 else math.inf)
            if not est > tau:
                break
            qn = qr_pos(s)
            qn = qr_pos(qn - q @ (q.T @ qn))
            q = np.concatenate([q, qn], axis=1)
            m = qn.T @ z
            hnext = np.concatenate([hnext, m @ h_unf(cores[k])], axis=0)
        ests.append(mode_ests)
        if keep:
            kept.append((z, q))
        lk = q.shape[1]
        ys[k - 1] = q.reshape(y.shape[0], y.shape[1], lk)
        _, n1, r2 = cores[k].shape
        y = hnext.reshape(lk, n1, r2)
    ys[d - 1] = y
    info = {"tau": tau, "nrmx": nrmx, "r0": r0, "ests": ests,
            "min_margin": min(margins) if margins else math.inf,
            "passes": sk.passes, "W": sk.w,
            "sketch_ranks": [1] + [int(c.shape[2]) for c in ys]}
    if keep:
        info["ZQ"] = kept
    if recompress:
        ys = recompress_rl(ys, tau=tau)
    info["ranks"] = [1] + [int(c.shape[2]) for c in ys]
    return ys, info


def partial_contractions_sum(tts, omegas, t):
    """Per-summand partial contractions with shared Omega (the remark on
    sums): W_k of the formal sum is these stacked by rows, summand order."""
    ws = [partial_contractions_rl(x, omegas, t) for x in tts]
    return {k: np.concatenate([w[k] for w in ws], axis=0) for k in ws[0]}


def round_sum_fixed(tts, ell, seed, weights=None, target_ranks=None):
    """Fixed-rank rounding of sum_i w_i X^(i): the rounding of the formal sum."""
    from .tt import formal_sum
    return round_fixed(formal_sum(tts, weights), ell, seed, target_ranks)


def round_sum_adaptive(tts, tol, ell_block, seed, weights=None, **kw):
    """Adaptive rounding of sum_i w_i X^(i): the rounding of the formal sum."""
    from .tt import formal_sum
    return round_adaptive(formal_sum(tts, weights), tol, ell_block, seed, **kw)
