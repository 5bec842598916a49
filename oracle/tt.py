"""TT-format utilities for the oracle (test infrastructure, CPU FP64).

Conventions (Sec. 2.2, Eq. 1-4 of the paper):
  * a TT tensor is a list of cores X_k of shape (r_{k-1}, n_k, r_k) with
    r_0 = r_d = 1, stored row-major;
  * the vertical unfolding V(X_k) is the (r_{k-1} n_k) x r_k matrix and the
    horizontal unfolding H(X_k) the r_{k-1} x (n_k r_k) matrix; in row-major
    storage both are plain reshapes (column index of H is i*r_k + b);
  * ||X|| is the Frobenius norm of the full tensor.

The norm and the difference norm are computed through right-to-left
orthogonalization (Sec. 2.2, the OrthogonalizeRL step of TT-Rounding):
after it, ||X|| = ||X_1||_F.  For a difference the formal difference TT
[A, -B] is orthogonalized, which stays accurate to O(u (||A|| + ||B||)),
unlike expanding <A,A> - 2<A,B> + <B,B>, which floors near sqrt(u).
"""

import numpy as np


def ranks_of(cores):
    return [1] + [int(c.shape[2]) for c in cores]


def dims_of(cores):
    return [int(c.shape[1]) for c in cores]


def h_unf(core):
    r0, n, r1 = core.shape
    return core.reshape(r0, n * r1)


def v_unf(core):
    r0, n, r1 = core.shape
    return core.reshape(r0 * n, r1)


def full(cores):
    """Dense tensor X(i_1..i_d) = X_1(:,i_1,:) ... X_d(:,i_d,:) (Eq. 1)."""
    acc = cores[0].reshape(cores[0].shape[1], cores[0].shape[2])
    shape = [cores[0].shape[1]]
    for c in cores[1:]:
        r0, n, r1 = c.shape
        acc = acc @ c.reshape(r0, n * r1)
        shape.append(n)
        acc = acc.reshape(-1, r1)
    return acc.reshape(shape)


def orthogonalize_rl(cores):
    """Right-to-left orthogonalization (Sec. 2.2): H(X_k)^T = QR for
    k = d..2, H(Y_k) = Q^T, V(Y_{k-1}) = V(X_{k-1}) R^T.  Returns a
    right-orthonormal TT equal to the input; Householder QR (LAPACK)."""
    ys = [np.array(c, dtype=np.float64, copy=True) for c in cores]
    d = len(ys)
    for k in range(d - 1, 0, -1):
        r0, n, r1 = ys[k].shape
        q, r = np.linalg.qr(h_unf(ys[k]).T)          # (n r1) x m, m x r0
        m = q.shape[1]
        ys[k] = q.T.reshape(m, n, r1)
        p0, pn, _ = ys[k - 1].shape
        ys[k - 1] = (v_unf(ys[k - 1]) @ r.T).reshape(p0, pn, m)
    return ys


def norm(cores):
    """||X|| via right-to-left orthogonalization."""
    ys = orthogonalize_rl(cores)
    return float(np.linalg.norm(ys[0]))


def formal_sum(tts, weights=None):
    """Formal sum sum_i w_i X^(i): first cores side by side (weights applied
    there), middle cores block diagonal, last cores stacked.  Ranks add."""
    s = len(tts)
    if weights is None:
        weights = [1.0] * s
    d = len(tts[0])
    out = []
    for k in range(d):
        ns = tts[0][k].shape[1]
        if d == 1:
            core = sum(w * t[0] for w, t in zip(weights, tts))
            out.append(np.array(core))
            continue
        if k == 0:
            out.append(np.concatenate([w * t[0] for w, t in zip(weights, tts)], axis=2))
        elif k == d - 1:
            out.append(np.concatenate([t[k] for t in tts], axis=0))
        else:
            r0 = sum(t[k].shape[0] for t in tts)
            r1 = sum(t[k].shape[2] for t in tts)
            core = np.zeros((r0, ns, r1))
            a = b = 0
            for t in tts:
                p0, _, p1 = t[k].shape
                core[a:a + p0, :, b:b + p1] = t[k]
                a += p0
                b += p1
            out.append(core)
    return out


def diff_norm(a, b):
    """||A - B|| computed stably from the formal difference [A, -B]."""
    return norm(formal_sum([a, b], [1.0, -1.0]))


def rel_err(x, y):
    return diff_norm(x, y) / norm(x)


def left_orth_defect(cores):
    """max_k ||V(Y_k)^T V(Y_k) - I||_max for k < d (left orthonormality)."""
    worst = 0.0
    for c in cores[:-1]:
        v = v_unf(c)
        worst = max(worst, float(np.abs(v.T @ v - np.eye(v.shape[1])).max()))
    return worst


def right_orth_defect(cores):
    """max_k ||H(Y_k) H(Y_k)^T - I||_max for k > 1 (right orthonormality)."""
    worst = 0.0
    for c in cores[1:]:
        h = h_unf(c)
        worst = max(worst, float(np.abs(h @ h.T - np.eye(h.shape[0])).max()))
    return worst


def inner(a, b):
    """<A, B> by a left-to-right contraction (used only where sqrt(u)
    relative accuracy is enough, e.g. statistical tests)."""
    acc = np.ones((1, 1))
    for ca, cb in zip(a, b):
        # acc: ra x rb ; new(ra', rb') = sum_{a,b,i} acc(a,b) A(a,i,a') B(b,i,b')
        acc = np.einsum('ab,aic,bid->cd', acc, ca, cb)
    return float(acc[0, 0])
