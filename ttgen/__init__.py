"""Seeded synthetic TT inputs shared by the oracle tests, the GPU tests and
the benchmark.  This module holds no arithmetic of the rounding method: it
only draws random cores (numpy PCG64) and lays them out, e.g. as a formal
sum whose ranks add.

The paper's own workloads (the Matern-kernel TT-cross tensor and the
TT-GMRES iterates of the parametric "cookie" PDE, Sec. 4.2-4.3) are not
available; these generators stand in for them with the shapes, ranks and
value distributions of the synthetic experiment of Sec. 4.1, at these sizes:

  c1   d=6, n=10, X = Z + 0.5 Z - 0.25 Z with Z of ranks 10, N(0,1) cores
       (formal ranks 30, true ranks 10);
  c2   sum of 4 random TTs (d=20, n=64, ranks 50, N(0,1)) with weights
       (1, 1e-2, 1e-4, 1e-6) on the first core (formal ranks 200);
  c3   d=10, n=256: left-orthonormal cores interleaved with diagonal
       singular values 10^(-(j-1)/8), j=1..200, plus a TT of ranks 100 with
       N(0, 1e-12) entries (formal ranks 300);
  c4   a batch of TTs with d in [4,16], n in [16,128], formal ranks in
       [8,128], each a sum of 3 N(0,1) TTs with weights (1, q, q^2);
  c5   Krylov-like sums of 8 TTs (d=30, n=32, ranks 50) with coefficients
       g_i 10^-i, mixed with 20% small requests (d=8, n=16, ranks 20).
  sec41  X = Y + 1e-5 Z with Y, Z normalized random TTs (Sec. 4.1 recipe).
"""

import numpy as np


def rng_for(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def clamp_ranks(dims, ranks):
    """Clamp interior ranks so that r_k <= prod(n_1..n_k) and
    r_k <= prod(n_{k+1}..n_d) (a TT never needs more)."""
    d = len(dims)
    out = list(ranks)
    for k in range(1, d):
        left = int(np.prod(dims[:k], dtype=object))
        right = int(np.prod(dims[k:], dtype=object))
        out[k] = int(min(out[k], left, right))
    out[0] = out[d] = 1
    return out


def random_tt(rng, dims, ranks, scale=1.0):
    """Cores X_k of shape (r_{k-1}, n_k, r_k) with i.i.d. N(0, scale^2)."""
    d = len(dims)
    return [scale * rng.standard_normal((ranks[k], dims[k], ranks[k + 1]))
            for k in range(d)]


def formal_sum(tts, weights):
    """sum_i w_i X^(i) as one TT: weights on the first cores (side by side),
    block-diagonal middle cores, stacked last cores."""
    d = len(tts[0])
    out = []
    for k in range(d):
        n = tts[0][k].shape[1]
        if k == 0:
            out.append(np.concatenate([w * t[0] for w, t in zip(weights, tts)], axis=2))
        elif k == d - 1:
            out.append(np.concatenate([t[k] for t in tts], axis=0))
        else:
            r0 = sum(t[k].shape[0] for t in tts)
            r1 = sum(t[k].shape[2] for t in tts)
            core = np.zeros((r0, n, r1))
            a = b = 0
            for t in tts:
                p0, _, p1 = t[k].shape
                core[a:a + p0, :, b:b + p1] = t[k]
                a += p0
                b += p1
            out.append(core)
    return [np.ascontiguousarray(c) for c in out]


def c1(seed=1001, d=6, n=10, r=10):
    rng = rng_for(seed)
    dims = [n] * d
    z = random_tt(rng, dims, clamp_ranks(dims, [1] + [r] * (d - 1) + [1]))
    return formal_sum([z, z, z], [1.0, 0.5, -0.25])


def c2_terms(seed=1002, d=20, n=64, r=50, weights=(1.0, 1e-2, 1e-4, 1e-6)):
    """The summands and weights of c2 (before forming the sum)."""
    rng = rng_for(seed)
    dims = [n] * d
    rk = clamp_ranks(dims, [1] + [r] * (d - 1) + [1])
    tts = [random_tt(rng, dims, rk) for _ in weights]
    return tts, list(weights)


def c2(seed=1002, d=20, n=64, r=50, weights=(1.0, 1e-2, 1e-4, 1e-6)):
    return formal_sum(*c2_terms(seed, d, n, r, weights))


def c3(seed=1003, d=10, n=256, r=200, noise_r=100, noise_sigma=1e-6, decay=8.0):
    """Orthonormal cores U_k (Gaussian QR) times diag(sigma) on their last
    index, sigma_j = 10^(-(j-1)/decay); the last core has orthonormal rows.
    Plus a N(0, noise_sigma^2) TT of ranks noise_r (pads formal ranks)."""
    rng = rng_for(seed)
    dims = [n] * d
    rk = clamp_ranks(dims, [1] + [r] * (d - 1) + [1])
    base = []
    for k in range(d):
        r0, r1 = rk[k], rk[k + 1]
        if k < d - 1:
            g = rng.standard_normal((r0 * n, r1))
            q, _ = np.linalg.qr(g)
            sig = 10.0 ** (-np.arange(r1) / decay)
            base.append((q * sig[None, :]).reshape(r0, n, r1))
        else:
            g = rng.standard_normal((n * r1, r0))
            q, _ = np.linalg.qr(g)
            base.append(q.T.reshape(r0, n, r1))
    nk = clamp_ranks(dims, [1] + [noise_r] * (d - 1) + [1])
    noise = random_tt(rng, dims, nk, scale=noise_sigma)
    return formal_sum([base, noise], [1.0, 1.0])


def c4_shapes(seed=1004, count=256):
    """(d, n, summand ranks) per TT of the batch."""
    rng = rng_for(seed)
    out = []
    for _ in range(count):
        d = int(rng.integers(4, 17))
        n = int(rng.integers(16, 129))
        formal = int(rng.integers(8, 129))
        s = max(1, int(round(formal / 3)))
        out.append((d, n, s))
    return out


def c4_one(seed, d, n, s, q=1e-4):
    rng = rng_for(seed)
    dims = [n] * d
    rk = clamp_ranks(dims, [1] + [s] * (d - 1) + [1])
    tts = [random_tt(rng, dims, rk) for _ in range(3)]
    return formal_sum(tts, [1.0, q, q * q])


def c4(seed=1004, count=256):
    shapes = c4_shapes(seed, count)
    return [c4_one(seed * 1000 + t, *shp) for t, shp in enumerate(shapes)]


def c5_terms(seed, small=False, terms=8):
    """The summands and coefficients of a c5 request."""
    rng = rng_for(seed)
    if small:
        d, n, r = 8, 16, 20
    else:
        d, n, r = 30, 32, 50
    dims = [n] * d
    rk = clamp_ranks(dims, [1] + [r] * (d - 1) + [1])
    tts = [random_tt(rng, dims, rk) for _ in range(terms)]
    g = rng.standard_normal(terms)
    coef = [float(g[i] * 10.0 ** (-i)) for i in range(terms)]
    return tts, coef


def c5_request(seed, small=False, terms=8):
    return formal_sum(*c5_terms(seed, small, terms))


def sum_terms(seed, d, n, r, count, weights=None):
    """count random TTs of ranks r (uniform n) and their weights (default
    1, 10^-3, 10^-6, ...), for sum-rounding tests."""
    rng = rng_for(seed)
    dims = [n] * d if np.isscalar(n) else list(n)
    rr = [1] + ([r] * (d - 1) if np.isscalar(r) else list(r)) + [1]
    rk = clamp_ranks(dims, rr)
    tts = [random_tt(rng, dims, rk) for _ in range(count)]
    if weights is None:
        weights = [10.0 ** (-3 * i) for i in range(count)]
    return tts, list(weights)


def sec41(seed=1041, d=10, n=100, r=50, eps=1e-5):
    """X = Y + eps Z with Y, Z random TTs of ranks r normalised to unit norm
    (normalisation by the exact norm from a left-to-right Gram sweep)."""
    rng = rng_for(seed)
    dims = [n] * d
    rk = clamp_ranks(dims, [1] + [r] * (d - 1) + [1])
    y = random_tt(rng, dims, rk)
    z = random_tt(rng, dims, rk)

    def _norm(cs):
        g = np.ones((1, 1))
        for c in cs:
            g = np.einsum('ab,aic,bid->cd', g, c, c)
        return float(np.sqrt(g[0, 0]))

    ny, nz = _norm(y), _norm(z)
    return formal_sum([y, z], [1.0 / ny, eps / nz])


def small_random(seed, d, n, r):
    """A tiny random TT (uniform n and r), for edge-case tests."""
    rng = rng_for(seed)
    dims = [n] * d if np.isscalar(n) else list(n)
    rr = [1] + ([r] * (d - 1) if np.isscalar(r) else list(r)) + [1]
    return random_tt(rng, dims, clamp_ranks(dims, rr))
