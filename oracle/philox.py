"""Philox4x32-10 and the Gaussian mode factors Omega_j (oracle side).

The paper draws the mode factors Omega_j (n_j x ell) with i.i.d. N(0,1)
entries (Sec. 2.3, Sec. 3.2, Algorithm "Residual sketching ... using KRPs")
and uses MATLAB's ``randn``; it fixes no generator.  This library fixes one so
that the GPU and the oracle draw the same numbers, each side implementing it
independently from its published definition:

* Philox4x32-10 (J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw,
  "Parallel random numbers: as easy as 1, 2, 3", SC'11): a 4x32-bit counter
  and a 2x32-bit key, ten rounds of two 32x32->64 multiplies with key bumps
  by the Weyl constants between rounds.
* Box-Muller (G. E. P. Box and M. E. Muller, 1958) turning two uniforms in
  (0,1) into two independent N(0,1) values.

Addressing (the build's own spec, identical on both sides):

  key     = (seed mod 2^32, seed >> 32)
  counter = (p, c, j, 0x4B525031)   p = row pair, c = global sketch column,
                                    j = mode index (1-based, as in the paper)
  u1 = (((w0 * 2^32 + w1) >> 11) + 0.5) * 2^-53,   u2 likewise from (w2, w3)
  Omega_j(2p,   c) = sqrt(-2 ln u1) * cos(2 pi u2)
  Omega_j(2p+1, c) = sqrt(-2 ln u1) * sin(2 pi u2)     (if 2p+1 < n_j)

Because every entry is addressed by (seed, j, c, i), a column of a partial
contraction W_k is the same whenever and in whatever chunk it is generated.

Parity: the raw words are pinned to the Random123 known-answer vectors in
``tests/golden/philox4x32_10_kat.txt``; the Gaussians by moment and KS tests.
"""

import numpy as np

PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
OMEGA_TAG = 0x4B525031
_MASK32 = np.uint64(0xFFFFFFFF)
_TWO_PI = 6.283185307179586


def philox4x32_10(ctr, key):
    """Apply Philox4x32-10 to arrays of counters.

    ctr: uint32 array of shape (..., 4); key: uint32 array of shape (..., 2)
    (broadcastable).  Returns uint32 array of shape (..., 4).
    """
    c = np.asarray(ctr, dtype=np.uint64)
    k = np.asarray(key, dtype=np.uint64)
    c0, c1, c2, c3 = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
    k0, k1 = k[..., 0], k[..., 1]
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + np.uint64(PHILOX_W0)) & _MASK32
            k1 = (k1 + np.uint64(PHILOX_W1)) & _MASK32
        p0 = PHILOX_M0 * c0          # exact: both factors < 2^32
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    out = np.stack(np.broadcast_arrays(c0, c1, c2, c3), axis=-1)
    return out.astype(np.uint32)


def _uniform53(whi, wlo):
    """Two 32-bit words -> uniform in (0,1) with 53 random bits."""
    v = (whi.astype(np.uint64) << np.uint64(32)) | wlo.astype(np.uint64)
    v = v >> np.uint64(11)
    return (v.astype(np.float64) + 0.5) * (2.0 ** -53)


def gaussian_factor(seed, mode, n, col0, ncols):
    """Omega_mode(:, col0:col0+ncols) as an (n x ncols) float64 array.

    mode is the 1-based TT mode index j; columns are global sketch columns.
    """
    seed = int(seed)
    npairs = (n + 1) // 2
    p = np.arange(npairs, dtype=np.uint64)[:, None]
    c = np.arange(col0, col0 + ncols, dtype=np.uint64)[None, :]
    ctr = np.empty((npairs, ncols, 4), dtype=np.uint64)
    ctr[..., 0] = p
    ctr[..., 1] = c
    ctr[..., 2] = np.uint64(mode)
    ctr[..., 3] = np.uint64(OMEGA_TAG)
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint64)
    w = philox4x32_10(ctr, key)
    u1 = _uniform53(w[..., 0], w[..., 1])
    u2 = _uniform53(w[..., 2], w[..., 3])
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = _TWO_PI * u2
    out = np.empty((2 * npairs, ncols), dtype=np.float64)
    out[0::2, :] = rad * np.cos(ang)
    out[1::2, :] = rad * np.sin(ang)
    return out[:n, :]


def gaussian_factors(seed, n_list, modes, col0, ncols):
    """Dict mode -> Omega_mode(:, col0:col0+ncols) for 1-based modes."""
    return {j: gaussian_factor(seed, j, n_list[j - 1], col0, ncols) for j in modes}
