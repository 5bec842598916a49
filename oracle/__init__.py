"""CPU FP64 oracle for KRP-sketched TT-rounding (test infrastructure only).

This package is the independent reference that the GPU library is checked
against.  It is plain NumPy/SciPy in float64 on the host, written from the
paper (Al Daas, Ballard, Grigori, Martinez Aguilar, Saibaba, Verma,
"Adaptive Randomized Tensor Train Rounding using Khatri-Rao Products",
arXiv 2511.03598) and shares no code with the HIP path: it imports nothing
from ``paper_2511_03598_amd`` and the library never imports it.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  The product path must never route through it.

Modules
-------
philox   Philox4x32-10 counter-based generator and the Gaussian mode factors
         (the paper draws Gaussian matrices; the generator spec is ours,
         see the module docstring).
tt       TT utilities: unfoldings, full reconstruction, right-to-left
         orthogonalization, stable norm and difference norm, formal sums.
ttsvd    Deterministic TT-rounding (Algorithm "TT-Rounding", Sec. 2.2).
krp      KRP partial contractions (Eq. 6-8, Algorithm "KRP-PartialContractionsRL"),
         fixed-rank Rand-Orth-KRP (Sec. 3.2), residual sketching and the
         adaptive Rand-Orth-KRP (Sec. 3.3), the norm estimate (Remark 1) and
         the recompression pass (Remark 2).

Parity status: every public function is pinned by a ``-m "not gpu"`` test in
``tests/test_oracle_*.py`` against a closed form, a brute-force computation,
a textbook special case or published test vectors.
"""

from . import philox, tt, ttsvd, krp  # noqa: F401
