"""FP64 CPU oracle for ball-harmonic rotational matching.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that the
GPU library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it; the product path
(``paper_2509_01180_amd``) never does, and the two share no code.

Every function follows the paper's definitions directly (Section II):

* ``basis``   -- ball harmonics psi_klm, Bessel zeros lambda_lk, the
                 frequency-ordered index set (Sec. II-A).
* ``expand``  -- coefficients of a voxel volume by midpoint quadrature.
* ``wigner``  -- Wigner small-d / D matrices, Euler angles, rotation metrics.
* ``score``   -- the per-degree cross-power xi^l and the rotational
                 cross-correlation of Eq. (2) with its Euler gradient.
* ``align``   -- frequency marching with multi-start gradient ascent
                 (Sec. II-C).

Readings where the paper is silent are documented in each module and in the
repository's design notes.
"""

from . import basis, expand, wigner, score, align  # noqa: F401
