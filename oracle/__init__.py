"""FP64 CPU oracle for the Zolotarev spectrum-filter eigensolver (Li & Yang).

TEST INFRASTRUCTURE ONLY.  Nothing in the product library may import, call,
link or execute anything in this package: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use it.
It shares no code with the GPU path; the only common module is ``pencils``
(seeded input construction, no method arithmetic).

Layout (each function cites the passage of the paper it follows):

* ``elliptic``  : complete elliptic integral K and Jacobi sn, cn, dn by the
  arithmetic-geometric mean (descending Landen) method.
* ``zolotarev`` : Zolotarev's function Z_2r(x; l) (Theorem 1, eq. ZoloFunc,
  coef), its error delta, the rescaled function (eq. rZ), composition
  (Theorem 2), partial fractions (Proposition 1, Corollary 1, Proposition 2).
* ``mobius``    : the Moebius map T(x) = gamma (x - alpha)/(x - beta) fixed by
  the eigengaps (eq. mo, eq. req).
* ``filt``      : the full coefficient plan of Algorithm 2 (lines 2-4) and the
  scalar filter R_ab(x) (eq. R2) evaluated two ways.
* ``dense``     : dense pencil eigensolver (Cholesky-reduced cyclic Jacobi),
  the exact matrix filter R_ab(B^-1 A) V and the operator G (eq. solve).
* ``subspace``  : Algorithm 1 with the exact filter (reference decay).
* ``sparse``    : large-N oracle: Sylvester inertia counts, shift-invert
  Lanczos windows, Kato-Temple bounds and a CPU Algorithm 1+2 baseline.

Parity status: every function is pinned by ``tests/test_oracle_*.py`` against
closed forms, invariants, mpmath, LAPACK or brute force, except the CPU
Algorithm 1+2 baseline's timing figures (a reported baseline, not a pin).
"""
