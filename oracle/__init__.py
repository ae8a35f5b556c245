"""CPU oracle for the bosonic many-body operators of arXiv:2005.13679.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import, call, link or execute anything in
this package.  The GPU library never uses it and shares no code with it.

The oracle is plain and slow on purpose, and follows the paper's definitions:

* ``combinatorics`` -- Eq. (nc) for the dimension, the index of a
  configuration as the particle cost sum of Eq. (TotalCost) (the map of
  Algorithm 1) and its inverse by bisection (the map of Algorithm 2), in pure
  Python, plus an enumeration of all configurations that does not use the
  hash.
* ``native`` -- the same maps in plain C (``mc_oracle.c``), plus the
  single/double jump maps by definition and H.C, rho1, rho2 by applying
  creation/annihilation operators to occupation vectors.
* ``dense`` -- textbook brute force: Kronecker-product ladder operators over
  (N+1)^M single-mode states, restricted to N particles.
* ``lanczos`` -- Lanczos with full reorthogonalisation and a tridiagonal
  eigensolver (Sec. VI).
* ``bethe`` -- Newton solver for the Lieb-Liniger Bethe-ansatz equations
  (Eqs. LLsystem and LLE0).

Every function of the oracle is pinned by tests that do not re-use it: values
the paper prints, closed forms, invariants and brute force.
"""
