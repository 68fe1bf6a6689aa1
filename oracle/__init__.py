"""CPU oracle for the FOSSILS / SPIR least-squares path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct float64 numpy code written from the paper (Epperly, Meier and
Nakatsukasa, "Fast randomized least-squares solvers can be just as accurate and stable as
classical direct solvers").  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  The HIP library never calls it, shares no
code with it, and the product path has no CPU fallback.

Modules
  philox          Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11) and
                  the sparse-sign column index/sign stream built on it.
  sketch          sparse sign embedding S (Section 4.2, "Choice of embedding") and S[A b].
  householder     textbook Householder QR and the QR least-squares solver (Section 1; the
                  classical backward-stable baseline).
  backward_error  Karlson-Walden estimate, its sketched variant (Section 4.1, eq:sketched-kw) and
                  the exact Walden-Karlson-Sun-Higham backward error for tiny inputs.
  solvers         sketch-and-solve, FOSSILS (Algorithms 2, 4 and 5), SPIR with CG (Algorithm 3),
                  and the single passes A^T(A z) / b - A x that the refinement loop is built on.

Pins (tests/test_oracle_*.py) tie every function to something other than itself; functions
without one say "parity unpinned" in their docstring.
"""
