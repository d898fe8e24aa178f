"""CPU oracle for weighted-quadrature mass-matrix formation on trimmed patches.

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it. It shares no code with the HIP library; both read
their inputs from ``paper_2101_08053_amd.workloads`` and nothing else.

It is a plain, slow, fp64 statement of what the method computes, written from
Marussig, "Fast formation and assembly of isogeometric Galerkin matrices for
trimmed patches" (arXiv 2101.08053):

* ``bspline``    -- B-splines of Sect. 2.1 (definition by recursion) and Eq. (1).
* ``quadrature`` -- Gauss-Legendre rules (library routine).
* ``wq``         -- weighted quadrature, Eqs. (4)-(5): point layout and weights.
* ``curves``     -- trimming curves of Sect. 2.2 and their crossings.
* ``trim``       -- element and function classes (Sect. 2.2), domain split
                    Eq. (8), and the cut-element rule (Sect. 3.1).
* ``geometry``   -- the pull-back coefficient c = |det J| (Sect. 2.1).
* ``assemble``   -- element Gauss reference, weighted-quadrature rows Eqs.
                    (6)-(7), hybrid Gauss (Sect. 3.2), naive weighted quadrature
                    on cut rows (Sect. 4.1, Table 1).
* ``dwq``        -- discontinuous weighted quadrature (Sect. 3.3, Eqs. (9)-(10)).
* ``project``    -- L2 projection (Sect. 4.2).
* ``matfree``    -- matrix-free product y = M(c) u and its gradient.

Pins (tests/test_oracle_*.py) tie every function to something other than
itself: library routines, closed forms, exact rationals, invariants and brute
force. Readings of passages where the paper is silent are listed in the module
that takes them.
"""
