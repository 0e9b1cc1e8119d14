"""CPU oracle for recursive bilinear fast matrix multiplication (arXiv 1507.00687).

TEST INFRASTRUCTURE ONLY: a plain, slow, obviously correct CPU implementation of what the
GPU path computes, used as the parity reference.  Only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import it; the product library never does, and
the two share no code.

Parity pins (tests/test_oracle_*.py) tie it to the paper: Brent equations in exact
arithmetic, Table 1 quantities, the stability vectors of the two non-uniform examples of section 5.2, exact
agreement with integer matrix products, the worked scaling examples 6.1-6.5, the closed
form of Lemma D.5 and the invariants of Lemma D.1.  Scaling at every level (a reading; the
paper prints no values for it) is pinned by exact integer products, its reduction to one
scaling at depth 1 and the per-node properties of the scaled operands.  Parity unpinned: the
distributions of the scaling study (their figure data is absent).
"""
