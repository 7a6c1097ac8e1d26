"""CPU FP64 oracle for the coset probabilities of a detector error model.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library, its
Python binding, the benchmark's timed path) imports, links or calls this
package; only the tests, the smoke check and the benchmark's CPU-baseline leg
do.  It shares no code with the GPU path.

Tiers (each module's header says what pins it):
  exact.py    O-1 brute force over error patterns / Paulis (the plain
              definition of p_{m,L}, paper Sec. 2.3-2.4);
              O-2 exact frontier contraction (variable elimination) of the same
              sum, in FP64 with a log-scale accumulator.
  network.py  the layered networks of the configurations, written from the
              paper's detector picture (Sec. 3.1, 3.3, 3.4, 5.1), the loop
              sector in the generator picture (Sec. 3.2), and the signed
              Walsh-Hadamard networks Z_b of the coset selection (Sec. 3.1).
  sweep.py    O-3 the fixed-chi boundary sweep with simple-update truncation
              (Sec. 4) followed by the boundary-MPS contraction of the final 2D
              network, with LAPACK QR/SVD; a signed variant for Z_b.
  grad.py     O-4 the exact gradient of log P(m) with respect to every
              mechanism rate (the affine split of P(m) in each rate, on O-2),
              the chain rule to shared rates, and central finite differences
              (of O-2, or of O-3 for the approximate value).

Parity unpinned: the boundary-MPS truncation in rows after the first (the
zip-up has no reduction to an optimal truncation there); it is pinned only
by the exact limit.
"""
