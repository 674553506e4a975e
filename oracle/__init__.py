"""CPU oracle for the two-site DMRG middle-site step (TEST INFRASTRUCTURE).

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import anything from this package.  The product
path (the HIP library and its Python binding) never imports, links or calls
it, and this package imports nothing from the product.

* ``oracle.fci``      -- O1, the definition: the determinant-space
  Hamiltonian built from the integrals (Appendix B, ab initio Hamiltonian)
  and the embedding W of the two-site space, so H_eff psi = W^T H W psi.
* ``oracle.blockops`` -- O2, plain FP64 renormalized-operator algebra:
  blocking (Appendix A, blocking formula), transformation (Appendix A,
  operator transformation) and the normal/complementary left-right
  decomposition, with every enlarged operator materialised.
* ``oracle.share``    -- integral masking of the sum of sub-Hamiltonians
  (Section II.B, processor assignment).

All arithmetic is float64.  Pins that tie these to something other than
themselves live in ``tests/test_oracle_*.py``.
"""
