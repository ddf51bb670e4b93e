"""FP64 CPU oracle for randomized T-HOSVD / ST-HOSVD with adaptive shifted power iteration.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package. The product path (the
HIP library and its Python binding) never imports, calls or links it, and this
package imports nothing from the product.

Contents:
  philox   - Philox4x32-10 counter-based generator and the Box-Muller map that
             defines the Gaussian test matrices Omega_k; the uniform and
             Khatri-Rao test matrices of the same streams.
  tensor   - mode-k unfolding, folding, mode-k product, Frobenius norms.
  rhosvd   - the method itself (shifted randomized T-HOSVD and ST-HOSVD, the
             unshifted model, the deterministic HOSVD, the power count chosen
             per mode by the per-vector-error test) step by step in FP64.

Parity status: every function is pinned by tests under tests/ against values
the paper prints, closed forms, invariants or brute force (test_oracle_*.py
name the pin of each function). No function here is "parity unpinned".
"""
