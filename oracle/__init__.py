"""FP64 CPU oracle for randomized block Gram-Schmidt (RBGS) QR.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or execute anything in this package; it
exists so that tests, the smoke check and the CPU-baseline leg of the
benchmark can check the GPU results against a plain, slow, obviously correct
implementation written from the paper (Balabanov & Grigori, "Randomized block
Gram-Schmidt process for the solution of linear systems and eigenvalue
problems", arXiv 2111.14641).

It shares no code with the GPU path.  The only thing both sides implement is
the *definition* of the sketching operator Theta (a counter-based Philox
generator and the maps from its output words to matrix entries); each side
implements that definition independently.

Modules
-------
philox   Philox-4xW-R counter-based generator (Salmon et al., SC'11).
theta    The sketching operators: Gaussian (Philox + Box-Muller written with
         basic IEEE single-precision operations only), sparse-sign (block
         CountSketch construction), and the identity.
rbgs     RBGS QR (Algorithm "RBGS" of Section 2 with steps 4-5 done either by
         RCholeskyQR or by RCholeskyQR with postponed sketching), the
         least-squares solvers of Section 2.1 and of the supplement, and the
         a-posteriori certificates of step 6.
metrics  Result metrics (factorization error, condition number, loss of
         sketched orthogonality).

Parity status of each function is stated in its docstring; every function
here is pinned by a test in tests/test_oracle_*.py against something other
than itself (a library routine, a closed form, an invariant or a bound from
the paper).
"""
