"""FP64 CPU oracle for randomized HSS compression, matvec and ULV solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything under ``oracle/``; only the test-suite, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the GPU library
(the two are independent implementations of the same paper,
Rouet/Li/Ghysels/Napov, "A distributed-memory package for dense Hierarchically
Semi-Separable matrix computations using randomization", arXiv 1503.05464).

It is deliberately plain: NumPy/SciPy in float64, loops over tree nodes, no
blocking, fusion or reordering beyond what the paper's algorithms state.

Modules
-------
philox   Philox4x64-10 counter-based generator + Box-Muller Gaussian columns
tree     binary cluster tree by interval bisection (Sec. 2.1)
interp   interpolative decomposition by column-pivoted Householder QR with the
         relative stopping rule R_ii/R_11 <= eps (Sec. 2.2, Sec. 3.2)
hss      Alg. 1 compression with the late-notification adaptive sampling of
         Alg. 5 run level-synchronously (Sec. 3.3); Alg. 2 matvec; dense
         reconstruction from the nested-basis definition (Eqs. 1-4)
ulv      Alg. 3 ULV-like factorization and Alg. 4 solve (Sec. 2.4-2.5, App. A)

Pins (what ties each function to the paper and to mathematics rather than to
itself) are listed in the tests ``tests/test_oracle_*.py``; the "parity
unpinned" items, if any, are named in the module docstrings.
"""
