"""Plain FP64 CPU oracle for the compactly-supported RBF approximation.

TEST INFRASTRUCTURE ONLY.  This package exists so that the HIP path can be
checked against a slow, obviously correct CPU computation written from the
paper.  Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import it; the library itself never does, and it shares no code
with the HIP kernels.

Contents
--------
``rbf_oracle``   basis functions, support predicate, design matrix A, normal
                 equations B = A^T A and g = A^T h, direct solve, evaluation,
                 sampled single-row recomputation, COO sparse product.
``mlp_oracle``   FP64 forward / backward / Adam for the 16-64-64-1 radius MLP
                 and the density features it reads.

Parity status of every function is stated in its module header.
"""
