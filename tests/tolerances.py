"""Numeric bars shared by the GPU parity tests.

The float64 path is held to relative 1e-10 on the fitted values,
||A (c - c*)||_2 / ||A c*||_2, with c* the oracle's Cholesky solution.  For the
normal-equation residual r = g - B c this error is at most
(||r|| / ||g||) sqrt(kappa(B)), so the GPU solves the parity cases to a
relative residual of 1e-13: the bar then holds up to kappa = 1e6 by the bound,
and in practice far beyond (the residual is spread over many eigenvectors).
"""
FP64_RTOL = 1e-13   # relative residual the float64 parity solves run to
FIT_FP64 = 1e-10    # relative error of the fitted values A c against the oracle's
