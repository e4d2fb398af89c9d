"""CPU oracle for the RJSMC hot path -- TEST INFRASTRUCTURE.

Plain FP64 implementations, written from the paper, that the HIP path is checked
against.  Only the test suite, the smoke check and the CPU-baseline leg of the bench
may import anything from this package; the product path never does.

    em   forward model (Cole-Cole, layered-earth TE recursion, J1 Hankel filter,
         frequency-to-time transform with gates), Gaussian log-likelihood, and its
         gradient by forward-mode tangents
    smc  Philox4x32-10, prior, tempering bisection on the total effective sample size,
         reweighting and evidence, within-model systematic resampling, RJ-MCMC
         mutation, and the Algorithm-1 driver; conjugate-Gaussian evidence toy
"""
