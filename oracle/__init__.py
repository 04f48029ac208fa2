"""CPU oracle for the click-probability hot path.  TEST INFRASTRUCTURE ONLY.

Only the tests, the package smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never calls, links or imports it, and
this package never imports the GPU library.

Every function is a plain, slow transcription of a definition or of the
paper's procedure (Popova & Rubtsov, "Cracking the Quantum Advantage threshold
for Gaussian Boson Sampling"), cited by section and equation:

  model.py    covariance of the lossy output state; the paper's X matrix
  exact.py    exact click probability by inclusion-exclusion over the click
              projector (fp64, numpy); exact128.c does the same in binary128
  sectors.py  photon-number sector weights of the sub-ensemble and their
              cluster moments, as power-series coefficients (no contour)
  fit.py      the per-sector exp-polynomial fit to the moments
  approx.py   the order-j estimate of a click-pattern probability
  fock.py     truncated Fock-basis brute force for tiny inputs
  grad.py     central finite differences of the oracle's log-probabilities

Precision: fp64 throughout, except the exact path's reference, which runs in
binary128 because the signed 2^n-term sum cancels by up to ~1e11.
"""
