"""CPU oracle for the INT8-slice FP64 GEMM emulation and the LU built on it.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product library, which must not
route through it and fails loudly when its HIP extension is missing.
The oracle and the GPU library share no code; the only common module is
``matgen`` (seeded input generators, no emulation arithmetic).

Parity status of each function (what pins it, in tests/test_oracle_pins.py):
  line_exponents, slice_digits  - frexp range identity, truncation bound,
                                  prefix property, integer inputs exact
  slice_products                - int64 brute force, integer GEMM identity
  recombine, dgemm_emu          - exact rational brute force with the
                                  round-once bound, eqn (3) example both ways,
                                  integer-exactness conditions on t
  dgemm_dd                      - exact rational brute force (tiny n)
  getf2/getrf/trsm/laswp/getrs  - Turing/Wilkinson/d-band closed forms
                                  (eqns (10)-(12)), PA = LU, LAPACK-style
                                  info on singular input
  potf2/potrf                   - closed 2 x 2 form, exact integer factors
                                  recovered at one slice, LAPACK's Cholesky,
                                  first non-positive pivot
  backward_error/scaled_residual - eqn (9) identity, exact rational residual
  gesv_ir                       - the delivered solution's double-double
                                  backward error meets the tolerance; forced
                                  failures take the fallback
  learned.features              - hand-computed statistics of small tiles,
                                  invariance under power-of-two line scaling
  learned.mlp_forward/grad      - zero weights give the uniform class
                                  distribution; central finite differences
  learned.adam_step             - first-step closed form (lr * sign(g))
  learned.decode                - hand-built cumulative distributions
  learned.tile_labels           - integer tiles of known digit counts:
                                  labels max(a + b - 1, s_lo) in closed
                                  form (several counts in one call)
  learned.getrf_tiles           - a constant slice map equals getrf; a one-
                                  slice tile leaves its backward error in
                                  that tile's columns only
(pins of the learned part: tests/test_learned_oracle.py)
"""
from .emu import (  # noqa: F401
    DIGIT_BITS, EPS, line_exponents, slice_digits, slice_products, recombine,
    dgemm_emu, dgemm_dd, rel_err_fro, getf2, trsm_unit_lower, laswp, getrf,
    getrs, residual_dd, backward_error, scaled_residual, pa_minus_lu, gesv_ir,
    potf2, potrf,
)
from ._clib import build_oracle  # noqa: F401
