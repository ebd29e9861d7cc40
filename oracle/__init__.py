"""Independent FP64 checker for the run-time Haar-domain relighting path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke entry point and the
benchmark's CPU-baseline leg may import or run anything in this package.  It
shares no code with the HIP library and imports nothing from it; the only
thing both sides consume in common is the seeded scene data of `scenes`.

Everything here follows the paper's definitions directly, written for
clarity rather than speed:
  * haar      -- orthonormal non-standard 2-D Haar per cube face (Sec. V.B:
                 H/V/D coefficients are finite differences at every scale).
  * sphere    -- rotation of a cube-map signal on the sphere, g(w) = f(R w)
                 (Sec. V.A, rotated-point relations), in exact integer
                 geometry.
  * select    -- non-linear approximation: keep the largest coefficients
                 (Sec. III, Haar-domain methods).
  * relight   -- outgoing radiance as the inner product of transfer and
                 rotated lighting (Sec. III, transfer function; Sec. V.C, last
                 algorithm step), evaluated as pixel rotate -> forward Haar ->
                 dense dot.
  * mlp       -- reference forward/backward of the learned transport decoder.
"""
