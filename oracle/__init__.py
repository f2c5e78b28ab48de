"""FP64 CPU oracle of the OPO split-step Fourier hot path.

Test infrastructure only: the test suite, the smoke check and the CPU leg of
the benchmark use it. The GPU library never imports, links or calls it.
"""
from .oracle import (  # noqa: F401
    Crystal, Cavity, build, fft, ifft, kappa, kerr, omega, dispersion, rk4, linear,
    ssfm_pass, ssfm_pass_unsym, gdd, eom, roundtrips, roundtrips_record,
    roundtrips_multi, propagate_adaptive,
)
