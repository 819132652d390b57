"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This package holds no part of the method's arithmetic (no dedispersion, no
correlation); it only builds voltage streams with the shapes and statistics of
the workloads, and injects dispersed pulses with a forward model of the sky:

* noise: circular complex Gaussian; "unit variance" means E|n|^2 = 1; the
  complex-int8 form rounds each component of N(0, sigma^2) half-to-even and
  clips it to [-127, 127];
* a pulse is complex Gaussian noise of the source under a boxcar of ``width``
  samples, identical at every antenna up to a geometric delay or phase,
  delayed in each frequency by the cold-plasma law of Eq. dmdelay (Sec. 2.1):
  higher frequencies arrive first;
* amplitude: single-antenna boxcar matched-filter S/N, a^2 = SNR sigma_n^2 / sqrt(w).

The generators take every random draw from numpy PCG64 (seeded) on the host,
or from torch's seeded device generator for the large streams.
"""

from .signals import (  # noqa: F401
    K_DM_SKY,
    chan_freqs,
    dm_grid,
    noise_complex,
    to_ci8,
    antenna_positions,
    direction_grid,
    dispersed_segment,
    inject_pulse,
    pulse_wave,
    make_c0,
    make_small,
    c1_params,
    c3_params,
    make_stream_device,
)
from .power import power_batch, sample_pulses  # noqa: F401
