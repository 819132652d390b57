"""FP64 CPU oracle for the coherent-dedispersion correlator.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call or link anything in this package; it exists so
that the tests, the smoke check and the CPU-baseline leg of the benchmark can
check the GPU path against a plain, slow, obviously correct implementation of
what Bannister & Cornwell (2011), "The Chirpolator and The Chimageator", define:

* the cold-plasma dispersion law (Sec. 2.1, Eq. dmdelay) and, from it, the
  coherent-dedispersion filter H(f, DM) (Sec. 2.3.2: convolve the voltages with
  the impulse response of the inverse of the ISM);
* the product of one antenna's voltage with another's conjugate (the
  "mixing" of Sec. 3.2, Eq. xpq), integrated and dumped at a fixed cadence
  (Sec. 5.1, the integrate-and-dump boundary of the cost model);
* the block partial DFT of Appendix A.3 (Eq. block_cic), whose k = 0 term is
  the integrate-and-dump of the mixed product;
* in ``oracle.chirpolator``, the Chirpolator pre-integrator itself (Sec. 3.2,
  App. A.3): mixing of antenna pairs, block partial DFTs over the bins
  |k| <= kmax, the block CIC moving sum, the closed form of a mixed chirp's DFT,
  the DFT factorisation across lengths and the shared negative-bin products;
* in ``oracle.imaging``, the post-integrator detection image P(theta) and
  E(theta) (Sec. 3.3, 3.4, App. A.1): 3-D baseline delays, the tone bin k0',
  the matched filter over 2F + 1 bins and the vector sum over pairs;
* in ``oracle.incoherent``, classical incoherent dedispersion of power beams
  (Sec. 2.3.1, 2.4.1): brute force over the delays of Eq. dmdelay, and the tree
  method for linear sweeps;
* in ``oracle.chimageator``, the Chimageator on a uniform linear array (Sec. 4):
  gridding of redundant spacings, block integration, the spatial DFT and the
  phase-corrected trajectory sums.

Everything is numpy in float64 / complex128.  The oracle shares no code with the
GPU path; only the seeded input generators (package ``synth``) serve both.
"""

from .dedisp import (  # noqa: F401
    K_DM,
    smear_samples,
    blocking,
    bin_offsets,
    chirp_cycles,
    chirp,
    dedisperse_stream,
    correlate_dumps,
    packed_index,
    pack_upper,
    run_oracle,
    channel_delays,
    dump_times,
)
from .quant import e4m3_quantize, e4m3_decode_table, fp16_quantize, quantize  # noqa: F401
