"""FP64 CPU oracle for fast-convolution (FC) filtered CP-OFDM.

This package is TEST INFRASTRUCTURE. Only the test-suite, the smoke check in
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it. The product (the C-ABI library and its Python binding) never imports,
links or executes anything here, and this package imports nothing from the
product. Both sides share only the seeded input generators in ``fcsynth``.

Modules
-------
numerology  NR cyclic-prefix rule, overlap split, block and symbol schedules.
fc          The exact FC method (literal evaluation of the paper's block
            matrices with dense DFT matrices), TX and RX, all processing models.
lin         What FC approximates: direct linear convolution with one centred
            period of the FC kernel ("plain" reference), TX and RX.
weights     Raised-cosine transition-band weights (reading of the paper's
            unspecified transition weights).
metrics     OFDM demodulation, EVM, out-of-band leakage, complexity formula.
"""
from . import numerology, fc, lin, weights, metrics  # noqa: F401
