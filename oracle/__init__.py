"""FP64 CPU oracle of the CPRA hot path.

TEST INFRASTRUCTURE: only tests/, the smoke check in __graft_entry__ and the
benchmark's cpu_baseline leg may import this package.  The product library
never calls it and shares no code with it.

Modules:
  fft    - own FFT (direct DFT <= 32 points, radix-2 combine steps above)
  rng    - counter-based SplitMix64 for the initial phases
  cpra   - input prep, W_0, carousel coupling (Eq. 4), HIO/ER, error
  stepd  - literal Fourier-slice insertion + 3D inverse FFT (step D)
  geometry - exact voxel projections at 0 and 90 degrees (for pins)

Parity pins (tests/test_oracle_*.py): brute-force DFT, numpy.fft,
Parseval, Fourier slice theorem on 16^3 objects, closed-form HIO/ER steps,
the fixed point of a true object, ER error monotonicity, the mirror seam
against directly projected neighbours, step D against numpy's inverse FFT of
an exactly sliced spectrum, published SplitMix64 outputs.
"""
from .cpra import Oracle, HIO, ER, WRAP_MIRROR, WRAP_PLAIN  # noqa: F401
