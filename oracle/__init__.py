"""CPU FP64 oracle for the Helmholtz FMM / BIE / GMRES hot path.

TEST INFRASTRUCTURE ONLY.  This package is a slow, plain reference written
from the paper (arXiv 1803.09948, "Extreme Scale FMM-Accelerated Boundary
Integral Equation Solver for Wave Scattering") and from textbook definitions.
Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import it.  It shares no code, headers, tables or constant generators with the
HIP library; the only common module is the seeded input generator `synth`,
which holds none of the method's arithmetic.

Modules
  special   spherical harmonics and spherical Bessel/Hankel functions (scipy)
  gaunt     Wigner 3j symbols (Racah formula, exact integers) and Gaunt integrals
  expansions solid harmonics, P2M/L2P and the translation operators (R|R), (S|R)
  tree      root cube, Morton keys, adaptive octree and dual tree traversal lists
  fmm       direct sum (eq. 11) and the CPU FMM matvec (Sec. 2.3)
  bie       flat-panel collocation matrix for eq. (7): Gauss points, near and
            self-panel integrals (Sec. 2.2, Listing 1 branches)
  gmres     dense restarted GMRES with modified Gram-Schmidt
  mie       Mie series for the sound-soft sphere (Sec. 6.4 observable)

Where the paper is silent or ambiguous, each function states the reading it
implements.

Parity status: every function here is pinned by a CPU test against a closed
form, an identity, brute force or a special case (tests/test_oracle_*.py);
none is "parity unpinned".
"""
