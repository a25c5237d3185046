"""FP64 CPU oracle for the particle-mesh step with compressed particles.

TEST INFRASTRUCTURE ONLY. This package is the plain, slow, obviously correct statement
of what the step computes, written from the paper (Emberson et al., "Cosmological
neutrino simulations at extreme scale", arXiv:1611.01545) and used only to check the
HIP path. Only the tests, the smoke check and the bench's CPU-baseline leg may import
it; the product library never calls it, and it shares no code with the HIP path.

Everything is numpy in float64. Library primitives serve as steps where noted
(numpy.fft for the discrete Fourier transforms, numpy.bincount for scatter-adds,
numpy.argsort(kind="stable") for the stable cell sort, scipy.special.k1 for the
modified Bessel function).

Conventions (the paper is silent on them; each is one of the readings listed in the
design notes):
  * box side L = 1, periodic; positions in [0, 1);
  * mesh arrays are indexed [z][y][x]; particle arrays are [n][3] with columns x, y, z;
  * mesh node c sits at c * Delta, Delta = 1 / n_mesh; cloud-in-cell (CIC) weights are
    node-centred;
  * forward DFT unnormalised with exp(-2 pi i n.c / n), inverse with 1/n^3;
  * Poisson kernel with Plummer softening eps = soft_cells * Delta, zero at k = 0;
  * gradient factor -i D(k_a), the fourth-order central-difference symbol (zero on
    the Nyquist index).

Parity status of each function is stated in its module docstring.
"""

from . import adjoint, codec, mesh, pp, split, step  # noqa: F401
