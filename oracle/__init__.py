"""CPU FP64 oracle for Wannier-to-Bloch interpolation of e-ph matrix elements.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the library never does.
It shares no code with the HIP path: it is plain NumPy complex128 with LAPACK
``eigh``, written to be checked against the paper by eye.

Conventions (readings of the paper; every one is listed in the design notes):

* k, q are fractional (reciprocal-lattice units) and R integer lattice
  vectors, so the phase factor of Eq. (7) is exp(+2 pi i k.R).
* H(k) = sum_R w_R exp(2 pi i k.R) H(R) and its eigenvectors V(k) (columns)
  give the gauge of Eq. (5) as U(k) = V(k)^dagger.  With that, the band
  factors of Eq. (7) become V(k+q)^dagger g V(k).
* D(q) = sum_R w_R exp(2 pi i q.R) C(R) / sqrt(M_kappa M_kappa'); the mode
  vector of Eq. (2) is u_{kappa alpha, nu}(q) = e_{kappa alpha, nu} / sqrt(M_kappa),
  omega = sqrt(|lambda|).
* WS weights w_R multiply each phase (all 1 in the stock workloads).

Parity status: every function here is pinned by the CPU tests (closed forms,
invariants, the coarse-grid round trip, brute force); none is "parity unpinned".
"""
from .core import (  # noqa: F401
    phases, hamiltonian_k, bands, dynamical_q, phonons, mode_vectors,
    g_re_q, wannier_gauge_pairs, interpolate, interpolate_single_loop,
    coarse_transform, degenerate_blocks, block_sums, band_sums,
    splitmix64_weights, element_index, weighted_loss, compare_block_sums,
    bose, fermi, gauss, linewidth,
)
