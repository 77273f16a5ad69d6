"""Plain, slow, FP64 CPU oracle of the random-sampling multiscale method.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package; the product path never does.  It shares no code with the HIP path
(the seeded input generators in :mod:`synth` aside) and imports nothing from
it.

Modules (each function cites the passage of the paper it follows):

* :mod:`oracle.philox`      Philox4x32-10 counter-based generator and the
  Box-Muller normals that draw the random boundary data.
* :mod:`oracle.elliptic`    Q1 finite elements for -div(a grad u) = 0, buffered
  patches, random local solves (banded Cholesky), restriction, traces,
  least-squares gluing and reconstruction, brute-force global solve.
* :mod:`oracle.kinetic`     discrete-ordinates upwind scheme for the 1D slab
  kinetic equation with isotropic scattering, the same stages.
* :mod:`oracle.rangefinder` Householder QR + SVD truncation of the snapshots.

Parity status: every function is pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_*.py`` except the reduced-basis global accuracy, which
the paper prints no values for (parity unpinned: GPU-vs-oracle only).
"""
