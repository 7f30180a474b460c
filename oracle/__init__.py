"""FP64 CPU oracle of the spectral-element Poisson solver (test infrastructure).

This package is the independent, deliberately plain reference that the GPU
library is checked against.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the library never does, and the two
share no code.  Every function follows the paper (Remacle, Gandham, Warburton,
"GPU accelerated spectral finite elements on all-hex meshes") step by step:

* :mod:`oracle.gll`        -- GLL points, weights, derivative matrix (Section 2.1)
* :mod:`oracle.numbering`  -- local/global node tables, gather/scatter (Section 2.2)
* :mod:`oracle.geometry`   -- Jacobian, metric factors, lumped mass (Sections 2.3-2.4)
* :mod:`oracle.operator`   -- matrix-free stiffness action, eq. (R) / eq. (ABC)
* :mod:`oracle.brute`      -- dense element matrices from full 3D basis gradients (pin only)
* :mod:`oracle.schwarz`    -- overlapping patches and fast-diagonalisation solves (Section 4.2, eq. (z))
* :mod:`oracle.coarse`     -- order-1 coarse space, restriction and prolongation (Section 4.1, eq. (coarse))
* :mod:`oracle.pcg`        -- preconditioned conjugate gradients (Algorithm 1)

Parity status per function is listed in each module header.
"""
