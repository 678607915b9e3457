"""CPU oracle for the collision hot path and the dynamical low-rank step.

TEST INFRASTRUCTURE ONLY.  Plain, slow, float64 implementations written from
the paper (Hu & Wang, "An adaptive dynamical low rank method for the nonlinear
Boltzmann equation") and from the mathematical definition of the Fourier-
Galerkin collision operator.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import anything from here; the
library in ``paper_2112_02695_amd`` never does, and this package imports
nothing from it.

Modules
-------
quadrature  radial Gauss-Legendre, circle and Lebedev-38 sphere rules
collision   the discrete collision operator: its definition as a direct
            spectral sum, the FFT form of the same operator, moments and the
            conservation projection
dlr         the fully discrete K-S-L low-rank step (Sec. 2.4), boundary
            ghost values (Sec. 2.3), error pieces (Sec. 5.1), basis add/drop
            (Sec. 3) and the steady-state driver
shock       the Mott-Smith shock quantities of Sec. 4 (alpha, beta, the
            logistic density profile)
carleman    the Carleman-form fast spectral operator (2D Maxwell molecules,
            3D hard spheres): its definition as a weighted direct sum and the
            fast form with filtered transforms
"""
