"""CPU oracle for the AIMx operator -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct NumPy/SciPy implementation (float64 /
complex128) of what the GPU library computes, written from the paper
"AIMx: An Extended Adaptive Integral Method for the Fast Electromagnetic
Modeling of Complex Structures" (Sharma & Triverio, arXiv 2009.02281):

* ``green``      -- the Helmholtz kernel and its static/dynamic split
                    (Sec. III, eqs. hgf, hgfs, hgfd, hgftaylor) and the
                    interpolation-error bound of Sec. IV-A (eq. Lbounds).
* ``mesh``       -- triangle areas and the 3-point quadrature rule.
* ``potential``  -- closed-form integral of 1/R over a flat triangle (the
                    "direct integration" of the static near field).
* ``aimx``       -- grid, stencils, projection P, interpolation W = P^T,
                    Toeplitz kernel H with the modified self term (eq. Hmm),
                    static near field and precorrection (eq. LAIMx).
* ``dense``      -- a dense direct-quadrature matvec of the same operator.
* ``solver``     -- restarted (F)GMRES and iterative refinement.
* ``mie``        -- the scalar single-layer series on a sphere.
* ``excitation`` -- plane-wave and Gaussian-patch right-hand sides.
* ``unet``       -- plain NumPy reference of the learned preconditioner.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never calls it and
shares no code with it.
"""
