"""CPU oracle for the integral-equation solver: TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 numpy/scipy implementation of what the GPU library computes,
written from the paper (Saputera et al., "3D induction log modelling with
integral equation method and domain decomposition preconditioning", GJI):

* ``green``    - Green's tensor of eqs. (5)-(7) and its method-of-moments
                 discretisation (section 2.2): midpoint rule off the diagonal,
                 equal-volume sphere integral on the diagonal;
* ``source``   - background fields of a point dipole in the homogeneous medium;
* ``operator`` - the FFT convolution of eq. (10) with 2x zero padding and the
                 operator (I - G dsigma) of eq. (8); the contraction form;
* ``dense``    - brute-force dense assembly of the same operator (no FFT);
* ``gmres``    - restarted GMRES (Saad & Schultz) with modified Gram-Schmidt,
                 and flexible GMRES (right preconditioner that may change);
* ``solve``    - full-domain solves and the relative residual of eq. (9);
* ``dd``       - Alg. 1: block Gauss-Seidel / Jacobi sweeps (eqs. 19-24)
                 with fixed or adaptive inner tolerance, and the Krylov outer
                 iteration over one sweep from zero;
* ``receivers``- magnetic field at receiver points (eqs. 4 and 6) by direct
                 summation over the cell currents;
* ``cnn``      - plain CPU reference of the learned-initial-guess network.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg
may import this package.  It shares no code with the HIP library, and the HIP
library never calls it.  Every input comes from the seeded generators in
``synth``.

Pins: every function here is checked in ``tests/test_oracle_*.py`` against
something other than itself (finite differences of eq. (5), numerical
quadrature of the self-cell sphere integral, dense brute force, dense LU,
closed-form limits, symmetries, App. A and App. C identities).  The only parts
without such a pin are iteration counts and timings (parity unpinned: the
paper's counts come from different hardware, models and formulation).
"""
