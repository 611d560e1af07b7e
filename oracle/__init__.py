"""CPU oracle for the spherical tree code -- TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 NumPy implementation of what the GPU library computes,
written from the paper (Chen & Jablonowski, "Fast Summation on the Sphere with
Applications to the Barotropic Vorticity Equation"):

* ``direct``   -- the midpoint-rule Biot-Savart sum of the discrete BVE system
                  (Sec. 2, the particle system for dx_i/dt), both denominators
                  1 - x.y and |x - y|^2 / 2 (Sec. 2, alternative kernel form).
* ``geometry`` -- icosahedral triangle tree, node circumcentres and radii,
                  exact point location (Sec. 3, grids and dual tree traversal).
* ``interp``   -- interpolation points and spherical Bernstein-Bezier basis
                  (Sec. 3, interpolation in triangles).
* ``tree``     -- the tree code: proxy weights, PP / PC / CP / CC interactions
                  and the dual tree traversal (Sec. 3).
* ``rk4``      -- classical RK4 on (x, zeta) (Sec. 2 and Sec. 4).
* ``forcing``  -- the vorticity forcing F_R of the polar-vortex collapse
                  experiment (Sec. 4.4) and the forced RK4 step.
* ``metrics``  -- the relative l2 errors E and E_N (Sec. 4).
* ``mlp``      -- FP64 forward/backward of the small interaction-gating MLP and
                  the calibration of its output biases.
* ``amr``      -- adaptive refinement and coarsening of the particle
                  triangulation (Appendix A; Gaussian vortex, Sec. 4.3).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The GPU library never calls it, and it imports
nothing from the GPU library: the two share only the seeded input generators
in ``synthetic``.
"""

from . import direct, geometry, interp, tree, rk4, metrics, forcing, amr  # noqa: F401
