"""FP64 CPU oracle for direct volume rendering of LR-spline volumes.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
restatement of what the rendering method computes, used to check the GPU
library.  Only the test suite, the smoke check and the benchmark's CPU-baseline
leg may import it; the product path never calls it and shares no code with it
(the two meet only in the seeded inputs made by ``lrgen``).

Modules
  bspline  Cox-de Boor evaluation of the LR B-splines (Eq. 1, Eq. 2)
  lookup   element search by linear scan (Sec. 3.2, the O(N) search)
  bezier   Bezier blocks by interpolation (Sec. 3.2.3), Bernstein evaluation, and
           the adjoint of the (linear) change of basis
  camera   ray generation and sample positions replayed in IEEE FP32
  render   transfer function, sampling schedules (fixed, Eq. 4 adaptive, fine
           fixed) and front-to-back compositing (Alg. 2, Eq. 3)
  grad     reverse-mode derivative of the Bezier-parameterised render and
           central finite differences
  streamline  explicit Runge-Kutta streamlines with the Eq. 4 heuristic step,
           constant or embedded error-controlled steps, and the error metric
           Eq. 7 against a small-step RKF5 reference (Sec. 5)

Pins (tests/test_oracle_*.py) tie every function to something other than
itself: partition of unity, polynomial reproduction through refinement,
scipy's NdBSpline on tensor meshes, the closed form 1-exp(-sigma L) for a
constant field, the textbook "over" operator, brute force on tiny inputs,
colorsys, and finite differences.
"""
