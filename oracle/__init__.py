"""Plain FP64 CPU oracle for the EnVar forward ensemble and its anomaly gradient.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it. It shares no code with the HIP library (its own geometry,
its own operators, a sparse direct Poisson solve instead of multigrid, a
two-pass cost instead of shifted running sums, an SVD least squares instead of
a Gram/Cholesky solve).

What it computes, and where the paper defines it:

* ``ns``      forced incompressible Navier-Stokes, eq. (forced_NS), in the
              semi-discrete form L dq/dt + N(q) = P f of eq. (discrete_NS),
              discretised on a uniform MAC grid with an explicit
              Adams-Bashforth-2 predictor and a Chorin projection.
* ``cost``    J(f) = observation term + penalty, eq. (Envarcost); the
              observation term is the time-integrated fluctuation energy of
              eq. (kinenergy) over the whole fluid domain.
* ``envar``   the N+1 forward evaluations of Sec. 3.3.1 (eq. fdapprox) and the
              least-squares reduction of {delta f_i, J_i} to a gradient in
              span of the perturbations (eq. gradient_EnVar, scalar-J form),
              plus the fixed-ensemble descent loop of Fig. (envar_loop).
* ``gn``      the vector-observation EnVar step: velocity sensors on the cavity
              lid (Sec. 4.1), fluctuation observations, Y by finite differences
              (eq. fdapprox), the Gauss-Newton Hessian and step (eq.
              Hessian_EnVar, eq. update_Newton) and the posterior variance
              (eq. posterior_covariance_matrix), and the EnVar loop over w with
              the Gauss-Newton or L-BFGS update (eq. update_Newton, update_BFGS).
* ``geometry`` also carries the paper's configuration (Sec. 2, Table
              tabgeometry, boundary conditions of Sec. 4.4): channel height
              1/2, uniform inflow, symmetry top, slip lower wall outside the
              no-slip segments next to the cavity.
* ``eigen``   the deterministic eigen-ensemble of Sec. 3.3.2: the tapered
              Gaussian covariance B of eq. (covarianceB) with the parameters of
              Sec. 4.2, its leading eigenpairs by a dense symmetric
              eigensolver, E = V_N mu_N^(1/2) sqrt(N - 1) (eq. eigenvm1), and the
              reconstruction error of App. A (eq. reconstruction_error).

Pins (tests/test_oracle_*.py): Taylor-Green linear AB2 recurrence and O(h^2)
nonlinear decay, energy conservation of the advection operator, the discrete
Poiseuille profile, divergence after projection, projection idempotence,
two-pass vs brute-force cost, closed-form gradients on quadratic costs,
central finite differences of the Navier-Stokes cost; for ``gn``: exact sensor
interpolation of linear fields, zero-mean fluctuations, a Gauss-Newton step
landing on the minimiser of an affine model (checked against an iterative
least-squares solver and central differences), the prior limit and
monotonicity of the posterior variance, the Gauss-Newton loop solving an
affine model in one step, the L-BFGS loop decreasing monotonically to the
same minimiser, and the two-loop recursion against the dense inverse-BFGS
update; for ``eigen``: the two-point closed form, the Kronecker spectrum of a
uniform-variance rectangle, E E^T / (N - 1) = B with every mode kept and the
Eckart-Young error when truncated, the taper's centre, corners and symmetry,
the separable product against the dense B, and the limits of the
reconstruction error; for the paper geometry: the viscous term of a uniform
stream on each kind of wall (0 on slip walls, -2 nu / h^2 on no-slip ones,
-nu / h^2 over the cavity) and a short forward that stays divergence-free with
the free stream kept at the symmetry top.
"""
