"""FP64 CPU oracle for the complex Ginzburg--Landau exponential stepper.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy/SciPy implementation of what the GPU library computes, written from
the paper (Caliari & Cassini, "Efficient simulation of complex
Ginzburg--Landau equations using high-order exponential-type methods").
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the HIP library and never
imports it; the library never imports this package.

Contents (each function cites the passage it follows):

* ``operators``  -- 1-D finite-difference operators A_mu (eq. ODEs), their
  exponentials by the closed-form sine/cosine eigen-decomposition and by
  ``scipy.linalg.expm``.
* ``tensor``     -- mu-mode product, Tucker operator (eq. Tucker), Kronecker
  sum K (eq. ODEs) for brute-force checks, K u via eq. (kronsumv).
* ``nonlinear``  -- g(u) of eq. (cqCGL), the exact cubic and quintic flows
  (eq. exsolcub and its quintic analogue in Section 4.3), one classical RK4
  step of u' = g(u) (eq. RK4 with K = 0) as the cubic-quintic sub-flow.
* ``steppers``   -- Strang (eq. Strang), split4 (eq. Richardson), Lawson2b
  (eq. lawson2b), Lawson4 (eq. lawson4, six exponential actions per step)
  and the three-term splittings of Section 4.3 exactly as written, plus a
  time loop.
* ``fourier``    -- periodic boundaries by the Fourier pseudospectral route of
  Section 3.2 (exp(t K) as a pointwise product between transforms).
* ``metrics``    -- relative 2-norm / infinity-norm errors and the observed
  order of convergence used in the paper's tables.
* ``surrogate``  -- FP64 residual CNN forward/backward (3x3 convolutions).

All arithmetic is complex128 / float64 unless a function says otherwise.
"""
