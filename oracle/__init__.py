"""Plain FP64 CPU oracle for the source-extended elastic FWI hot path.

TEST INFRASTRUCTURE ONLY. Only the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything under ``oracle/``. The product
path (the HIP library and its Python binding) never imports, calls or links it, and the
oracle imports nothing from the product package: the two share no code.

Modules
-------
``elastic2d``   eq.(1)-(4), (6), (8) data term: 2D isotropic elastic velocity-stress
                propagation (forward, exact discrete transpose, per-shot gradient).
``elastic3d``   the same for 3D (9 fields).
``vti2d``       the 2D propagation, transpose and gradient in a VTI medium (Thomsen eps,
                delta = eps / 2) at fixed eps and density, as in the field example.
``regularizer`` eq.(8) regularization term with the operators W (eq.(11)), S_w (eq.(12))
                and S^T, written as dense per-point matrices.
``checkpoint``  the 16-bit checkpoint encodings (per-snapshot max-abs scaling).
``zoi``         the sources' zones of influence, eq.(10): weights b_s and sinkhole flags.
``receiver``    the field-like DAS sampling K_r of eq.(3): gauge-length mean, strain rate,
                resampling, its transpose and the per-shot gradient through it.
``bspline``     the cubic B-spline model parameterization (expansion and its transpose).
``precondition`` the comparison methods: approximate inverse pseudo-Hessian (velocity
                autocorrelation summed over shots, clipped, scaled), near-offset mute; the
                gradient preconditioning of eq.(15) is ``regularizer.final_model``.

Every function is FP64 and unblocked; arrays are NumPy. Where the paper is silent
(discretization, absorbing boundary, source injection, DAS sampling details) the reading
taken is stated in the docstring of the function that implements it.
"""
