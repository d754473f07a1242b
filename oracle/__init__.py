"""CPU FP64 oracle for the HiKF hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check of the package entry point and the CPU
baseline leg of the benchmark may import anything from here.  The product
path (the HIP library and its Python binding) never calls into this package,
and this package never imports the product package; the two share only the
seeded input generators in ``synth``.

Contents, each a plain NumPy/SciPy restatement of what the paper defines:

* ``kernels``     covariance kernels K(r) (Sec. 3.3 list; Sec. 4.2 eq.
                  ``equation_Q``) and a test-only polynomial kernel.
* ``kf_dense``    tier A: the conventional random-walk Kalman filter,
                  Sec. 2.2 eqs. ``KF_forecast``..``eqn_KF_Pa`` (Algorithm
                  ``algorithm_Kalman``).
* ``kf_crosscov`` tier B: the cross-covariance filter of Algorithm
                  ``Algorithm_HiKF`` / Sec. 3.1 eqs. ``eqn_kalmangin_new``,
                  ``eqn_KF_forecast_new``, ``eqn_KF_pred_new``.
* ``cq_exact``    tier C: the exact product C_Q = Q H^T (Sec. 3.2) by three
                  independent routes (dense, FFT circulant embedding, direct
                  sums on chosen rows).
* ``bbfmm``       FP64 black-box FMM with Chebyshev interpolation, the
                  approximation Sec. 3.2 uses for Q H^T (Fong & Darve 2009,
                  cited there); reference for the GPU's H^2 error split.
* ``enkf``        the perturbed-observation ensemble Kalman filter of
                  Sec. 2.3 (eqs. ``equation_samplemean``,
                  ``equation_samplecov1``, ``equation_samplegain_enkf``) on the
                  random-walk model, with the draws passed in.
* ``truth``       random-walk truths with covariance Q (Sec. 2.1 eq.
                  ``equation_random_walk``) for building test streams.

Parity status: every function above is pinned by a test in
``tests/test_oracle_*.py`` except where its docstring says
"parity unpinned".
"""
