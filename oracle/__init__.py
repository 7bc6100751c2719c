"""CPU oracle for the ADMM / reduced-KKT PCG hot path — TEST INFRASTRUCTURE ONLY.

Plain, slow, float64 NumPy/SciPy code that states what the method computes,
written from the paper ("GPU Acceleration of ADMM for Large-Scale Quadratic
Programming", Schubiger, Banjac, Lygeros) in its order and notation:

* ``formats``   — COO / CSR / CSC and the upper-triangle → full expansion (Section 5.3, 6.2)
* ``spmv``      — the definition y_i = Σ_j a_ij x_j with extended-precision accumulation
* ``ruiz``      — modified Ruiz equilibration (Algorithm 2, Section 3.3)
* ``kkt``       — objective, residuals, optimality conditions (Section 2.1, eq. opt_cond) and the duality gap
* ``pcg``       — the reduced-KKT operator, its Jacobi diagonal (Section 6.3.1) and PCG (Algorithm 3)
* ``admm``      — OSQP's ADMM (Algorithm 1) with the direct solve of the full KKT system (eq. kkt)
* ``activeset`` — brute-force active-set enumeration for tiny QPs (independent check of the optimum)
* ``hutchinson``— diagonal-of-inverse estimates from Rademacher probes

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import anything here. The product path (the HIP library and its
binding) never does, and shares no code with this package.
"""
