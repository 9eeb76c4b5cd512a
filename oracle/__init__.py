"""CPU FP64 oracle for Subspace-Orbit Randomized SVD (Kaloorazi & de Lamare).

This package is TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it. The product path
(``paper_1804_00462_amd``) never imports, links or executes anything here, and
this package imports nothing from the product path: the two share no code.

Contents
  philox   Philox4x64-10 counter-based generator (Salmon et al., SC'11).
  normal   Gaussian draws from Philox words by Box-Muller, with log/sin/cos
           written out from +, -, *, / and sqrt only (bitwise reproducible).
  sorsvd   The method itself: Alg. 3 (basic SOR-SVD) and Alg. 4 (power
           method), eqs. (T1), (AT1), (M), the truncated core SVD and the lift.
  bounds   Eckart-Young floor (Th. 1), Th. 4 / Th. 5 deterministic bounds,
           Th. 6 / Th. 7 expectation bounds.
  mlp      FP64 reference of the (k, q) predictor network (forward, backward,
           Adam) used to check the GPU training kernels.
  rpca     Robust PCA by the ALM-SOR-SVD iteration (Table III).

Every function is pinned by a ``-m "not gpu"`` test in ``tests/test_oracle_*.py``
against something other than itself (numpy's independent Philox, closed forms,
the paper's printed Eckart-Young floor, LAPACK on special cases, theorem bounds).
"""
