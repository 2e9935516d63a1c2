"""CPU oracle for the stencil-as-structured-sparse-product path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, links or
calls this package; only the tests, the smoke check and the benchmark's CPU
baseline do.  It shares no code with the planner or the HIP kernels.

Contents
--------
direct      plain FP64 stencil stepper (C, OpenMP), the definition of the
            result (paper Section 2.2 and its commented Box-2D9P pseudo-code)
bruteforce  explicit operator matrix of one sweep on tiny grids, plus an exact
            rational-arithmetic stepper
fpformat    exact round-to-nearest-even into binary16 / bfloat16
tables      plan-time tables re-derived from the paper step by step: layout
            morphing (Section 3.1), hierarchical two-level matching
            (Section 3.2, Algorithm 1), 2:4 grouping and compression, hi/lo
            split, gather table, layout-exploration model (Section 3.3,
            Eqs. 6-11), temporal-fusion composition
matchers    exhaustive pair-matching and exact 2:4-grouping solvers used as
            independent validators of Algorithm 1 on small shapes
"""
