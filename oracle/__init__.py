"""Plain, slow, obviously-correct CPU FP64 oracle for the DG-AMR hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
product path (the HIP library and its Python binding) never imports, calls or
links it, and shares no code with it.

Paper: Abdi, Almgren, Giraldo, Jankov, "Comparison of adaptive mesh refinement
techniques for numerical weather prediction" (arXiv 2404.16648).

Modules
  refelem  -- 1-D reference-element operators (section 3.3: LGL integration,
              L2 projections built from the mass and mixed mass matrices).
  forest   -- oct-tree forest, 2:1 balance, face and transfer tables
              (section 3.1 forest of trees; section 4.3 2:1 balance).
  euler    -- compressible Euler in hydrostatic-perturbation form (section 2.1),
              strong-form dGSEM with Rusanov flux (section 2.2), mortars
              (section 3.3), SSP-RK3 stage, budgets, indicator, transfers,
              adjoint and JVP by automatic differentiation of the same code.

Every function is pinned by a ``-m "not gpu"`` test in ``tests/`` against a
closed form, an invariant, a special case or brute force; the few results
with no such pin say "parity unpinned" in their docstring.
"""
