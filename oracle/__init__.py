"""Plain FP64 CPU oracle for the regularised tensor-equation solver.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports, calls or links
this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it, as the independent reference the
GPU path is checked against.  It shares no code with the GPU path (the only
common dependency is the seeded input generator package ``workload``, which
holds none of the solver's arithmetic).

Every routine is written from the paper (Morozov & Hunziker, "Solving Tensor
Structured Problems with Computational Tensor Algebra") in float64 NumPy, with
no blocking, fusion or reordering beyond what the cited definition states:

* ``tensor``  -- separable transformation as a chain of mode products
  (Sec. 2.1, eq. separable_transf) and the inner product (App. A.6).
* ``normal``  -- the regularised normal operator and right-hand side built from
  the transposition rule (App. A.7) and the Kronecker-sum form of Sec. 4.1.
* ``cg``      -- the tensor conjugate-gradient iteration of Fig. Tensor_CG.
* ``jacobi``  -- the main diagonal of the operator, the stationary tensor
  Jacobi iteration of Fig. Tensor_Jacobi and the diagonal preconditioner.
* ``multigrid`` -- the tensor multigrid V-cycle of Fig. TMG (separable
  restriction and prolongation, Jacobi smoothing, direct coarsest solve).
* ``dense``   -- the matrix-equivalent form of the tensor equation (Sec. 3),
  assembled column by column and solved by Cholesky (tiny sizes only).
* ``judge``   -- the FP64 relative residual used to judge any solution.
* ``wsnet``   -- the learned warm-start network (separable per-mode
  convolutions, Table 1) with forward, backward (App. A.8) and Adam.
* ``precond`` -- the tensor-inverse preconditioner (the separable part of the
  operator inverted mode by mode, Sec. 3) and preconditioned CG.
* ``scattered`` -- the scattered-measurement operator of the application
  (Sec. 6): Khatri-Rao rows (Sec. 2.2), normal operator as a CP sum.
"""
from .tensor import mode_product, multi_mode_product, inner
from .normal import (
    gram,
    reg_factor,
    forward,
    rhs,
    normal_apply,
    normal_apply_literal,
    regulariser_apply,
    NormalOperator,
)
from .cg import cg, CGResult, lanczos_extremes
from .dense import assemble, dense_solve
from .judge import relative_residual
from . import wsnet
from . import precond
from . import scattered
from . import jacobi
from . import multigrid

__all__ = [
    "mode_product", "multi_mode_product", "inner",
    "gram", "reg_factor", "forward", "rhs", "normal_apply",
    "normal_apply_literal", "regulariser_apply", "NormalOperator",
    "cg", "CGResult", "lanczos_extremes",
    "assemble", "dense_solve", "relative_residual", "wsnet", "precond", "scattered",
    "jacobi", "multigrid",
]
