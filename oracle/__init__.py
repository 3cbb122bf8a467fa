"""CPU FP64 oracle for sign(H_W) b -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP library
(paper_0910_1048_amd): its Wilson operator is a naive C routine with full
spin matrices and an independently derived adjoint (wilson_ref.c), and its
algorithms are plain numpy/scipy restatements of the paper:

  wilson    -- H_W(mu) = gamma5 D_W(mu), forward, adjoint, sampled sites, dense
  dense     -- sign(A) b by eigendecomposition, by Schur-Sylvester, Hermitian case;
               exact rational target g_s(cA) b
  rational  -- Neuberger coefficients, circle theorem, number of poles
  krylov    -- two-sided Lanczos sign, restarted FOM and GMRES rational, multishift
               BiCG, LR deflation, accuracy measure
  eigen     -- critical left/right eigenpairs for LR deflation (dense definition)
"""
from . import dense, eigen, krylov, rational, wilson  # noqa: F401
from .wilson import WilsonRef  # noqa: F401
