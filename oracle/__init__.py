"""Plain FP64 CPU oracle for recycling BiCG (RBiCG).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and the
CPU-baseline leg of the benchmark may import this package.  The product path
(the HIP library and its Python binding) never calls it, and the two share no
code: the oracle is written directly from the paper (Ahuja, de Sturler,
Gugercin, Chang, "Recycling BiCG with an Application to Model Reduction").

Modules
  krylov   -- BiCG (Algorithm 1) and RBiCG (Algorithm 2) with the cycle-wise
              recycle-space update of Sec. 4 (plain explicit products).
  recycle  -- T from the iteration scalars (Sec. 4.1), harmonic Ritz pencils
              (eq. finalGenEigValue and its dual mirror), eigenvalue selection,
              SVD biorthogonalization (Sec. 4.3, eqs. equationSVD/equationForUC).
  drivers  -- sequences of dual systems, shifted pairs (sigma I - A) sharing one
              recycle space, FP32-inner / FP64-outer refinement, bilinear forms.
  rng      -- SplitMix64 counter generator used when x~ must be re-seeded.
  irka     -- IRKA (Algorithm 3, E = I or general E) with direct solves, and
              transfer functions of the full and reduced models.
  precond  -- split ILU(0) preconditioning in red-black ordering and
              sequences of split-preconditioned RBiCG solves.

Pinned against: dense direct solves, CG and SciPy's BiCG iterates (textbook
special cases), exact-eigenvector deflation, biorthogonality, the T-from-scalars
identity, harmonic-Ritz exactness on invariant subspaces, published SplitMix64
outputs.  Results without such a pin are marked "parity unpinned" where they
are defined.
"""
from .krylov import bicg, rbicg, SolveResult, as_csr
from .recycle import (t_from_scalars, harmonic_pencils, select_eigvecs,
                      biorthogonalize, first_cycle_eigvecs)
from .drivers import (rbicg_sequence, shifted_pairs, mixed_refine, bilinear)
from . import precond
from .rng import splitmix64, reseed_vector
from . import irka

__all__ = ["bicg", "rbicg", "SolveResult", "as_csr", "t_from_scalars",
           "harmonic_pencils", "select_eigvecs", "biorthogonalize",
           "first_cycle_eigvecs", "rbicg_sequence", "shifted_pairs",
           "mixed_refine", "bilinear", "splitmix64", "reseed_vector"]
