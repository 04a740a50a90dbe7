"""FP64 CPU oracle for the Brand-update K-factor path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library, its Python
binding, the serving loop) imports, links or runs anything in this package;
only the tests, the smoke check and the benchmark's CPU-baseline leg do.  The
oracle shares no code with the HIP path: the only common module is the seeded
input generator, which holds none of the method's arithmetic.

Modules
-------
bprocess  Oracle-D: the dense definition.  Keeps the d x d B-process iterate
          (Section 3.2, the B-process equation) and the true exponentially
          averaged K-factor (Section 2.1 / the EA K-factor process), with a
          full symmetric eigendecomposition per step.
brand     Oracle-B: the structured FP64 algorithm the paper states
          (Algorithm 3, Symmetric Brand, driven as in Algorithm 4, B-KFAC),
          with a Householder thin QR and a dense eigh of the small core;
          and the re-orthonormalisation of a drifted representation.
precond   The regularised inverse applied on both sides of a layer gradient:
          dense Cholesky solves (definition), the low-rank spectral form of
          Algorithm 1 (its inverse-application lines), the factored form of
          Algorithm 8, and spectrum continuation (Section 3.5).
rsvd      B-R-KFAC (Algorithm 5): the dense EA factor and the randomized SVD
          (range finder with re-orthonormalised power iterations) whose
          rank-r result overwrites a factor's representation.
correct   B-KFAC-C (Algorithms 6 and 7): the light correction of a
          representation on randomly chosen modes against the EA factor.
metrics   Basis-invariant comparisons (reconstruction, eigenvalues,
          orthonormality, preconditioned-gradient error) and the error
          metrics of the paper's numerical study (Section 4.2).
"""
from .bprocess import DenseFactor, truncate_rank, sorted_eigh  # noqa: F401
from .brand import BrandFactor, symmetric_brand, reorthonormalize  # noqa: F401
from .precond import (precondition_dense, lowrank_inverse_apply, precondition_lowrank,  # noqa: F401
                      precondition_factored, spectrum_continuation)
from .rsvd import ea_update, range_basis, rsvd, rsvd_overwrite  # noqa: F401
from .correct import light_correction  # noqa: F401
from .metrics import (e_rec_dense, e_rec_lowrank, e_D, e_orth, e_S, e_S_proj,  # noqa: F401
                      regularised_inverse_lowrank, e_inverse, e_angle)
