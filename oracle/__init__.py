"""Plain FP64 CPU oracle of the wide-band ADMM reconstruction.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import it.  The GPU library never calls,
links or imports anything here, and this package imports nothing from the GPU
package.
"""
from .muffin_oracle import (Params, Problem, State, soft, dct_nu, idct_nu,
                            run, admm_iteration, objective, residuals,
                            energy, jvp_run, mse_loss, mse_grad,
                            set_workers, solve_adaptive)
from .wavelets import (DIRAC, PAPER_DICTIONARY, Dictionary, daubechies_filter,
                       dwt2, idwt2, dwt_levels)
from .spectral import (DCT, CHEBYSHEV, SPECTRAL_DIRAC, SpectralDictionary, chebyshev_basis,
                       basis_matrix)
from .visibility import (VisProblem, vis_forward, vis_adjoint, toeplitz_kernel, toeplitz_apply, cg)

__all__ = ["Params", "Problem", "State", "soft", "dct_nu", "idct_nu", "run",
           "admm_iteration", "objective", "residuals", "energy", "jvp_run",
           "mse_loss", "mse_grad", "set_workers", "solve_adaptive", "DIRAC", "PAPER_DICTIONARY",
           "Dictionary", "daubechies_filter", "dwt2", "idwt2", "dwt_levels", "DCT", "CHEBYSHEV",
           "SPECTRAL_DIRAC", "SpectralDictionary", "chebyshev_basis", "basis_matrix", "VisProblem",
           "vis_forward", "vis_adjoint", "toeplitz_kernel", "toeplitz_apply", "cg"]
