"""FP64 CPU oracle of the online PARAFAC subspace-tracking step (single coil).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke check of
``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may import or
call anything in this package.  The GPU library never does, and this package
imports nothing from the GPU library; the two share no code.

What it follows (Mardani, Giannakis, Ugurbil, "Tracking Tensor Subspaces with
Informative Random Sampling for Real-Time MR Imaging", arXiv 1609.04104):

* ``dft``      -- the orthonormal, symmetric DFT matrices F_l, F_r of Sec. IV
                  (2-D DFT written F(X) = F_l X F_r).
* ``tsl``      -- Algorithm 3 (tomographic MRI) with one coil and an all-ones
                  sensitivity map: the S1 ridge step of Sec. III-A, the residual,
                  the back-projection Theta = F^{-1}(Xi) of Sec. IV-B, the
                  majorization-minimization step size of Sec. III-A (eq. 6) and the
                  parallel factor updates of Algorithm 3; the output frame is
                  A[t] diag(gamma_t) B[t]^T as in Sec. IV-A.  A second, independent
                  formulation runs Algorithm 2 (k-space interpolation) on the
                  transformed factors.  ``epochs`` runs the batch mode of
                  Sec. VI-D: passes over stored frames, state carried over.
                  ``CoilOracle`` is Algorithm 3 with C coils and sensitivity
                  maps (Sec. IV-B), line masks.
* ``sampler``  -- Algorithm 4 (random subsampling): whole rows with the
                  row-marginal score of Sec. VI-C, and single entries with the
                  score of eq. 13; draws with replacement.
* ``philox``   -- the Philox4x64-10 counter-based generator (Salmon, Moraes,
                  Dror, Shaw, SC'11), which supplies the sampler's uniforms.

Everything is float64 / complex128 and written for readability, not speed.
Readings taken where the paper is silent or garbled are listed in the module
docstrings next to the code that takes them.
"""

from .dft import dft_matrix, fft2_unitary, ifft2_unitary
from .tsl import (TslOracle, KspaceOracle, regression_matrix, ridge_gamma,
                  ridge_gamma_svd, back_projection, step_alpha, gershgorin,
                  instantaneous_cost, gram_pivot_ratio, epochs, CoilOracle,
                  coil_regression_matrix, coil_gain)
from .sampler import (line_scores, line_weights_prefix, draw_lines, uniform_draws,
                      point_scores, expected_count, point_weights_prefix, point_draw_probabilities,
                      draw_points)
from .philox import philox4x64_10

__all__ = [
    "dft_matrix", "fft2_unitary", "ifft2_unitary", "TslOracle", "KspaceOracle",
    "regression_matrix", "ridge_gamma", "ridge_gamma_svd", "back_projection",
    "step_alpha", "gershgorin", "instantaneous_cost", "gram_pivot_ratio", "epochs", "CoilOracle",
    "coil_regression_matrix", "coil_gain", "line_scores",
    "line_weights_prefix", "draw_lines", "uniform_draws", "point_scores",
    "expected_count", "point_weights_prefix", "point_draw_probabilities", "draw_points",
    "philox4x64_10",
]
