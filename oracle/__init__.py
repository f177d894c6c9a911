"""FP64 CPU oracle for coefficients-learning OMP (CLOMP) and plain OMP.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the GPU path is checked against.  Only the test suite, the
package smoke check and the CPU-baseline leg of the benchmark may import it.
The product path (the HIP library and its Python binding) never imports,
links or calls anything here, and this package imports nothing from the
product path: the two share no code.  Inputs come from the seeded generators,
which hold none of the method's arithmetic.

All arithmetic is float64.  Arrays given as float32 or bfloat16 are upcast
exactly (both embed in float64), so "the instance" is always the stored values.

Conventions (paper: Methods, "Mathematic Model", Eq. (1)-(3)):
  A  -- measurement matrix, m x n, given as a numpy array of shape (m, n)
  y  -- measurements, length m
  s  -- sparse coefficients, length n (the paper's s; the C ABI calls it x)
  S  -- support: list of selected column indices in selection order
The residual is taken as r = y - A s.  Eq. (2) writes r = A s - y; only |A^T r|
enters the selection, so the sign is immaterial there, and every gradient here
is derived from the loss, not from r.

Modules
  omp        O1  plain OMP, least squares on the support by Householder QR
  clomp      O2  CLOMP: argmax selection + Adam steps on the masked coefficients
  clomp_paper  F1  paper-mode CLOMP: normalised-threshold multi-selection, one
                   Adam step per iteration, R iterations
  iht        F4  normalised iterative hard thresholding (comparison method)
  prior      F2  total-variation prior of Eq. (5) on x = D s (explicit DCT-II D)
  image_prior  F2  image priors of Eq. (6) (2-D total variation) and Eq. (7)
                   (local variation, 3 x 3 windows) and CLOMP on the columns of
                   one image with both
  brute      O3  exhaustive support search for tiny instances
  grad       O4  loss/gradient of 1/2||A(mask*s) - y||^2;  O5 one Adam step
  lstsq      O6  least squares on a support;  FP64 residual norm
  incremental    O1 with an updated QR (classical Gram-Schmidt twice) and O2
                 with the gradient in Gram form G_S s_S - b_S: the same
                 quantities at sizes the plain renderings cannot reach
  separation     "well-separated instance" test used to gate support identity,
                 and the separated prefix of a long support

Parity status
  O2's pre-refinement Adam iterate s_adam has no closed form: parity unpinned
  except through the independent autograd + torch.optim.Adam rendering in the
  test suite (same definition, independent implementation).
"""

from .lstsq import lstsq_support, resid_norm_fp64
from .grad import grad_fp64, adam_step_fp64
from .omp import omp_fp64
from .clomp import clomp_fp64, ClompParams
from .clomp_paper import clomp_paper_fp64, PaperParams
from .iht import iht_fp64
from .prior import dct_synthesis, forward_difference, tv_1d, tv_grad_coeffs, lstsq_support_tv
from .brute import bruteforce_support
from .separation import (well_separated, separation_report, separated_prefix, common_prefix,
                         perturbed_atoms, perturbed_vector)
from .incremental import omp_cgs2_fp64, clomp_gram_fp64
from .image_prior import (tv_2d, tv_2d_grad, lv, lv_grad, image_prior_loss, image_prior_grad,
                          clomp_image_fp64)

__all__ = [
    "lstsq_support", "resid_norm_fp64", "grad_fp64", "adam_step_fp64",
    "omp_fp64", "clomp_fp64", "ClompParams", "clomp_paper_fp64", "PaperParams", "iht_fp64",
    "dct_synthesis", "forward_difference", "tv_1d", "tv_grad_coeffs", "lstsq_support_tv",
    "bruteforce_support",
    "well_separated", "separation_report", "separated_prefix", "common_prefix",
    "perturbed_atoms", "perturbed_vector", "omp_cgs2_fp64", "clomp_gram_fp64",
    "tv_2d", "tv_2d_grad", "lv", "lv_grad", "image_prior_loss", "image_prior_grad",
    "clomp_image_fp64",
]
