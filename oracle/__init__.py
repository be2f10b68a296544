"""FP64 CPU oracle for the ADMM reconstruction of convolutional inverse problems.

TEST INFRASTRUCTURE ONLY. Nothing in the library's product path may import,
call or execute anything in this package: only the test suite, the smoke check
and the CPU-baseline leg of the benchmark use it. It shares no code with the
GPU library (kernels, headers, tables, helpers); the only thing both consume is
the seeded input generator module.

Source: Dogan & Oktem, "Efficient Algorithms for Convolutional Inverse
Problems in Multidimensional Imaging" (arXiv 2006.08303). Each function cites
the section / equation it implements. The oracle is deliberately plain and slow:
spatial-domain circular convolution for the forward model, explicit transform
matrices, a dense Cholesky solve of the normal equations for small problems,
and the step order of Algorithms 1 and 2 in the paper's notation.

Modules:
  model     forward model y_k = sum_s h_{k,s} * x_s (Eq. forward model), its
            adjoint, dense block matrix H for tiny grids (Eq. forwardModel).
  priors    analysis operators T (2D/3D DCT, wavelet x DCT, anisotropic TV
            2D/3D), isotropic TV per slice and coupled along the slices
            (Chambolle's algorithm), soft thresholding (Eq. solt_trans),
            patch extraction P_j (Eq. patch_based), convolutional dictionary
            synthesis (Eq. conv_dic).
  xupdate   x-update solvers: dense normal equations (Eq. solx_Trans /
            solx_synt), per-frequency S x S solves (Eq. solx_Trans_DFT /
            solx_synt_DFT), recursive 2x2 block inversion (Eq. recinv).
  admm      Algorithm 1 (analysis) and Algorithm 2 (synthesis: patch and
            convolutional dictionaries), objectives and KKT residuals.
"""
from . import model, priors, xupdate, admm  # noqa: F401
