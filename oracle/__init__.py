"""FP64 CPU oracle for variational PAT reconstruction (test infrastructure).

This package is a plain, slow reference implementation written from the paper
(Boink et al., "A Framework for Directional and Higher-Order Reconstruction in
Photoacoustic Tomography", arXiv:1707.02245). It exists only to check the HIP
library: tests, the smoke check and the CPU-baseline leg of the benchmark may
use it; the library itself never does, and the two share no code.

Everything is NumPy/SciPy in float64. Operators are explicit sparse matrices
built from their definitions (Sec. 3.3.1 uses matrix versions of K, grad and
the symmetrised gradient, with the transpose as adjoint), and the solver takes
the steps of Algorithms 1 and 2 in the paper's order.

Modules:
  geometry  -- detector/time geometry and the circular-mean matrix A (eq. K_def)
  operators -- forward-difference gradient, symmetrised gradient, directional grad
  wavelet   -- the dual-tree wavelet transform W of the wavelet model (Sec. 2.2)
  prox      -- proximal maps of F1*, F2*, F3*, G (Sec. 3.2)
  pdhg      -- preconditioners (Sec. 3.3.2), PDHGM (Alg. 1, 2), gap (Sec. 3.3.3)
  metrics   -- PSNR (Sec. 5.4)
  pressure  -- calibrated forward model and preprocessing (Sec. 4.1, 4.2)
  unet      -- the warm-start network (forward, hand-written backward, Adam)
"""
from . import geometry, operators, prox, wavelet, pdhg, metrics, unet, pressure  # noqa: F401
