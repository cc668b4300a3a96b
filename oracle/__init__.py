"""Plain FP64 CPU oracle for the MPT reduced-order hot path.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test-suite, the smoke check in
__graft_entry__.py and the CPU baseline leg of the benchmark may
import or call anything here.  It shares no code with the GPU library and does
not import it.

Every function follows the paper's definitions directly (Section 3 eq. (NRI),
(Rmatrixmeth), (I_tensor_coeffs); Section 4 eqs. (D), (SVD), (truncSVD),
(ReducedA), (podprealmpt), (podpimagmpt); Lemma 4.1 and Algorithm 1) with
library primitives (LAPACK SVD / solve, SuperLU) as steps and no blocking,
fusion or reordering beyond what those definitions state.  Tensors are taken by
explicit sums over grid faces and conductor edges (the analogue of the paper's
integral method), which the matrix method must reproduce up to rounding.

Parity-unpinned items are named in the docstring of the function concerned.
"""
