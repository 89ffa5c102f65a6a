"""CPU oracle for Iterative Hessian Sketching with sparse embeddings
(Cormode and Dickens, "Iterative Hessian Sketch in Input Sparsity Time").

TEST INFRASTRUCTURE ONLY. This package is a plain, slow float64 numpy/scipy
statement of what the GPU library computes. It exists to check that library:
only the tests, the smoke entry point and the benchmark's CPU-baseline leg may
import it. It shares no code with the GPU path; both sides draw their inputs
from the separate `workloads` package.

Contents and the passages they follow:
  philox   Philox4x64-10 (the hash behind S; the paper leaves it open)
  sketch   CountSketch / SJLT (Sec. 2), streaming application to dense and
           CSR data (Sec. 2, "Time Complexity"), the adjoint S^T G, and the
           explicit S for brute force
  dense_sketch  the Gaussian and SRHT sketches the paper compares with
           (Sec. 2, "Sketching Results"): Box-Muller entries from Philox, the
           radix-2 Hadamard transform of zero-padded rows, uniform row sampling
  ihs      Gram (SA)^T SA and the gradient A^T (b - A x) (Sec. 1 after Eq.(2);
           App. A.1.1 "Iteration Time Costs"), the QP of Eq.(2) over R^d, the
           l1 ball and the l2 ball, the outer loop (Eq.(2), Thm 2.2), x_OPT of
           Eq.(1), the error of Def. A.1, the derivative of x_OPT, and the
           reduced-access variant of the conclusion (one fixed sketch as the
           preconditioner of conjugate gradients)

Pins (tests/test_oracle_*.py) tie each function to something other than
itself: numpy's Philox stream, a dense S built entry by entry, scipy's
Sylvester Hadamard matrix, the normal law of the Gaussian entries, integer-valued
data (exact in any order), Lemmas A.5-A.7, closed-form sketch variance,
math.fsum, hand-solved projections, KKT conditions, brute-force enumeration of
l1 faces, the exact IHS error recurrence, finite differences, finite
termination and the Chebyshev bound of conjugate gradients.

Parity unpinned: the inner iterates of the l1 and l2 QP solvers (only their
solutions are pinned, through KKT and brute force), and the float rounding
order inside the Gram and the gradient (bounded, not matched).
"""
from . import philox, sketch, dense_sketch, ihs  # noqa: F401
