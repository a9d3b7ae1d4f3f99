"""Plain FP64 CPU oracle for the vertical-extrapolation multigrid PCG.

Test infrastructure only: the test-suite, the smoke check and the CPU
baseline leg of the benchmark call into this package; the GPU library never
does.  It is written for clarity, in the order and notation of the paper
(Kramer, Cotter & Pain, "Solving the Poisson equation on small aspect ratio
domains using unstructured meshes"), with NumPy/SciPy as the only helpers.

Modules
-------
fem       P1 assembly of the stiffness and mass matrices, boundary handling
          (Section 3, eqs. Ax=b, phi_decomposition, equation_decomposition).
ordering  node ordering (top block first), greedy colouring.
extrap    vertical extrapolation operator E~ (Section 5.4).
amg       smoothed aggregation hierarchy and V-cycle (Sections 5.1, 6).
precond   the preconditioners of Section 6 (VL + additive smoother, VL + SOR,
          Jacobi) and eq. ourpreconditioner.
pcg       preconditioned conjugate gradients.
solver    end-to-end setup + solve in the device node order.

Every public function cites the passage it follows.  Functions whose result
no independent pin checks say "parity unpinned" in their docstring.
"""
