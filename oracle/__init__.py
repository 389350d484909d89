"""CPU FP64 oracle for domain decomposition of entropic unbalanced OT.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the bench's
CPU-baseline leg may import this package; the product path never does.

The oracle is plain, dense and slow on purpose: every cell problem is solved
with explicit cost matrices and library log-sum-exp, with no separable
factorisation, no re-centring and no fusion, so that each step can be checked
against the paper by eye.  It shares no code with the HIP library.

Modules
  uot   the global problem: primal, dual, KL, dense Sinkhorn, the cell
        Y-update root (Sec. 2.2 and Sec. 4.1)
  dd    partitions, basic-cell marginal state, cell subproblems, the parallel
        (Algorithm 4) and sequential (Algorithm 3) iterations, GetWeights,
        tracked score, primal-dual certificate (Sec. 3 and Sec. 4)
  grad  gradients of the optimal value by the envelope theorem

Parity status of each function is stated in its docstring; functions with no
independent pin say "parity unpinned".
"""
