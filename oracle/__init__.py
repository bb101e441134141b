"""CPU oracle for block-randomized stochastic tensor-ring decomposition.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this package: only the tests, the small check in the repository's
entry module and the CPU-baseline leg of the benchmark may use it.  It shares
no code with the HIP library; the two meet only at the seeded input
generators of ``tr_inputs``, which hold none of the method's arithmetic.

Plain FP64 numpy/scipy, written from the paper (Yu, Li, Zhou,
"Block-Randomized Stochastic Methods for Tensor Ring Decomposition"):

* ``philox``   — Philox4x64-10 and Lemire bounded integers (the paper fixes
                 no generator; these make draws reproducible);
* ``tr``       — Section 2 definitions: multi-index, unfoldings, subchain
                 product/tensor, slices-Hadamard product, objective, full
                 gradient (``eq:gradient``), Hessian block, RSE;
* ``sampling`` — Section 3.2 laws (uniform, leverage, Euclidean, optimal),
                 Algorithm SSDTP's draws, the mode pick;
* ``brsgd``    — Algorithm TR-BRSGD and the scaled variant of Section 3.3;
* ``entry``    — sampled-entry loss and its gradient for all cores;
* ``batched``  — many independent problems, each stepped as above.
"""
