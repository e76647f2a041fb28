"""CPU oracle for the tiled QR factorization (Bouwmeester, Jacquelin, Langou,
Robert, "Tiled QR factorization algorithms", 2011).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
FP64 reference that the GPU library is checked against.  Only the test suite,
the smoke check and the CPU-baseline leg of the benchmark may import it; the
product library never does, and it shares no code with the HIP path.

Modules
-------
trees     elimination lists of every tree (Sec. 3.1, Sec. 3.2, Algorithm 4),
          validity conditions (Sec. 2.2) and the coarse-grain time-step model
          (Table 2).
dag       expansion of a list into kernel tasks (Algorithms 2 and 3) and the
          as-soon-as-possible schedule with the Table 1 weights (Sec. 2.3).
kernels   the six tile kernels as unblocked Householder code (Sec. 2.1).
tiled     the tiled driver, apply_q, least squares and iterative refinement.
brute     textbook unblocked Householder QR of the whole matrix.
mlp       FP64 two-hidden-layer MLP forward/backward/Adam for the makespan
          model of the tree/tile selector (no counterpart in the paper).

Parity status of every function is stated in its module header.
"""
