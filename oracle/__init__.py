"""CPU oracle for hierarchical transformer preconditioning (arxiv 2605.13343).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only tests, the package smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the HIP library.

Everything here is a plain, slow, float64 implementation that follows the
paper's statement of each step, so that a reader can check it by eye:

  grid.py       Morton order, 7-point multiphase assembly, node/global features
  partition.py  weak-admissibility H-matrix partition and packed-factor layout
  network.py    encoder, diagonal and off-diagonal attention stacks, highways,
                decoder heads (PyTorch CPU float64; autograd supplies gradients)
  hmatrix.py    leaf Gram, explicit dense M, the FMM-style apply chain
  pcg.py        preconditioned conjugate gradients (identity, Jacobi, learned M)
  loss.py       spectrally smoothed probes, cosine-Hutchinson loss, AdamW

Parity status of each function is stated in its docstring.  Parts pinned only
by internal invariants (the network forward) say "parity unpinned" against
the paper, because the paper prints no weights or activations.
"""
