"""Reference oracle for the Hierarchical Subspace Iteration Method (HSIM).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 CPU
implementation of what the GPU library computes, written from the paper
(Nasikun & Hildebrandt, "The Hierarchical Subspace Iteration Method for
Laplace-Beltrami Eigenproblems").  Only the test-suite, the smoke check and
the benchmark's CPU-baseline leg may import it; the library never does, and
the two share no code (only the seeded mesh generators in ``synth`` feed
both).

Modules
-------
assembly   cotangent stiffness S and lumped mass M (Section 3.1, eq. massStiffMatrices)
jacobi     cyclic Jacobi for the dense (generalized) symmetric eigenproblem
sim        the Subspace Iteration Method (Algorithm 1) and the convergence
           test (eq. conv2); one-iteration reference steps
hierarchy  vertex hierarchy by farthest point sampling (Algorithm 3),
           prolongation operators (eq. radius, eq. basis), Galerkin operators
           (Algorithm 2) and the level-size / subspace-size / shift rules
hsim       the Hierarchical Subspace Iteration Method (Algorithm 2)
metrics    eigenpair error measures (relative residual, cluster-aware
           eigenvector error)
gradient   eigenvalue / eigenvector derivatives with respect to vertex
           positions (dense reference)

Every function names the passage of the paper it follows.  Where the paper is
silent or garbled the reading taken is stated in the docstring.
"""
