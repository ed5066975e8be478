"""Plain FP64 CPU oracle for the low-rank (Burer-Monteiro) SDP method.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct reference
that the GPU library is checked against.  It may be imported only by ``tests/``,
by ``__graft_entry__.smoke()`` and by the CPU-baseline leg of ``bench.py``; the
product path never imports, links or executes anything here, and nothing here
imports the product package.  The only code shared with the GPU side is the
seeded input generator module ``synth`` (which holds none of the method's
arithmetic).

Everything is float64 numpy / scipy with library primitives (sparse matrix
products, ``numpy.roots``, dense and Lanczos eigensolvers) used as single steps.
There is no blocking, fusion or reordering beyond what each definition states.

Sign convention.  The paper's appendix (exact line search) writes the augmented
Lagrangian as  <C,X> + lam^T (b - A(X)) + rho/2 ||b - A(X)||^2  and its error
measures use C - A*(lam) and <C,X> - lam^T b; the oracle uses that convention
throughout and calls the multiplier ``y`` and the penalty ``sigma``.  The form in
the introduction (eq. for the BM augmented Lagrangian, multiplier update
lam <- lam + rho (A(RR^T) - b)) is the same method with lam replaced by -y.

Modules
-------
problem   problem data: C, the stacked constraint matrix over nonzero columns, b
kernels   the per-iteration quantities: (C - A*(y))V, A(UV^T), gradient,
          Lagrangian, exact line-search coefficients and step, ALM measures
lbfgs     the L-BFGS direction (two-loop recursion, H0 = I)
alm       the Burer-Monteiro ALM solve and the splitting (ADMM) phase
certify   dual certificates (minimum eigenvalue), brute-force max cut
mlp       the warm-start MLP (forward, backward, Adam) in float64
"""
