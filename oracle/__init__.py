"""FP64 CPU oracle for the cell-centred finite-volume step and Poisson solve.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product library
never calls it, and it shares no code with the GPU path (it reads the same
raw mesh and input fields from the ``synth`` input generator, nothing else).

It is a plain, slow, readable NumPy/SciPy transcription of the method of
Kissami & Ratnani, "Manapy: MPI-based framework for solving PDEs using
finite volume on unstructured grids" (arXiv 2203.00925):

* ``geometry``  - cell/face/ghost/node geometry, node-neighbour stencils,
                  least-squares node weights, diamond coefficients (Sec. 2.1);
* ``fv``        - the residual of eq. (4): least-squares cell gradient
                  (Algorithm 1), Barth-Jespersen limited MUSCL upwind flux
                  (eq. (15)), node interpolation (Algorithm 2), diamond
                  diffusive flux (eq. (diamond)), and the 3-stage Runge-Kutta
                  update (eq. (6));
* ``poisson``   - the matrix of eqs. (7)/(laplace), the matrix-free operator it
                  comes from, Jacobi-preconditioned CG and a direct-solve pin
                  (Sec. 2.2 and Sec. 3.4);
* ``local``     - the same residual and matrix rows evaluated for a sample of
                  cells from their neighbourhood only, for checks on meshes
                  too large for the global oracle.

Readings of points the paper leaves open (ghost centres, limiter formula,
the garbled Runge-Kutta line, the CFL rule, ...) are stated where they are
used.  Every function is pinned by a CPU test against something other than
itself: closed forms, linear exactness, brute-force least squares, a direct
solve, conservation, or the paper's annex example.
"""
