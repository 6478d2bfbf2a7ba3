"""CPU FP64 oracle for the tensor-product three-body eigensolver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls into this
package: only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark import it.  It is a plain, slow, obviously correct NumPy/SciPy
restatement of what the method computes, written from the paper
(Thies, Hof, Zimmermann, Efremov, "Tensor Product Scheme for Computing Bound
States of the Quantum Mechanical Three-Body Problem"):

* ``cheb``      - Chebyshev-Gauss-Lobatto collocation second-derivative matrices
                  with Dirichlet conditions (Sec. 3.1, eq. (7)), Clenshaw-Curtis
                  weights for the symmetry check.
* ``physics``   - Jacobi-coordinate kinetic coefficients (Sec. 2, eq. (2)) and
                  the pair potential V = u(|y - x/2|) + u(|y + x/2|) (eq. (3)).
* ``operator``  - the Hamiltonian applied in tensor form (eqs. (9)-(11)) and as
                  an explicit Kronecker matrix (eqs. (7), (8)).
* ``twobody``   - heavy-light two-body problem (eq. (1)): ground energy (the
                  preconditioner shift) and the depth v0 for a binding energy.
* ``precond``   - kinetic-only shifted Sylvester preconditioner solved by
                  Bartels-Stewart (Sec. 4.2, eq. (14)).
* ``orth``      - block orthogonalisation.
* ``jdqr``      - block Jacobi-Davidson QR with preconditioned GMRES on the
                  correction equation (Sec. 4.1, eqs. (12)-(13)).
* ``dense``     - dense eigenvalues of the explicit matrix (brute force).

Every function computes in FP64 unless stated otherwise.  Where the paper is
silent the reading taken is stated in the function's docstring.
"""
