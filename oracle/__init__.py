"""CPU FP64 oracle for the mixed-basis (2D plane waves x B-splines) problem and its
1D-periodic form (plane waves along one axis x B-splines along the other two).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package; the library's compute
path never does.  It shares no code with the HIP library: its B-splines,
quadrature, G sets, matrix elements and solver are written here from the
paper's definitions with numpy / scipy primitives.

Modules
-------
bspline   : knot sequence, Cox-de Boor recursion (eqs. 1-2), derivative (eq. 3),
            Gauss-Legendre rule per interval, 1D overlap / derivative matrices
            (Sec. II.A and the overlap / kinetic elements of Sec. II.B.1).
lattice   : reciprocal vectors, in-plane G sets, k-points (basis of Sec. II.B.1).
operators : dense S, T, local potential (grid-consistent and analytic forms),
            Kleinman-Bylander projectors (Sec. II.B.1), H assembly.
solve     : lowest eigenpairs of H c = eps S c by LAPACK (generalized form of
            Sec. II.B.2), residuals.
rows      : selected rows of H x and S x without a dense matrix (same
            definitions, evaluated one output at a time) for large cells.
matfree   : matrix-free H x and S x (local part by a dense per-plane sum or
            through the grid with library FFTs) and the lowest eigenpairs by a
            library block eigensolver, for cells too large for dense assembly.
density   : electron density on the Gauss planes and the Hartree potential in
            the (z, g) form (Sec. II.B.1), by explicit sums.
wire      : the 1D-periodic form (end of Sec. II.B.2): dense S and H, matrix-free
            and row-wise H x, projector factors F(G) X(i) Z(j).

Parity status: every function is pinned by the CPU tests: bspline, lattice and
operators against closed forms, brute-force quadrature, library routines and
mathematical invariants (tests/test_oracle_bspline.py, test_oracle_operators.py,
test_oracle_physics.py); rows and matfree against the dense matrices of
operators, and matfree's eigensolver against LAPACK (test_oracle_operators.py,
test_oracle_matfree.py); density against closed forms and invariants
(test_oracle_density.py); wire against separable spectra, closed forms, direct
quadrature and its own dense matrices (test_oracle_wire.py).  None is "parity unpinned".
"""
