// Dense FP64 linear algebra used by the host-side setup.
//
//  * ls_householder: least squares min ||C X - R||_F by Householder QR
//    (Section 2.3.3: each SAI block column is a small dense overdetermined
//    least-squares problem solved by QR).  Column-major storage, panel-blocked
//    with the compact WY form so that the trailing update is a matrix product.
//  * sym_eig: symmetric eigendecomposition by Householder tridiagonalisation
//    followed by implicit QL iterations with Wilkinson-type shifts (Golub & Van
//    Loan, Ch. 8); used for the cached block inverses of the Jacobi and
//    Gauss-Seidel smoothers (Section 2.3.1) and for the bottom pseudo-inverse
//    (Section 2.2, "Bottom solver").
#pragma once
#include <vector>
#include <cstddef>

namespace ldgmg {

// C: m x n column-major (leading dim m), overwritten.  R: m x k column-major,
// overwritten.  On success X (n x k column-major) holds the solution and the
// function returns true; returns false when the triangular factor has a
// diagonal entry below 1e-13 * max |diag| (numerically rank deficient).
bool ls_householder(int m, int n, int k, double* C, double* R, double* X);

// A: n x n symmetric, row-major (only read).  w: n eigenvalues (ascending),
// V: n x n row-major with eigenvectors in columns.
void sym_eig(int n, const double* A, double* w, double* V);

// out = pseudo-inverse of symmetric A (n x n, row-major) with eigenvalues
// |lambda| <= rel_tol * max|lambda| treated as zero.
void sym_pinv(int n, const double* A, double* out, double rel_tol);

}  // namespace ldgmg
