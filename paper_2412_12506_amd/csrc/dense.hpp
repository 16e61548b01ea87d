// Dense FP64 linear algebra used by the host-side setup.
//
//  * ls_householder: least squares min ||C X - R||_F by Householder QR
//    (Section 2.3.3: each SAI block column is a small dense overdetermined
//    least-squares problem solved by QR).  Column-major storage, panel-blocked
//    with the compact WY form so that the trailing update is a matrix product.
//  * ls_block_normal: the same least-squares problem when C is block sparse
//    and well conditioned, by the normal equations C^T C X = C^T R formed
//    block by block (only the nonzero blocks of C enter), a tiled Cholesky
//    factorisation and one step of refinement from the residual R - C X
//    (Bjorck, Numerical Methods for Least Squares Problems, Sec. 2.9).  The
//    correction of the refinement step measures kappa(C)^2 u; when it is not
//    small the caller falls back to ls_householder.
//  * sym_eig: symmetric eigendecomposition by Householder tridiagonalisation
//    followed by implicit QL iterations with Wilkinson-type shifts (Golub & Van
//    Loan, Ch. 8); used for the cached block inverses of the Jacobi and
//    Gauss-Seidel smoothers (Section 2.3.1) and for the bottom pseudo-inverse
//    (Section 2.2, "Bottom solver").
#pragma once
#include <cstddef>
#include <utility>
#include <vector>

namespace ldgmg {

// C: m x n column-major (leading dim m), overwritten.  R: m x k column-major,
// overwritten.  On success X (n x k column-major) holds the solution and the
// function returns true; returns false when the triangular factor has a
// diagonal entry below 1e-13 * max |diag| (numerically rank deficient).
bool ls_householder(int m, int n, int k, double* C, double* R, double* X);

// Block-sparse C: mb x nb blocks of size bs x bs; rows[a] lists the nonzero
// blocks of block row a as (block column, pointer to the bs x bs block,
// row-major).  The right-hand side is the identity in block row `pos` and zero
// elsewhere.  On success X (nb*bs x bs, column-major as for ls_householder)
// holds the solution and the function returns true.  Returns false, leaving X
// undefined, when the Cholesky factorisation meets a pivot below
// 1e-24 * max diag(C^T C) or the refinement correction exceeds 1e-8 of the
// solution (max norms).
bool ls_block_normal(int bs, int mb, int nb,
                     const std::vector<std::vector<std::pair<int, const double*>>>& rows, int pos,
                     double* X);

// A: n x n symmetric, row-major (only read).  w: n eigenvalues (ascending),
// V: n x n row-major with eigenvectors in columns.  For n >= 256 the work is
// split over up to nthreads threads (results do not depend on the count).
void sym_eig(int n, const double* A, double* w, double* V, int nthreads = 1);

// out = pseudo-inverse of symmetric A (n x n, row-major) with eigenvalues
// |lambda| <= rel_tol * max|lambda| treated as zero.
void sym_pinv(int n, const double* A, double* out, double rel_tol, int nthreads = 1);

}  // namespace ldgmg
