// Host FP64 evaluation of sign(T) e_1 for a small complex tridiagonal T.
#pragma once

#include <complex>

namespace sgn {

struct SmallSignInfo {
    double min_abs_re = 0.0;     // min |Re lambda| over the eigenvalues of T
    double norm = 0.0;           // infinity norm of T
    double eigvec_growth = 0.0;  // largest 2-norm of a unit-diagonal eigenvector of the Schur factor
};

// T(i,i) = diag[i], T(i+1,i) = sub[i], T(i,i+1) = sup[i] (i < k-1).
// y (length k) receives sign(T) e_1.  Returns 0 on success, 1 bad size,
// 2 QR iteration did not converge, 3 an eigenvalue lies on the imaginary axis.
int small_sign_e1(int k, const std::complex<double> *diag, const std::complex<double> *sub,
                  const std::complex<double> *sup, std::complex<double> *y, SmallSignInfo *info);

// Eigenvalues and unit-norm right eigenvectors of a general complex n x n matrix
// a (row-major): Householder reduction to Hessenberg form, the complex Schur
// form by the same QR sweeps, eigenvectors of the triangular factor by back
// substitution.  vec (row-major n x n) receives the eigenvector of lam[i] in
// column i.  Returns 0, 1 for a bad size, 2 if the QR iteration did not converge.
int small_eig(int n, const std::complex<double> *a, std::complex<double> *lam, std::complex<double> *vec);

}  // namespace sgn
