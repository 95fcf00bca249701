// FP64 Cholesky factorisation and SPD solve for the ALS normal equations
// (W F^T = M^T, Section "Optimizing the CP-PPL tensor-network": W is the
// Hadamard product of the other factors' Grams and is solved by Cholesky).
#pragma once

#include "common.h"

namespace cpppl {

constexpr int CHOL_NB = 64;

// Lower Cholesky of the R x R row-major SPD matrix A.  The strictly-lower
// off-diagonal blocks of L overwrite those of A; the factored 64 x 64 diagonal
// blocks (padded with the identity) go to Dsave (diag_save_elems(R) doubles).
// A pivot that is <= 0 or not finite sets status[0] = 1 and is replaced by 1
// so that the factorisation stays finite.
void cholesky(double* A, int64_t R, double* Dsave, int* status, hipStream_t s);
int64_t diag_save_elems(int64_t R);

// X (R x n, row-major) <- (L L^T)^{-1} X for the factor left by cholesky().
void spd_solve(const double* A, const double* Dsave, int64_t R, double* X, int64_t n,
               hipStream_t s);

// A_ii += delta * trace(A) / R.
void add_ridge(double* A, int64_t R, double delta, hipStream_t s);

}  // namespace cpppl
