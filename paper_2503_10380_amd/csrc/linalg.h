// FP64 inverse of the ALS normal-equation matrix W (Section "Optimizing the
// CP-PPL tensor-network": W is the Hadamard product of the other factors'
// Grams; the update is F = M W^{-1}).
//
// W is inverted by the block sweep (Gauss-Jordan) operator: sweeping every
// 64 x 64 pivot block of a symmetric positive-definite matrix once turns it
// into -W^{-1}.  Each block step is one launch of one work-group per output
// tile; two buffers alternate so no launch reads what it writes, and the
// inverse of the next pivot block is formed one launch ahead by the group
// that computes that block.  The factor update is then one GEMM,
// F^T = W^{-1} M^T, and the inversion only needs the Grams, so it can run
// before the MTTKRP it is applied to is ready.
#pragma once

#include "common.h"

namespace cpppl {

constexpr int INV_NB = 64;

// Doubles of the pivot-inverse buffer that spd_inverse_neg needs.
constexpr int64_t INV_DBUF = 2 * INV_NB * INV_NB;

// -W^{-1} of the R x R row-major SPD matrix in bufA (overwritten), using bufB
// as the second buffer and dbuf (INV_DBUF doubles) for the pivot inverses;
// returns the buffer holding the result.  A pivot that is <= 0 or not finite
// sets status[0] = 1 and is replaced by 1 so that the result stays finite.
double* spd_inverse_neg(double* bufA, double* bufB, double* dbuf, int64_t R, int* status,
                        hipStream_t s);

// A_ii += delta * trace(A) / R.
void add_ridge(double* A, int64_t R, double delta, hipStream_t s);

}  // namespace cpppl
