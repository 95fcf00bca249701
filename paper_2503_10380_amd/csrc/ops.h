// Element-wise, layout and reduction kernels of the CP-PPL sweep (host launchers).
//
// Factor storage: every factor is kept transposed, FT[r][n] (R x n, row-major),
// so a factor is directly the k-contiguous A operand of the GEMMs, a column of
// the paper's factor matrix is a contiguous row here, and W F^T = M^T is a
// left-side solve.
#pragma once

#include "common.h"
#include "gemm.h"

namespace cpppl {

// y[b][c][r] = x[b][r][c], with conversion to `yt`.
void transpose_batched(const double* x, void* y, DType yt, int64_t batch, int64_t rows,
                       int64_t cols, hipStream_t s);
// Same for an FP64 output with an FP64 input that may live anywhere (alias-free).
// out[p][X][q] = b[X][p][q] (rows of length v move), with conversion.
void permute_pxq(const double* b, void* out, DType ot, int64_t nx, int64_t v, hipStream_t s);
// y[i] = convert(x[i]).
void convert(const double* x, void* y, DType yt, int64_t n, hipStream_t s);
// y[i] += x[i] (FP64).
void axpy1(const double* x, double* y, int64_t n, hipStream_t s);
// Kt[r][i*o + j] = gT[r][i] * rT[r][j] (* ij_scale[i*o + j], * r_scale[r] when given),
// converted to `kt`.
void khatri_rao_t(const double* gT, const double* rT, int64_t o, int64_t R, void* Kt, DType kt,
                  hipStream_t s, const float* ij_scale = nullptr, const double* r_scale = nullptr);
// x[i][j][a][b] <- (x[i][j][a][b] + x[j][i][b][a]) / 2 in place (o x o x v x v, FP64).
void symmetrize_pairs(double* x, int64_t o, int64_t v, hipStream_t s);
// OCP e4m3 copies with power-of-two scales:
// scale[r] = least 2^e (e in [-126, 127]) with max_k |x[r][k]| <= 448 * 2^e, rows x len row-major;
void e4m3_row_scales(const double* x, int64_t rows, int64_t len, float* scale, hipStream_t s);
// q[i] = e4m3(x[i] / scale[((i / div) % mod) / grp]), round to nearest even, saturating;
void quantize_e4m3(const double* x, uint8_t* q, int64_t n, const float* scale, int64_t div,
                   int64_t mod, int64_t grp, hipStream_t s);
// out[X*v + q] = scale[X].
void expand_scales(const float* scale, float* out, int64_t nx, int64_t v, hipStream_t s);
// dt[ijab] = (w[ijab] + scale (cp[ijab] + cp[jiba]) / 2) / (e_occ[i] + e_occ[j] - e_vir[a]
// - e_vir[b]) - t[ijab]: one Jacobi step of D t = w + scale R(t) with the pair-symmetrised
// CP tensor for R, as a change of t (o x o x v x v, FP64; dt may alias w).
void jacobi_delta(const double* cp, const double* w, const double* e_occ, const double* e_vir,
                  double scale, const double* t, double* dt, int64_t o, int64_t v, hipStream_t s);
// tau[i][j][c][d] = t2[i][j][c][d] + t1[i][c] t1[j][d] (t1 is o x v), FP64.
void dress_tau(const double* t2, const double* t1, double* tau, int64_t o, int64_t v, hipStream_t s);
// w = g1 .* g2 .* g3 (n elements); g3 may be null.
void hadamard(const double* g1, const double* g2, const double* g3, double* w, int64_t n,
              hipStream_t s);
// lam[r] = ||FT[r][:]||_2, FT[r][:] /= lam[r] (rows with zero norm are left as they are).
void row_normalize(double* FT, int64_t R, int64_t n, double* lam, hipStream_t s);
// FT[r] = alpha * sum_s part[s][r] (split order), then row_normalize, then (if
// lowp) the BF16 copy: one launch for the split-K reduction, the
// normalisation and the conversion that follow the factor solve, with the same
// arithmetic in the same order as those three steps.
void finish_factor(const double* part, int splits, int64_t R, int64_t n, double alpha, double* FT,
                   double* lam, void* lowp, hipStream_t s);
// Occupied-mode reductions of HT[r][i*o + j]:
//   which = 0: M[r][i] = sum_j HT[r][i*o+j] * other[r][j]   (gamma update)
//   which = 1: M[r][j] = sum_i HT[r][i*o+j] * other[r][i]   (rho update)
void occ_reduce(const double* HT, const double* other, double* M, int64_t o, int64_t R, int which,
                hipStream_t s);
// Fit scalars after a sweep, written to sc[]:
//   sc[0] = <R, CP> = sum_r lam_r sum_n MT[r][n] FT[r][n]
//   sc[1] = ||CP||^2 = lam^T (G0 .* G1 .* G2 .* G3) lam
//   sc[2] = residual^2 = max(norm_r2 - 2 sc[0] + sc[1], 0), sc[3] = fit, sc[4] = loss
// `rowbuf` holds 2R doubles of scratch; norm_r2 is read from device memory.
void fit_scalars(const double* MT, const double* FT, int64_t n, const double* lam,
                 const double* const G[4], int64_t R, const double* norm_r2, double* rowbuf,
                 double* sc, hipStream_t s);
// dst[q][0:n[q]] = src[q][0:n[q]] for q < count (1..5), one launch.
void copy_doubles(const double* const* src, double* const* dst, const int64_t* n, int count,
                  hipStream_t s);
// out = lamA^T (X0 .* X1 .* X2 .* X3) lamB for R x R cross products (eta terms).
void weighted_hadamard_sum(const double* const X[4], const double* lamA, const double* lamB,
                           int64_t R, double* rowbuf, double* out, hipStream_t s);
// E = sum_r lam_r sum_ab aT[r][a] tau[r][a][b] bT[r][b]; tau in `tt`.
void energy_from_tau(const void* tau, DType tt, const double* aT, const double* bT,
                     const double* lam, int64_t R, int64_t v, double* rowbuf, double* out,
                     hipStream_t s);
// acc[0] += sum x^2, acc[1] += sum x y over a rows x cols block with row
// strides ldx, ldy (deterministic two-pass; `partial` holds 2*1024 doubles).
void sumsq_dot_accumulate(const double* x, const double* y, int64_t rows, int64_t cols,
                          int64_t ldx, int64_t ldy, double* partial, double* acc, hipStream_t s);
// Scalar helpers on device memory.
void set_scalar(double* p, double v, hipStream_t s);
// eta = sqrt(max(nn - 2 np + pp, 0)) / sqrt(pp), from sc_eta[0..2] = (nn, np, pp).
void finish_eta(double* sc_eta, hipStream_t s);
// Count non-finite entries of x into *flag (flag must be zeroed by the caller).
void nonfinite_check(const double* x, int64_t n, int* flag, hipStream_t s);
// FT[r][i] (R x n) = uniform [-1, 1) number offset + i R + r of a counter-based
// SplitMix64 stream seeded with `seed` (Steele, Lea and Flood, OOPSLA 2014).
void random_factor(double* FT, int64_t n, int64_t R, uint64_t seed, uint64_t offset, hipStream_t s);
// p[i] = v for i < n.
void fill_doubles(double* p, int64_t n, double v, hipStream_t s);
// Zero n ints / doubles with a kernel (graph-capture safe).
void zero_ints(int* p, int64_t n, hipStream_t s);
void zero_doubles(double* p, int64_t n, hipStream_t s);
// Scale the columns of C (R x P, row-major) by lam[p] and multiply in X1 .* X2 (R x P each).
void hadamard_scale_cols(const double* X0, const double* X1, const double* X2, const double* lamP,
                         double* C, int64_t R, int64_t P, hipStream_t s);
// Sign-aligned difference: y[r][n] = sign(<F1[r],F0[r]>) * F1[r][n] - F0[r][n], as float,
// written with row stride ldy.  Used for the warm-start network targets.
void aligned_delta_f32(const double* F1, const double* F0, int64_t R, int64_t n, float* y,
                       int64_t ldy, hipStream_t s);
// y[r][off + n] = (float) x[r][n] * (scale ? scale[r] : 1)
void pack_rows_f32(const double* x, const double* scale_inv, int64_t R, int64_t n, float* y,
                   int64_t ldy, int64_t off, hipStream_t s);
// x[r][n] += (double) y[r][off + n]
void add_rows_from_f32(const float* y, int64_t ldy, int64_t off, int64_t R, int64_t n, double* x,
                       hipStream_t s);

}  // namespace cpppl
