/*
 * cpppl.h -- C ABI of the MI355X (gfx950) library for the matrix-free CP
 * decomposition of the CCSD particle-particle-ladder (PPL) tensor.
 *
 * What is computed (K. Pierce, "Towards Using Matrix-Free Tensor
 * Decompositions to Systematically Improve Approximate Tensor-Networks"):
 *   R_ijab = sum_cd (sum_X B^X_ac B^X_bd) t_ijcd        (eq. dfB, no singles)
 * is fitted by a rank-R CP model
 *   CP_ijab = sum_r lambda_r gamma_ir rho_jr alpha_ar beta_br   (eq. cp-ppl)
 * with alternating least squares (Section "Optimizing the CP-PPL
 * tensor-network", eq. full_der and the W Gram-Hadamard product; the paper
 * solves the normal equations by Cholesky, this library by an explicit FP64
 * inverse of W from the block sweep (Gauss-Jordan) operator, applied as one
 * GEMM).  R is never formed: each factor's MTTKRP is a chain of contractions
 * of t and B against the other three factors (eq. distribute, eq. foreachr).
 *
 * Conventions for every call:
 *  - Every call returns a cpppl_status; no C++ exception crosses this ABI.
 *  - Arrays are row-major, FP64 unless stated.  `on_device` = 0: host pointer;
 *    non-zero: device pointer on the context's device, ordered on its stream.
 *  - The caller owns every buffer it passes; inputs are copied into the
 *    context's workspace before the call returns.
 *  - Calls that return host values synchronise the context's stream; the
 *    others only enqueue work.
 *  - One host thread per context; several contexts may coexist.
 *  - After CPPPL_E_HIP the context must be destroyed; other errors leave it usable.
 *  - cpppl_last_error() gives a message for the last failing call on a context.
 */
#ifndef CPPPL_H
#define CPPPL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CPPPL_API __attribute__((visibility("default")))

typedef struct cpppl_ctx cpppl_ctx; /* opaque, library-owned */
typedef struct cpppl_mlp cpppl_mlp; /* opaque, library-owned */

typedef enum {
  CPPPL_OK = 0,
  CPPPL_E_ARG = -1,         /* bad argument (null pointer, size, mode) */
  CPPPL_E_STATE = -2,       /* call out of order (e.g. ALS before inputs) */
  CPPPL_E_HIP = -3,         /* HIP runtime error; context must be destroyed */
  CPPPL_E_NOMEM = -4,       /* bound workspace too small / host allocation failed */
  CPPPL_E_NOT_SPD = -5,     /* normal-equation matrix W not SPD (a pivot of its block sweep
                               inverse <= 0 or not finite) after ridge retries */
  CPPPL_E_NONFINITE = -6,   /* NaN or Inf in inputs or results */
  CPPPL_E_UNSUPPORTED = -7  /* operation not available in this configuration */
} cpppl_status;

/* Operand precision of the MTTKRP contractions.  Grams, W, its inverse and the solve,
 * the factor masters, the fit and the energy are FP64 in all of them, and the
 * FP64 masters of t and B are kept for the FP64 refinement sweeps. */
typedef enum {
  CPPPL_FP64 = 0,    /* FP64 operands, FP64 accumulation */
  CPPPL_BF16 = 1,    /* bfloat16 operands (t, B, factors, intermediates), FP32 accumulation */
  CPPPL_FP8_E4M3 = 2 /* ablation: t and B stored as OCP e4m3 (largest value 448, round to
                        nearest even) times a power-of-two scale per (ij) row of t and per
                        X slice of B, the least one that keeps the row or slice in range;
                        dequantised exactly to bfloat16 inside the GEMMs; factors and
                        intermediates bfloat16, FP32 accumulation.  Needs v % 8 == 0. */
} cpppl_precision;

typedef struct {
  int64_t o;    /* occupied orbitals (i, j) */
  int64_t v;    /* virtual orbitals (a, b, c, d) */
  int64_t nx;   /* density-fitting auxiliary functions X */
  int64_t rank; /* CP rank R, 1 <= R <= 4096 */
  int64_t singles; /* non-zero: reserve room for the singles-dressed operands
                      (cpppl_load_singles); 0: doubles only */
} cpppl_dims;

typedef struct {
  int max_sweeps;        /* number of ALS sweeps (upper bound when a stop rule is set) */
  int stop_rule;         /* 0: none; 1: |fit_n - fit_{n-1}| < tol (eq. canon);
                            2: eta < tol (eq. N3_stopping);
                            3: |E_n - E_{n-1}| < tol, E = E_CP after each sweep (the energy
                               contraction below; with stop_window w, |E_n - E_{n-w}| / w) */
  double tol;
  int refine_fp64_sweeps;/* BF16 contexts: FP64 sweeps appended after the BF16 ones */
  int history_cap;       /* entries available in the report's history arrays */
  int energy;            /* non-zero: compute E_CP = sum R~ t after the last sweep */
  int timing;            /* non-zero: time kernel classes with HIP events */
  double refine_tol;     /* > 0: the FP64 refinement stops once |fit_n - fit_{n-1}| < refine_tol,
                            the first refinement sweep compared with the last BF16 one (at
                            most refine_fp64_sweeps sweeps); 0: run them all */
  int stop_window;       /* stop rule 1 on the main sweeps: compare |fit_n - fit_{n-w}| / w with
                            tol, w = stop_window (1..64; 0 means 1), to average out the
                            evaluation noise of BF16 fits */
  int eta;               /* non-zero: evaluate eta (eq. N3_stopping) after every sweep (implied
                            by stop_rule 2); otherwise the report's eta values are NaN */
  int near_cache;        /* non-zero: keep the last six iterates; when the call runs n > 5
                            sweeps, the (n-5)th becomes the near-optimal cache used by
                            CPPPL_WS_NEAR_OPTIMAL (otherwise the previous cache stays) */
  int energy_every;      /* non-zero: evaluate E_CP = sum CP t after every sweep (into the
                            report's energy_hist; implied by stop_rule 3).  In the sweep
                            dtype: FP64 sweeps give it in FP64, BF16 / FP8 sweeps from a
                            bfloat16 tau.  tau' = KR(gamma, rho)^T t of the updated factors
                            is what the next sweep starts from, so it is formed once and
                            reused: the cost is O(R v^2) per sweep, not an extra product. */
  double refine_etol;    /* > 0: the FP64 refinement stops once |E_n - E_{n-1}| < refine_etol
                            between two FP64 refinement sweeps (E_CP in FP64, at least two
                            refinement sweeps).  With refine_tol also set, both must hold. */
} cpppl_als_opts;

/* Kernel classes timed when opts.timing is set (index into ms_class / n_class). */
enum {
  CPPPL_T_KR_T2 = 0,   /* tau = KR(gamma, rho)^T t   (S2) */
  CPPPL_T_Y = 1,       /* Y = F^T B                  (S3 / S7 / S8) */
  CPPPL_T_Z = 2,       /* per-r Y tau                (S4 / S7) */
  CPPPL_T_M = 3,       /* M = B . Z, split-K         (S5 / S7) */
  CPPPL_T_G = 4,       /* per-r G = Y_a^T Y_b        (S8) */
  CPPPL_T_H = 5,       /* H = t . G, split-K         (S9) */
  CPPPL_T_SOLVE = 6,   /* occupied reductions of H, Grams, solve F = M W^-1, normalise */
  CPPPL_T_FIT = 7,     /* fit, eta, energy scalars (S11, S12) */
  CPPPL_T_INV = 8,     /* W and its inverse (side stream for alpha, beta, gamma: overlapped) */
  CPPPL_T_COUNT = 16
};

typedef struct {
  int sweeps_done;       /* sweeps run in this call (including refinement) */
  int ridge_retries;     /* retries of the W inverse with a ridge shift W + delta tr(W)/R I
                            after a failed pivot (delta = 1e-14 * 100^k, k = 0..4) */
  double fit;            /* 1 - ||R - CP|| / ||R||  (eq. cpfit) after the last sweep */
  double loss;           /* 0.5 ||R - CP||^2 (eq. loss_function) */
  double inner;          /* <R, CP> */
  double cp_norm2;       /* ||CP||^2 (eq. cp_norm2) */
  double eta;            /* ||CP_n - CP_{n-1}|| / ||CP_{n-1}|| of the last sweep */
  double energy_cp;      /* sum_ijab CP_ijab t_ijab if opts.energy, else NaN */
  double ms_total;       /* wall time of the sweeps (host clock, stream synchronised) */
  double ms_class[16];   /* summed kernel-class times (opts.timing) */
  int n_class[16];       /* kernel launches per class (opts.timing) */
  double* fit_hist;      /* caller-owned, history_cap entries, or NULL */
  double* eta_hist;      /* caller-owned, history_cap entries, or NULL */
  double* ms_hist;       /* caller-owned, per-sweep milliseconds, or NULL */
  int refine_done;       /* of sweeps_done, the FP64 refinement sweeps */
  double* energy_hist;   /* caller-owned, history_cap entries, or NULL: E_CP after each sweep
                            where it was evaluated (opts.energy_every, stop_rule 3, refine_etol),
                            else NaN */
  int careful_sweeps;    /* sweeps redone synchronously from their snapshot after a failed
                            pivot of a W inverse (each then retries with ridge shifts) */
} cpppl_als_report;

/* ---- lifecycle ----------------------------------------------------------- */

/* Create a context for `dims` and operand precision `prec` on HIP device
 * `device`, enqueuing on `hip_stream` (a hipStream_t; NULL = default stream).
 * The context needs a device workspace before any other call (bind_workspace).
 * E_ARG for bad dims, an unknown precision, or FP8 with v % 8 != 0. */
CPPPL_API cpppl_status cpppl_create(const cpppl_dims* dims, cpppl_precision prec, int device,
                                    void* hip_stream, cpppl_ctx** out);
/* Bytes of device workspace a context with these dims and precision needs. */
CPPPL_API cpppl_status cpppl_workspace_size(const cpppl_dims* dims, cpppl_precision prec,
                                            size_t* bytes);
/* Give the context `bytes` of device memory at `dev_ptr` (256-byte aligned),
 * owned by the caller and kept alive until cpppl_destroy. E_NOMEM if too small. */
CPPPL_API cpppl_status cpppl_bind_workspace(cpppl_ctx* ctx, void* dev_ptr, size_t bytes);
CPPPL_API cpppl_status cpppl_destroy(cpppl_ctx* ctx);

/* ---- inputs --------------------------------------------------------------- */

/* Doubles amplitudes t[i][j][a][b] (o, o, v, v) (tau of eq. B with t1 = 0). */
CPPPL_API cpppl_status cpppl_load_t2(cpppl_ctx* ctx, const double* t, int on_device);
/* Virtual-virtual DF block b[X][p][q] (nx, v, v) = D^{pX}_q of eq. SQG.  No
 * symmetry in (p, q) is assumed. */
CPPPL_API cpppl_status cpppl_load_df(cpppl_ctx* ctx, const double* b, int on_device);
/* Replace R by an explicit CP tensor sum_p lam_p fi_ip fj_jp fa_ap fb_bp with
 * rank_p <= rank columns (fi, fj: o x rank_p; fa, fb: v x rank_p; lam: rank_p
 * or NULL for ones).  MTTKRPs then use the Gram identity; no energy. */
CPPPL_API cpppl_status cpppl_load_planted(cpppl_ctx* ctx, const double* fi, const double* fj,
                                          const double* fa, const double* fb, const double* lam,
                                          int64_t rank_p, int on_device);
/* ||R||^2 and E_exact = sum R t, in FP64 (computed once per loaded t and B;
 * R is streamed in blocks, never stored whole).  energy_exact may be NULL. */
CPPPL_API cpppl_status cpppl_norm_r2(cpppl_ctx* ctx, double* norm_r2, double* energy_exact);

/* ---- factors: (i, j, a, b) = (gamma o x R, rho o x R, alpha v x R, beta v x R) ---- */

/* lam may be NULL (ones).  Factors need not be normalised. */
CPPPL_API cpppl_status cpppl_set_factors(cpppl_ctx* ctx, const double* fi, const double* fj,
                                         const double* fa, const double* fb, const double* lam,
                                         int on_device);
/* The paper's random guess (Section "An improved initial guess strategy":
 * factors drawn uniformly from [-1, 1]) on the device: element (row, r) of factor m, in the
 * API order (i, j, a, b) = (gamma, rho, alpha, beta), is
 * u(offset_m + row * R + r) with offset_m the element count of the factors
 * before m, where u(c) = 2^-52 (z >> 11) - 1 and z is output number c + 1 of
 * SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) seeded with `seed`; lambda = 1.
 * Reproducible from the seed alone; synchronises. */
CPPPL_API cpppl_status cpppl_init_random(cpppl_ctx* ctx, uint64_t seed);
/* Any output pointer may be NULL. */
CPPPL_API cpppl_status cpppl_get_factors(cpppl_ctx* ctx, double* fi, double* fj, double* fa,
                                         double* fb, double* lam, int on_device);

/* ---- work ---------------------------------------------------------------------- */

/* Singles (T1) dressing of the PPL tensor (Section "The Density Fitting
 * approximation": eq. B, eq. fulldfB and the Dbar intermediate of eq. dfB).
 * t1 is o x v row-major with t1[i][a] = t^a_i; b_vo is X x v x o row-major with
 * b_vo[X][a][k] = D^{aX}_k, the virtual-occupied block of the DF tensor.  The
 * context then contracts tau_ijcd = t_ijcd + t1[i][c] t1[j][d] in place of t
 * and Dbar^X_bd = D^X_bd - 2 sum_k D^X_bk t1[k][d] on the b side (alpha keeps
 * D):  R_ijab = sum_cd (sum_X D^X_ac Dbar^X_bd) tau_ijcd.  The dressing stays
 * with the context: later cpppl_load_t2 / cpppl_load_df calls are dressed with
 * the same t1, and cpppl_warm_start's dt is added to the doubles part.  ||R||^2
 * and E_exact become those of the dressed tensor, and E_CP = sum CP tau.
 * t1 == NULL removes the dressing (b_vo is then ignored).  Needs dims.singles
 * != 0 (E_UNSUPPORTED otherwise) and t2 and the DF tensor loaded (E_STATE);
 * not available for planted tensors.  on_device: pointers are device memory. */
CPPPL_API cpppl_status cpppl_load_singles(cpppl_ctx* ctx, const double* t1, const double* b_vo,
                                          int on_device);

/* Run ALS sweeps (order alpha, beta, gamma, rho) from the current factors. */
CPPPL_API cpppl_status cpppl_als(cpppl_ctx* ctx, const cpppl_als_opts* opts,
                                 cpppl_als_report* report);
/* The MTTKRP of one mode (0 i, 1 j, 2 a, 3 b) at the current factors, in
 * precision `prec` (FP64, or the context's own precision; anything else is
 * E_UNSUPPORTED): m_out is n_mode x R (the
 * numerator of eq. full_der for that factor, without lambda). */
CPPPL_API cpppl_status cpppl_mttkrp(cpppl_ctx* ctx, int mode, cpppl_precision prec, double* m_out,
                                    int on_device);
/* fit, <R, CP> and ||CP||^2 at the current factors (one FP64 MTTKRP). */
CPPPL_API cpppl_status cpppl_fit(cpppl_ctx* ctx, double* fit, double* inner, double* cp_norm2);
/* The CP tensor at the current factors, CP_ijab = sum_r lambda_r gamma_ir rho_jr
 * alpha_ar beta_br (eq. cp-ppl), formed explicitly in FP64 as one o^2 x v^2 x R
 * GEMM of two Khatri-Rao products, into out (o x o x v x v row-major, o^2 v^2
 * doubles, caller-owned; device memory if on_device, else host).  symmetrize
 * != 0 then replaces it by (CP_ijab + CP_jiba) / 2, the pair symmetry the ALS
 * does not enforce (Section "The CPD approximation of the PPL tensor-network",
 * the reconstruction for the rest of the CCSD iteration).  Synchronises; drops
 * the cached Y_beta. */
CPPPL_API cpppl_status cpppl_reconstruct(cpppl_ctx* ctx, double* out, int symmetrize, int on_device);
/* One step of a CCD-like Jacobi iteration driven by the CP-approximated ladder
 * (Section "Role of the Initial Guess"; the reconstruction and pair
 * symmetrisation of Section "The CPD approximation of the PPL tensor-network"):
 * with the CP tensor at the current factors, formed in FP64 as in
 * cpppl_reconstruct and pair-symmetrised, R~_ijab = (CP_ijab + CP_jiba) / 2,
 *   dt_ijab = (w_ijab + scale R~_ijab) / (e_i + e_j - e_a - e_b) - t_ijab,
 * i.e. t + dt solves D t' = w + scale R~ for the driver w (o, o, v, v; e.g.
 * (ia|jb)) and the orbital energies e_occ (o) and e_vir (v).  t is the
 * context's doubles amplitudes (without the singles dressing); the context's t
 * is not changed: pass dt to cpppl_warm_start to take the step, with the
 * initial guess of the next ALS.  on_device: w, e_occ, e_vir and dt are device
 * pointers (else host).  Synchronises; drops the cached Y_beta and tau.
 * E_STATE without t, B and factors (or for a planted tensor). */
CPPPL_API cpppl_status cpppl_jacobi_step(cpppl_ctx* ctx, const double* w, const double* e_occ,
                                         const double* e_vir, double scale, double* dt,
                                         int on_device);
/* E_CP = sum_ijab CP_ijab t_ijab at the current factors, FP64. */
CPPPL_API cpppl_status cpppl_energy(cpppl_ctx* ctx, double* e_cp);

/* ---- learned warm start (previous converged factors -> next warm start) ------------ */

/* Multi-layer perceptron applied per rank column: in_dim -> hidden (x n_hidden,
 * ReLU) -> out_dim, FP32.  Hidden weights start U(-1/sqrt(fan_in), 1/sqrt(fan_in))
 * from a counter-based generator (SplitMix64) keyed by `seed`, biases and the
 * last layer at zero (an untrained network predicts no correction).
 * `capacity` = rows of training pairs it can hold.  The network owns its
 * device memory (hipMalloc on `device`); its calls use the default stream and
 * return after the work is done. */
CPPPL_API cpppl_status cpppl_mlp_create(int in_dim, int hidden, int n_hidden, int out_dim,
                                        int64_t capacity, uint64_t seed, int device,
                                        cpppl_mlp** out);
CPPPL_API cpppl_status cpppl_mlp_destroy(cpppl_mlp* mlp);
/* Parameters packed in the order W1, b1, W2, b2, ... (W_l: fan_out x fan_in). */
CPPPL_API cpppl_status cpppl_mlp_num_params(const cpppl_mlp* mlp, int64_t* n);
CPPPL_API cpppl_status cpppl_mlp_get_params(cpppl_mlp* mlp, float* out, int on_device);
CPPPL_API cpppl_status cpppl_mlp_set_params(cpppl_mlp* mlp, const float* in, int on_device);
/* Forward pass on n_rows rows of x (n_rows x in_dim) -> y (n_rows x out_dim). */
CPPPL_API cpppl_status cpppl_mlp_forward(cpppl_mlp* mlp, const float* x, int64_t n_rows, float* y,
                                         int on_device);
/* Loss = mean (y_pred - y)^2 and its gradient (packed like the parameters). */
CPPPL_API cpppl_status cpppl_mlp_grad(cpppl_mlp* mlp, const float* x, const float* y,
                                      int64_t n_rows, float* loss, float* grads, int on_device);
/* Append rows to the training set (x: n x in_dim, y: n x out_dim). */
CPPPL_API cpppl_status cpppl_mlp_add_rows(cpppl_mlp* mlp, const float* x, const float* y,
                                          int64_t n_rows, int on_device);
CPPPL_API cpppl_status cpppl_mlp_clear_rows(cpppl_mlp* mlp);
/* Number of stored training rows, and a copy of them (x: n x in_dim, y: n x out_dim). */
CPPPL_API cpppl_status cpppl_mlp_num_rows(const cpppl_mlp* mlp, int64_t* n);
CPPPL_API cpppl_status cpppl_mlp_get_rows(cpppl_mlp* mlp, float* x, float* y, int on_device);
/* Adam (lr, 0.9, 0.999, 1e-8) over the stored rows in mini-batches of `batch`
 * rows (shuffled by a counter-based generator keyed by seed; batch <= 0: full
 * batch, no shuffle).  loss_hist (host, epochs entries) may be NULL. */
CPPPL_API cpppl_status cpppl_mlp_train(cpppl_mlp* mlp, int epochs, float lr, int64_t batch,
                                       uint64_t seed, float* loss_hist);
/* Standardise the stored rows for training and remember how: per input column
 * x' = (x - mean) / std and per output column y' = y / rms over the stored rows
 * (a constant or zero column keeps scale 1).  Rows added later are
 * standardised on the way in, and the learned warm start applies the same map
 * to its features and undoes it on the network's output; cpppl_mlp_forward /
 * cpppl_mlp_grad / cpppl_mlp_train act on the standardised numbers.  Saved and
 * loaded with the parameters.  E_STATE if already standardised, E_ARG with
 * fewer than two rows. */
CPPPL_API cpppl_status cpppl_mlp_standardize(cpppl_mlp* mlp);
/* The standardisation (host arrays; any may be NULL): x_mu, x_inv (in_dim:
 * mean and 1/std) and y_sc (out_dim: rms).  E_STATE if not standardised. */
CPPPL_API cpppl_status cpppl_mlp_get_standardization(cpppl_mlp* mlp, float* x_mu, float* x_inv,
                                                     float* y_sc);
CPPPL_API cpppl_status cpppl_mlp_save(cpppl_mlp* mlp, const char* path);
CPPPL_API cpppl_status cpppl_mlp_load(cpppl_mlp* mlp, const char* path);

/* Warm-start strategies. */
enum {
  CPPPL_WS_PLAIN = 0,       /* previous converged factors (the paper's "optimal guess") */
  CPPPL_WS_LEARNED = 1,     /* previous factors + first-order change + network correction,
                               judged against PLAIN and FIRST_ORDER */
  CPPPL_WS_FIRST_ORDER = 2, /* previous factors + first-order ALS change from dR (no network) */
  CPPPL_WS_NEAR_OPTIMAL = 3 /* the near-optimal cache (see cpppl_als_opts.near_cache); PLAIN
                               while no cache exists.  No features are formed. */
};

/* Feature width of the warm-start network for these dims: 2 (2o + 2v) + 1. */
CPPPL_API int64_t cpppl_ws_in_dim(const cpppl_dims* dims);
CPPPL_API int64_t cpppl_ws_out_dim(const cpppl_dims* dims);

/* Advance the amplitudes by dt (o, o, v, v) and warm-start the factors.
 * Computes the matrix-free MTTKRP of dR (the PPL tensor of dt) at the current
 * (previous converged) factors, forms per-column features [F, D, log10
 * (||dt|| / ||t||)] with D = dR-MTTKRP W^-1 / lambda the first-order change
 * of each factor column (modes i, j, a, b), then sets t <- t + dt and the
 * factors to the chosen candidate.  FIRST_ORDER forms F + D; LEARNED forms
 * F + D and F + D + the network's correction (through the network's
 * standardisation, see cpppl_mlp_standardize).  The judge keeps, of PLAIN and
 * the candidates formed, the one with the lowest ||CP||^2 - 2 <R, CP> (R of
 * the new t); *chosen reports it (a CPPPL_WS_* value).  The raw features are
 * kept for cpppl_ws_training_rows.  mlp may be NULL unless strategy is LEARNED. */
CPPPL_API cpppl_status cpppl_warm_start(cpppl_ctx* ctx, const double* dt, int on_device,
                                        int strategy, cpppl_mlp* mlp, int* chosen);
/* After ALS from a warm start: write the R training rows of that step (the
 * raw features of the warm start, and targets = the current (converged)
 * minus the previous factors, per column, sign-aligned, minus the first-order
 * change D: what the first-order candidate misses) into the network's
 * training set (standardised on the way in if the network is). */
CPPPL_API cpppl_status cpppl_ws_training_rows(cpppl_ctx* ctx, cpppl_mlp* mlp);

/* ---- MTTKRP without allocation ------------------------------------------------ */

/* For callers that cannot allocate device memory (code under HIP stream / graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the FP64
 * matrix-free MTTKRP of cpppl_mttkrp, for one mode (0 i, 1 j, 2 a, 3 b), with
 * no context and no allocation.  All pointers are device pointers on the
 * current HIP device, row-major FP64, caller-owned: t (o, o, v, v), b (nx, v, v),
 * fi, fj (o x R), fa, fb (v x R), m_out (n_mode x R, written).  Work is
 * enqueued on hip_stream (a hipStream_t; NULL = default stream); the call does
 * not synchronise.  Intermediates live in one 64 MiB device array of the
 * library (one per device, held until the process ends), so a problem must fit
 * it: modes a, b need 2oR + Ro^2 + Rv^2 + Xv^2 + 2RXv + Rv doubles, modes i, j
 * oR + 2RXv + Rv^2 + Ro^2 + Ro (each term rounded up to 32), at most 8 Mi
 * doubles; larger problems return CPPPL_E_NOMEM before any work is enqueued.
 * Every call on a device uses that device's array: calls that overlap on one
 * device (other streams or threads) race and must be serialised by the caller.
 * E_ARG for NULL pointers, a bad mode or bad dims; E_HIP for a launch error. */
CPPPL_API cpppl_status cpppl_mttkrp_noalloc(const cpppl_dims* dims, const double* t,
                                            const double* b, const double* fi, const double* fj,
                                            const double* fa, const double* fb, int mode,
                                            double* m_out, void* hip_stream);

/* ---- errors and build identity --------------------------------------------- */
CPPPL_API const char* cpppl_last_error(const cpppl_ctx* ctx);
CPPPL_API const char* cpppl_status_str(cpppl_status s);
/* SHA-256 (hex) of the HIP sources and headers this library was built from
 * (static string), so that a caller can refuse a library built from other sources. */
CPPPL_API const char* cpppl_build_hash(void);

#ifdef __cplusplus
}
#endif

#endif /* CPPPL_H */
