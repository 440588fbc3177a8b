/*
 * gwlt.h -- C ABI of the MI355X (gfx950) LT-AC G0W0 hot path.
 *
 * The operations follow Toelle, Niemeyer & Neugebauer, "Accelerating
 * Analytic-Continuation GW Calculations with a Laplace Transformation and
 * Natural Auxiliary Functions" (LT-GW).  Each entry point names the passage
 * that defines what it computes.
 *
 * Conventions (apply to every call unless stated otherwise)
 *   - Row-major storage, auxiliary (RI) index fastest.
 *   - Orbital indices are absolute (0 = lowest orbital, frozen core first).
 *     "Active" orbitals are those above the n_fc frozen-core orbitals.
 *   - Occupied-virtual rows are i-major: row (i - i0) * n_virt + a, so
 *     occupied chunks are contiguous.
 *   - Three-index tensors are FP64 for GW_FP64 and FP32 for GW_FP32 and
 *     GW_BF16X3 (the BF16 hi/lo split happens in the kernels' tile loads,
 *     never in storage).  Matrices M, K, U are always FP64.
 *   - Complex numbers are interleaved (re, im) FP64 pairs.
 *   - "device" pointers are HIP device memory owned by the caller and
 *     borrowed until the work enqueued by the call has completed on the
 *     context's stream.  "host" arrays are read (or written) during the call
 *     and may be reused as soon as it returns.
 *   - Calls are asynchronous on the context's stream unless they return host
 *     results (gw_naf_compress with finalize, gw_qp_solve, gw_g0w0), which
 *     synchronise the stream before returning.
 *   - Every call returns a gw_status and never throws or aborts.  Argument
 *     errors are detected before anything is enqueued; the message is
 *     available from gw_last_error.  Errors raised by device work (a
 *     non-positive-definite pivot in the screening, a failed eigensolver)
 *     are reported by the next synchronising call or gw_sync.
 *   - One context per host thread; a context holds its workspace (device
 *     memory grown on demand) and is not thread-safe.
 */
#ifndef GWLT_H
#define GWLT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GW_OK = 0,
  GW_EINVAL = 1,          /* invalid argument (null pointer, bad size)      */
  GW_ENOMEM = 2,          /* device allocation failed                      */
  GW_EDEVICE = 3,         /* HIP runtime or device error                   */
  GW_ENOTSPD = 4,         /* 1 - Pi not positive definite in the screening */
  GW_EPADE = 5,           /* Pade nodes coincide                           */
  GW_ENOCONV = 6,         /* an iterative solver did not converge          */
  GW_EUNSUPPORTED = 7     /* precision or mode not implemented             */
} gw_status;

typedef enum {
  GW_FP64 = 0,            /* FP64 throughout                               */
  GW_FP32 = 1,            /* contractions on FP32 MFMA, FP64 screening     */
  GW_BF16X3 = 2           /* contractions as hi*hi + hi*lo + lo*hi BF16
                             MFMA products with FP32 accumulation          */
} gw_precision;

typedef struct gw_ctx_s* gw_ctx;

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  The stream is borrowed.
 * GW_EINVAL: `out` is NULL or no such device; GW_EDEVICE: the HIP runtime
 * reports no usable device (its message is in gw_last_error(NULL));
 * GW_ENOMEM: the staging buffers could not be allocated. */
gw_status gw_create(gw_ctx* out, int device, void* hip_stream);
/* Release the context and its workspace (waits for its stream first). */
gw_status gw_destroy(gw_ctx ctx);
/* Switch the stream later calls enqueue on. */
gw_status gw_set_stream(gw_ctx ctx, void* hip_stream);
/* Wait for the stream; report deferred device-side errors. */
gw_status gw_sync(gw_ctx ctx);
/* Message of the last failure on ctx (ctx may be NULL: the calling thread's
 * last failure of a context-free call).  Valid until the next call. */
const char* gw_last_error(gw_ctx ctx);
const char* gw_status_string(gw_status s);

/* Kernel timing.  While enabled, HIP events bracket the hot kernels on the
 * context's stream (the polarizability SYRK "chi_syrk_f32"/"chi_syrk_f64", the NAF metric "naf_syrk", the
 * self-energy contraction "bwb_f32"/"bwb_f64", the screening sweep
 * "screen_sweep", the NAF transform "naf_gemm_f32"/"naf_gemm_f64" and the
 * eigensolver "naf_eig").  gw_profile_get (synchronises) returns, for one
 * name, the summed event time (ms), the number of launches and the summed
 * algorithmic flops and bytes of those launches; zeros if none ran.
 * Enabling or disabling clears the accumulated figures. */
gw_status gw_profile_enable(gw_ctx ctx, int enable);
gw_status gw_profile_get(gw_ctx ctx, const char* kernel, double* total_ms,
                         int64_t* launches, double* flops, double* bytes);

/* ------------------------------------------------- a1: frozen core, bounds */

/* Sec. 3 (computational details).  From all orbital energies eps[n_occ +
 * n_virt] (host, ascending within the occupied and the virtual block) and
 * the number n_fc of frozen-core orbitals: the Fermi level, taken as the
 * HOMO-LUMO midpoint (the paper leaves it undefined), and the interval of
 * the Laplace variable y = w^2 + (e_a - e_i)^2: y_min = (e_LUMO - e_HOMO)^2 +
 * omega_min^2 (omega_min the smallest integration frequency) and y_max =
 * max((e_vmax - e_i,min)^2, 1e4) over active occupied i.  Host only. */
gw_status gw_prepare(int n_occ, int n_fc, int n_virt, const double* eps,
                     double omega_min, double* eps_F, double* y_min,
                     double* y_max);

/* ------------------------------------------------------------ a3: grids */

/* Modified Gauss-Legendre rule on [0, inf) (Sec. 2 after Eq. 7, Sec. 3):
 * w_k = x0 (1 + t_k) / (1 - t_k), weight_k = 2 x0 v_k / (1 - t_k)^2 with
 * (t_k, v_k) the n-point Gauss-Legendre rule; ascending w.  Host arrays of
 * length n.  1 <= n <= 4096, x0 > 0. */
gw_status gw_freq_grid_mgl(int n, double x0, double* omega, double* weight);

/* Minimax Laplace grid (Eqs. 8-9, Sec. 3): points x[n_lt] and weights
 * w[n_lt] (host, x ascending) minimising max |1/y - sum_m w_m exp(-x_m y)|
 * on [y_min, y_max].  err_norm (may be NULL) receives the equioscillation
 * level of the normalised problem on t = y / y_min in [1, y_max / y_min].
 * 1 <= n_lt <= 20, 0 < y_min < y_max.  GW_ENOCONV if the Remez exchange
 * fails. */
gw_status gw_lt_grid_minimax(int n_lt, double y_min, double y_max,
                             double* x, double* w, double* err_norm);

/* Accuracy-driven Laplace grid (Sec. 3): the smallest n_lt <= max_lt
 * (<= 20) whose normalised minimax error (err_norm of gw_lt_grid_minimax)
 * is at most eps_lt, with its points and weights (x, w host [max_lt]).
 * GW_ENOCONV (with *err_norm the error reached at max_lt) if none is. */
gw_status gw_lt_grid_auto(double eps_lt, int max_lt, double y_min, double y_max, int* n_lt,
                          double* x, double* w, double* err_norm);

/* Minimax of 1/t on [1, R] by n_lt exponentials (the normalised problem
 * behind gw_lt_grid_minimax): alpha (ascending), omega host [n_lt], err the
 * equioscillation level (may be NULL).  With a starting guess (alpha0,
 * omega0, host [n_lt]) only the Remez exchange runs from it; with NULL the
 * built-in table of converged solutions seeds it, falling back to a
 * from-scratch start.  Used to regenerate that table. */
gw_status gw_minimax_inverse(int n_lt, double R, const double* alpha0,
                             const double* omega0, double* alpha,
                             double* omega, double* err);

/* ------------------------------------------------------------- a2: NAF */

/* Natural auxiliary functions, Eqs. 11-13.  Adds the metric contribution
 * of one chunk of rows, K += s (R_oo^T R_oo + 2 R_ov^T R_ov) with s = 2
 * (closed shell; the virtual-virtual block is omitted, Sec. 2), into
 * K (device [n_aux][n_aux] FP64; overwritten instead when accumulate == 0).
 * R_oo (device [n_oo_rows][n_aux]) holds the occupied-occupied rows of both
 * orders (ij and ji); R_ov (device [n_ov_rows][n_aux]) the
 * occupied-virtual rows; either may be NULL with zero rows.
 * With finalize != 0 the call then diagonalises K in FP64 on the device
 * (K is destroyed), keeps the eigenvectors whose eigenvalue is > eps_naf
 * (strict), at most max_keep of them when max_keep > 0, and writes
 *   U       device [n_aux][n_aux] FP64: row p < *n_naf holds the
 *           eigenvector of the p-th largest eigenvalue, so rows
 *           0 .. *n_naf-1 are the NAF basis (U^T of Eq. 13); later rows are
 *           unspecified,
 *   *n_naf  host, number of kept functions (>= 1 unless all eigenvalues are
 *           <= eps_naf, then 0),
 *   eigvals host [n_aux] or NULL: eigenvalues in descending order.
 * finalize synchronises the stream. */
gw_status gw_naf_compress(gw_ctx ctx, gw_precision prec, int n_aux,
                          int64_t n_oo_rows, const void* R_oo,
                          int64_t n_ov_rows, const void* R_ov, double* K,
                          int accumulate, int finalize, double eps_naf,
                          int max_keep, int* n_naf, double* U,
                          double* eigvals);

/* Eq. 13: R_out[r][q] = sum_P R_in[r][P] U[q][P] for q < n_naf.
 * R_in device [n_rows][n_aux], R_out device [n_rows][ld_out] (ld_out = 0
 * means n_naf; columns n_naf .. ld_out-1 are set to zero), both FP64
 * (GW_FP64) or FP32 (otherwise; the product is accumulated in FP32 MFMA
 * with FP64 partial sums).  U as returned by gw_naf_compress. */
gw_status gw_naf_apply(gw_ctx ctx, gw_precision prec, int n_aux, int n_naf,
                       const double* U, int64_t n_rows, const void* R_in,
                       void* R_out, int64_t ld_out);

/* ----------------------------------------------- a4: LT polarizability */

/* Eq. 10: for every Laplace point m,
 *   M^m_PQ += sum_ia R_ia,P  w_m D_ia exp(-D_ia^2 x_m)  R_ia,Q,
 * D_ia = eps_a[a] - eps_i[i], over one chunk of n_i active occupied
 * orbitals.  x_lt, w_lt host [n_lt] (n_lt <= 32); eps_i host [n_i];
 * eps_a host [n_virt]; R_chunk device [n_i * n_virt][ld_R] (i-major; ld_R
 * >= n_naf is the row stride, 0 means n_naf; rows padded to a multiple of
 * 128 columns take the kernel's unguarded load path).
 * M device [n_lt][n_naf][n_naf] FP64.  accumulate == 0 overwrites M,
 * otherwise adds.  Only the lower triangle P >= Q is updated until a call
 * with finalize != 0, which copies it onto the upper triangle (M is then
 * exactly symmetric).  The scale is computed in FP64 and applied to one
 * operand in the tile loads; FP32 and BF16x3 accumulate in FP32 within
 * blocks of 256 rows and in FP64 across blocks. */
gw_status gw_polarizability_lt(gw_ctx ctx, gw_precision prec, int n_naf,
                               int n_lt, const double* x_lt,
                               const double* w_lt, int n_i, int n_virt,
                               const double* eps_i, const double* eps_a,
                               const void* R_chunk, int64_t ld_R,
                               int accumulate, int finalize, double* M);

/* The polarizability without the Laplace transform (Eq. 3, the baseline the
 * paper's speed-ups are measured against): for each frequency j (omega
 * host [n_w]) the sum over states
 *   P_j = sum_ia R_ia D_ia / (omega_j^2 + D_ia^2) R_ia^T,
 * so that Pi_j = -2 s P_j.  The same scaled SYRK as gw_polarizability_lt
 * with one "point" per frequency.  Arguments as there; P device
 * [n_w][n_naf][n_naf] FP64. */
gw_status gw_polarizability_sos(gw_ctx ctx, gw_precision prec, int n_naf, int n_w,
                                const double* omega, int n_i, int n_virt,
                                const double* eps_i, const double* eps_a,
                                const void* R_chunk, int64_t ld_R, int accumulate,
                                int finalize, double* P);

/* ------------------------------------------------ a5 + a6: screening */

/* Eqs. 2 and 10: for each frequency j (omega host [n_w]),
 *   Pi_j = -2 s sum_m exp(-omega_j^2 x_m) M^m   (s = 2),
 *   W_hat_j = (1 - Pi_j)^-1 - 1,
 * with the inverse formed in FP64 by a blocked symmetric Gauss-Jordan
 * sweep.  M device [n_lt][n_naf][n_naf] FP64 (symmetric); x_lt host.
 * W_hat device [n_w][n_naf][n_naf], FP64 for GW_FP64, FP32 otherwise
 * (rounded from the FP64 result); both triangles are written.
 * A non-positive pivot (1 - Pi not positive definite) is reported as
 * GW_ENOTSPD by the next synchronising call.  omega_j = 0 gives the static
 * screened interaction W_hat(0) that a Bethe-Salpeter step built on the
 * quasiparticle energies takes (Sec. 3, static screening). */
gw_status gw_screen(gw_ctx ctx, gw_precision prec, int n_naf, int n_lt,
                    const double* x_lt, const double* M, int n_w,
                    const double* omega, void* W_hat);

/* Eq. 2 from sum-over-states polarizabilities (gw_polarizability_sos):
 * W_hat_j = (1 + 2 s P_j)^-1 - 1 for P device [n_w][n_naf][n_naf] FP64;
 * otherwise as gw_screen. */
gw_status gw_screen_sos(gw_ctx ctx, gw_precision prec, int n_naf, int n_w, const double* P,
                        void* W_hat);

/* ------------------------------------- a7 + a8: diagonal self-energy */

/* Eq. 2 then Eq. 7.  For every QP state n (row block of R_qp) and active
 * orbital m:  W_nm(i omega_j) = R_nm^T W_hat_j R_nm  (the B.W.B
 * contraction, on MFMA), then
 *   Sigma_n(e_F + i wp_k) = -(1/pi) sum_j w_omega_j sum_m
 *        a / (a^2 + omega_j^2) W_nm(i omega_j),  a = i wp_k + eps_F - eps_m,
 * in FP64.  R_qp device [n_qp][n_mo][ld_R] (m over active orbitals; row
 * stride ld_R >= n_naf, 0 means n_naf);
 * eps_mo host [n_mo] (active orbital energies); omega, w_omega host [n_w];
 * W_hat as written by gw_screen; omega_pade host [n_pade].
 * sigma_iw device [n_qp][n_pade] complex; accumulate != 0 adds this
 * frequency batch to it.  W_nm: optional device [n_w][n_qp][n_mo] FP64
 * output (NULL to skip). */
gw_status gw_sigma_diag(gw_ctx ctx, gw_precision prec, int n_naf, int n_qp,
                        int n_mo, const double* eps_mo, double eps_F,
                        const void* R_qp, int64_t ld_R, int n_w,
                        const double* omega,
                        const double* w_omega, const void* W_hat,
                        int n_pade, const double* omega_pade, int accumulate,
                        double* sigma_iw, double* W_nm);

/* gw_sigma_diag for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, results and errors as gw_sigma_diag, but the
 * call's buffers (row-dot partials, W_nm staging and, for GW_FP32, the
 * k-major copy of R_qp) live in a fixed per-GPU scratch array of 64 MiB
 * that the library holds from its loading until the process ends; nothing
 * is allocated or freed.  A call needing more than 64 MiB returns GW_EINVAL
 * (split the frequencies or the QP states over calls with accumulate = 1).
 * Every call on one GPU uses that GPU's single array: calls that overlap
 * on one GPU (several streams or contexts) race, so serialise them. */
gw_status gw_sigma_diag_noalloc(gw_ctx ctx, gw_precision prec, int n_naf, int n_qp,
                                int n_mo, const double* eps_mo, double eps_F,
                                const void* R_qp, int64_t ld_R, int n_w,
                                const double* omega, const double* w_omega,
                                const void* W_hat, int n_pade,
                                const double* omega_pade, int accumulate,
                                double* sigma_iw, double* W_nm);

/* ------------------------------------------------ a9: Pade + QP solve */

/* Sec. 2 and Sec. 3: Thiele continued-fraction Pade approximant through
 * (i omega_pade_k, Sigma_n(e_F + i omega_pade_k)) (Vidberg-Serene), then the
 * fixed point E = eps_n + Re Sigma_n(E - eps_F + i eta) + static_n from
 * E = eps_n, stopping when |dE| < tol or after max_iter steps; FP64 on the
 * device.  eps_n, static_n (NULL = 0) host [n_qp]; sigma_iw device as from
 * gw_sigma_diag.  Outputs host [n_qp]: eps_qp, z_factor (may be NULL;
 * Z = 1 / (1 - dRe Sigma/dE) at the solution), status (0 converged,
 * 1 not converged within max_iter, 2 non-finite).  GW_EPADE when two
 * Pade nodes coincide.  Synchronises the stream. */
gw_status gw_qp_solve(gw_ctx ctx, int n_qp, const double* eps_n,
                      const double* static_n, double eps_F, int n_pade,
                      const double* omega_pade, const double* sigma_iw,
                      double eta, double tol, int max_iter, double* eps_qp,
                      double* z_factor, int* status);

/* ------------------------------------------------- the whole G0W0 step */

typedef struct {
  int n_occ, n_fc, n_virt, n_aux;   /* orbital and auxiliary counts       */
  int n_lt, n_freq, n_pade, n_qp;   /* grid sizes and number of QP states */
  double eps_naf;                   /* NAF threshold (strict ">")         */
  int max_keep;                     /* NAF cap, 0 = none                  */
  double x0;                        /* modified GL scale (Ha), e.g. 0.5   */
  double eta;                       /* real-axis broadening (Ha)          */
  double tol;                       /* QP convergence (Ha)                */
  int max_iter;                     /* QP iterations                      */
  int freq_batch;                   /* frequencies per screening batch,
                                       0 = all at once                    */
  int no_lt;                        /* 1: polarizability as the sum over
                                       states at every frequency (Eq. 3,
                                       the AC baseline without the Laplace
                                       transform); 0: Laplace form        */
  double eps_lt;                    /* > 0: accuracy-driven Laplace grid,
                                       the smallest one whose normalised
                                       minimax level is <= eps_lt (Sec. 3),
                                       with n_lt as its upper bound (0 or
                                       past 20: 20); 0: n_lt points      */
} gw_params;

typedef struct {
  int n_naf;                        /* kept natural auxiliary functions   */
  double lt_err_norm;               /* minimax level of the Laplace grid  */
  double t_naf_ms, t_chi_ms, t_screen_ms, t_sigma_ms, t_qp_ms, t_total_ms;
  int n_lt;                         /* Laplace points taken (last cycle)  */
} gw_stats;

/* One LT-AC G0W0 evaluation (a1-a9 in order): NAF compression of the raw
 * tensors, grids, LT polarizability, screening, self-energy and QP energies.
 * eps host [n_occ + n_virt]; qp host [n_qp] absolute indices of active QP
 * orbitals; static_n host [n_qp] or NULL.  Raw tensors on the device over
 * active orbitals: R_oo [o][o][n_aux], R_ov [o * n_virt][n_aux],
 * R_qp [n_qp][o + n_virt][n_aux] (o = n_occ - n_fc), FP64 for GW_FP64 and
 * FP32 otherwise.  Outputs host [n_qp]: eps_qp, z_factor (or NULL),
 * status; sigma_iw host [n_qp][n_pade] complex or NULL; stats or NULL.
 * Device intermediates live in the context's workspace.  Synchronises. */
gw_status gw_g0w0(gw_ctx ctx, gw_precision prec, const gw_params* params,
                  const double* eps, const int* qp, const double* static_n,
                  const void* R_oo, const void* R_ov, const void* R_qp,
                  double* eps_qp, double* z_factor, int* status,
                  double* sigma_iw, gw_stats* stats);

/* Eigenvalue-self-consistent GW (Sec. 3, Table 3): n_cycles G0W0
 * evaluations sharing one NAF basis (it depends only on the tensors).  Cycle
 * 0 uses eps; cycle c > 0 uses the orbital energies made from cycle c-1's
 * quasiparticle energies: QP states take them, other active occupied
 * orbitals are shifted by the correction of the lowest QP state, other
 * active virtual orbitals by that of the highest (frozen core unchanged).
 * Each cycle rebuilds everything that depends on the energies: the Laplace
 * grid bounds and points, the Laplace matrices M^m, the screening, the
 * self-energy with its Fermi level.  The QP equation keeps the starting
 * point as its base, E_n = eps_n + static_n + Re Sigma^c_n(E_n), with
 * Sigma^c built from the cycle's energies.  Arguments as for gw_g0w0;
 * outputs host: eps_qp [n_cycles][n_qp] (row c = cycle c), status
 * [n_cycles][n_qp], z_factor [n_qp] of the last cycle (or NULL), eps_last
 * [n_occ + n_virt] the energies the next cycle would use (or NULL).  stats
 * (or NULL): NAF time, chi/screen/sigma/QP times summed over the cycles,
 * total.  Synchronises. */
gw_status gw_evgw(gw_ctx ctx, gw_precision prec, const gw_params* params, int n_cycles,
                  const double* eps, const int* qp, const double* static_n,
                  const void* R_oo, const void* R_ov, const void* R_qp,
                  double* eps_qp, double* z_factor, int* status, double* eps_last,
                  gw_stats* stats);

/* ------------------------------------------------------------ autotuner */

/* Launch-shape autotuning.  With tuning on (the default), the first call of
 * a kernel family on a new shape times its candidate launch shapes with HIP
 * events and keeps the fastest for that shape on this context: the outer
 * pivot width of the screening sweep (64, 128 or 256 columns, i.e. the rank
 * of its trailing update) and the split-K factor of the Laplace SYRK.  Later
 * calls on the shape, and calls inside a graph capture, use the kept choice
 * (or the default when none is kept yet).  Results do not depend on the
 * choice beyond rounding order.  enable: 0 off (defaults), 1 on, 2 on and
 * forget the kept choices, -1 leave as is; *n_tuned (may be NULL) receives
 * the number of kept choices. */
gw_status gw_autotune(gw_ctx ctx, int enable, int* n_tuned);

/* Restrict the launch-shape candidates of one kernel family on this context
 * to the codes c with c % modulus == residue (modulus 0 lifts the
 * restriction; a restriction that matches no candidate of a shape is
 * ignored for it).  With tuning on the autotuner times the remaining
 * candidates; with tuning off the first remaining one is used.  For tests
 * that cover every shape, and for pinning a shape.  Families and codes:
 *   "syrk3"  BF16x3 polarizability SYRK: 4 S + shape, S the split-K factor;
 *            128 x 128 tiles: shape 0: 4 waves, 2 LDS stages; 1: 4 waves,
 *            3 stages; 2: 8 waves, 2 stages; 3: 256 x 128 tiles, 8 waves,
 *            3 stages
 *   "syrk"   FP32 / FP64 polarizability SYRK: the split-K factor S
 *   "screen", "screen_sos"  screening sweep: outer pivot width (64, 128, 256)
 *   "bwb3"   BF16x3 B W B contraction: waves per workgroup
 *   "eigvec" NAF eigenvectors (not timed by the autotuner): 0 the twisted
 *            factorisation for isolated eigenvalues and inverse iteration
 *            for clusters; 1 LU inverse iteration for every vector
 * Errors: GW_EINVAL for a NULL ctx or family, modulus < 0, or a residue
 * outside [0, modulus). */
gw_status gw_autotune_restrict(gw_ctx ctx, const char* family, int modulus, int residue);

/* Keep the autotuner's choices across processes.  gw_autotune_save writes
 * the choices kept on this context to the text file `path` (overwritten):
 * a first line naming the format and the device (architecture and
 * compute-unit count), then one line "<choice> <shape key>" per tuned
 * shape.  gw_autotune_load reads such a file into the context's kept
 * choices (replacing those of the same shapes; *n_loaded, may be NULL,
 * receives the number read).  A loaded choice is used like one timed on
 * the context: only while it is among the shape's current candidates (see
 * gw_autotune_restrict), otherwise the shape is tuned or defaulted as
 * usual.  Errors: GW_EINVAL for a NULL ctx or path, a file that cannot be
 * opened or written, a file saved on another kind of device, or a
 * malformed line (the context is then left unchanged); GW_EDEVICE when
 * the device properties cannot be read. */
gw_status gw_autotune_save(gw_ctx ctx, const char* path);
gw_status gw_autotune_load(gw_ctx ctx, const char* path, int* n_loaded);

/* ----------------------------------------------------------- workspace */

/* Largest sizes the per-step calls will see on a context. */
typedef struct {
  int n_aux;        /* raw auxiliary functions (NAF metric and transform)    */
  int n_naf;        /* natural auxiliary functions                            */
  int n_occ_act;    /* active occupied orbitals                               */
  int n_virt;       /* virtual orbitals                                       */
  int n_mo;         /* orbitals in the self-energy sum (active)               */
  int n_qp;         /* QP states                                              */
  int n_lt;         /* Laplace points                                         */
  int n_w;          /* frequencies per gw_screen / gw_sigma_diag call         */
  int n_pade;       /* Pade nodes                                             */
  int chunk_i;      /* occupied orbitals per chunk of the chunked calls,
                       0 = all of them                                        */
} gw_dims;

/* Grow the context's workspace now to what gw_naf_compress (metric part),
 * gw_naf_apply, gw_polarizability_lt, gw_screen, gw_sigma_diag and
 * gw_qp_solve need for sizes up to *dims in precision prec, so that later
 * calls within those sizes allocate nothing (in particular while being
 * captured into a graph).  The workspace never shrinks while the context
 * lives. */
gw_status gw_reserve(gw_ctx ctx, gw_precision prec, const gw_dims* dims);

/* ------------------------------------------------------ graph capture */

/* Capture the device work of the following calls on ctx into a HIP graph
 * and replay it.  Between gw_graph_begin and gw_graph_end the calls are
 * recorded, not run: ctx enqueues on a private capturing stream, and the
 * host arrays the calls receive are copied into a device arena owned by the
 * graph, so every replay sees the values given at capture.  Capturable:
 * gw_naf_compress without finalize, gw_naf_apply, gw_polarizability_lt,
 * gw_screen, gw_sigma_diag and their batched twins.  Calls that return host
 * results or synchronise (finalize, gw_qp_solve, gw_g0w0, gw_sync,
 * gw_profile_*, gw_set_stream) fail with GW_EUNSUPPORTED while capturing,
 * as does any call that would have to grow the context's workspace: run
 * the sequence once eagerly first.  While a graph lives, calls that would
 * grow the workspace fail (the graph holds its buffers' addresses).
 * gw_graph_launch enqueues a replay on ctx's stream; device arrays named at
 * capture are read and written again in place.  gw_graph_destroy waits for
 * ctx's stream, then releases the graph and its arena. */
typedef struct gw_graph_s* gw_graph;
gw_status gw_graph_begin(gw_ctx ctx);
gw_status gw_graph_end(gw_ctx ctx, gw_graph* out);
gw_status gw_graph_launch(gw_ctx ctx, gw_graph graph);
gw_status gw_graph_destroy(gw_graph graph);

/* ---------------------------------------- batched twins (many molecules) */

/* The batched calls run the same computation as their single-molecule
 * twins for n_jobs independent problems of uneven size in one launch per
 * kernel: every work unit (tile, frequency, QP state) of every job goes
 * into one grid, longest units first.  Arguments per job mean what they
 * mean in the single call. */

/* Eqs. 11-13 for each job (see gw_naf_compress): both metric contributions
 * of every job in two launches, then the FP64 eigendecompositions as
 * batched divide-and-conquer solves over groups of similar n_aux (each
 * metric padded with a decoupled -1 diagonal block, which the exact block
 * structure keeps out of the kept eigenvectors).  Always finalises: K is
 * destroyed, U receives the eigenvectors as rows (descending), n_naf the
 * kept count, eigvals (host, may be NULL) the eigenvalues.  Synchronises. */
typedef struct {
  int n_aux;
  int64_t n_oo_rows;
  const void* R_oo;         /* device [n_oo_rows][n_aux] */
  int64_t n_ov_rows;
  const void* R_ov;         /* device [n_ov_rows][n_aux] */
  double* K;                /* device [n_aux][n_aux] FP64 work */
  double eps_naf;
  int max_keep;
  double* U;                /* device [n_aux][n_aux] FP64 */
  int n_naf;                /* out */
  double* eigvals;          /* host [n_aux] or NULL */
} gw_naf_job;
gw_status gw_naf_compress_batched(gw_ctx ctx, gw_precision prec, int n_jobs,
                                  gw_naf_job* jobs);

/* Eq. 13 for each job (see gw_naf_apply), one launch. */
typedef struct {
  int n_aux, n_naf;
  const double* U;          /* device, as from the compression */
  int64_t n_rows;
  const void* R_in;         /* device [n_rows][n_aux] */
  void* R_out;              /* device [n_rows][ld_out] */
  int64_t ld_out;           /* 0 = n_naf */
} gw_naf_apply_job;
gw_status gw_naf_apply_batched(gw_ctx ctx, gw_precision prec, int n_jobs,
                               const gw_naf_apply_job* jobs);

/* Eq. 10 for each job (see gw_polarizability_lt); all jobs share n_lt. */
typedef struct {
  int n_naf, n_i, n_virt;
  const double* x_lt;       /* host [n_lt] */
  const double* w_lt;       /* host [n_lt] */
  const double* eps_i;      /* host [n_i] */
  const double* eps_a;      /* host [n_virt] */
  const void* R_chunk;      /* device [n_i * n_virt][ld_R] */
  int64_t ld_R;             /* 0 = n_naf */
  double* M;                /* device [n_lt][n_naf][n_naf] FP64 */
} gw_chi_job;
gw_status gw_polarizability_lt_batched(gw_ctx ctx, gw_precision prec, int n_lt,
                                       int n_jobs, const gw_chi_job* jobs,
                                       int accumulate, int finalize);

/* Eqs. 2 and 10 for each job (see gw_screen); all jobs share n_lt.
 * A non-positive pivot is reported as GW_ENOTSPD by the next synchronising
 * call, naming the job and frequency. */
typedef struct {
  int n_naf;
  const double* x_lt;       /* host [n_lt] */
  const double* M;          /* device [n_lt][n_naf][n_naf] FP64 */
  int n_w;
  const double* omega;      /* host [n_w] */
  void* W_hat;              /* device [n_w][n_naf][n_naf] */
} gw_screen_job;
gw_status gw_screen_batched(gw_ctx ctx, gw_precision prec, int n_lt, int n_jobs,
                            const gw_screen_job* jobs);

/* Eqs. 2 and 7 for each job (see gw_sigma_diag). */
typedef struct {
  int n_naf, n_qp, n_mo;
  const double* eps_mo;     /* host [n_mo] */
  double eps_F;
  const void* R_qp;         /* device [n_qp][n_mo][ld_R] */
  int64_t ld_R;             /* 0 = n_naf */
  int n_w;
  const double* omega;      /* host [n_w] */
  const double* w_omega;    /* host [n_w] */
  const void* W_hat;        /* device [n_w][n_naf][n_naf] */
  int n_pade;
  const double* omega_pade; /* host [n_pade] */
  double* sigma_iw;         /* device [n_qp][n_pade] complex */
  double* W_nm;             /* device [n_w][n_qp][n_mo] FP64 or NULL */
} gw_sigma_job;
gw_status gw_sigma_diag_batched(gw_ctx ctx, gw_precision prec, int n_jobs,
                                const gw_sigma_job* jobs, int accumulate);

/* Pade + QP fixed point for each job (see gw_qp_solve); one launch for all
 * states of all jobs.  Synchronises. */
typedef struct {
  int n_qp;
  const double* eps_n;      /* host [n_qp] */
  const double* static_n;   /* host [n_qp] or NULL */
  double eps_F;
  int n_pade;
  const double* omega_pade; /* host [n_pade] */
  const double* sigma_iw;   /* device [n_qp][n_pade] complex */
  double* eps_qp;           /* host [n_qp] */
  double* z_factor;         /* host [n_qp] or NULL */
  int* status;              /* host [n_qp] */
} gw_qp_job;
gw_status gw_qp_solve_batched(gw_ctx ctx, int n_jobs, const gw_qp_job* jobs,
                              double eta, double tol, int max_iter);

/* One molecule of gw_g0w0_batched: its sizes, NAF rule, energies, raw
 * tensors (as for gw_g0w0) and host outputs. */
typedef struct {
  int n_occ, n_fc, n_virt, n_aux, n_qp;
  double eps_naf;
  int max_keep;
  const double* eps;        /* host [n_occ + n_virt] */
  const int* qp;            /* host [n_qp] absolute indices of active orbitals */
  const double* static_n;   /* host [n_qp] or NULL */
  const void* R_oo;         /* device [o][o][n_aux] */
  const void* R_ov;         /* device [o * n_virt][n_aux] */
  const void* R_qp;         /* device [n_qp][o + n_virt][n_aux] */
  double* eps_qp;           /* host [n_qp] */
  double* z_factor;         /* host [n_qp] or NULL */
  int* status;              /* host [n_qp] */
  double* sigma_iw;         /* host [n_qp][n_pade] complex or NULL */
  int n_naf;                /* out: kept natural auxiliary functions */
} gw_mol;

/* Grid sizes and QP settings shared by all molecules of a batch. */
typedef struct {
  int n_lt, n_freq, n_pade;
  double x0, eta, tol;
  int max_iter;
} gw_batch_params;

#define GW_BATCH_GRAPH 1    /* replay the post-NAF work as one HIP graph */

typedef struct {
  double t_naf_ms;          /* NAF of all molecules (eager)               */
  double t_rest_ms;         /* polarizability .. QP of all molecules      */
  double t_total_ms;
  int graph_replayed;       /* 1 if the post-NAF work ran as a cached graph */
} gw_batch_stats;

/* G0W0 for n_mol molecules of uneven size (a1-a9 for each).  The NAF stage
 * runs eagerly: both metric SYRKs of all molecules in two launches, the
 * eigendecompositions as batched FP64 solves over groups of similar size
 * (each metric padded with a decoupled -1 diagonal block, which the exact
 * block structure keeps out of the kept eigenvectors), the transforms per
 * molecule.  Each molecule gets its own Laplace grid.  The rest (Laplace
 * polarizability, screening, self-energy, QP) runs as batched launches; with
 * GW_BATCH_GRAPH in flags those launches are captured once into a HIP graph
 * after an eager run and replayed by later calls whose sizes, NAF counts and
 * device inputs are unchanged.  Synchronises. */
gw_status gw_g0w0_batched(gw_ctx ctx, gw_precision prec, const gw_batch_params* params,
                          int n_mol, gw_mol* mols, int flags, gw_batch_stats* stats);

#ifdef __cplusplus
}
#endif

#endif /* GWLT_H */
