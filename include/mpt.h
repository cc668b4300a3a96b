/*
 * mpt.h - C ABI of libmpt: the data-parallel hot path of the adaptive POD
 * method for magnetic polarizability tensor (MPT) spectral signatures
 * (Elgy & Ledger, arXiv 2307.05590), built for AMD Instinct MI355X (gfx950).
 *
 * Conventions for every call
 *   - All numeric arrays are device pointers owned by the caller; the library
 *     never frees caller memory.  Scratch memory is caller-provided through
 *     (ws, ws_bytes) arguments whose minimum size is returned by the matching
 *     *_ws_size query (host call, no device work).
 *   - Complex numbers are FP64 pairs (re, im) laid out like double2 /
 *     std::complex<double>; every matrix is row-major with the stated leading
 *     dimension.  "Hermitian" outputs are stored in full.
 *   - Work is enqueued on the handle's HIP stream and is asynchronous unless a
 *     call says it synchronises.  Calls on one handle must not overlap.
 *   - Every call returns an mpt_status; on failure mpt_last_error() returns a
 *     message that stays valid until the next call on the handle.  Argument
 *     errors are detected on the host before any launch.
 *
 * Notation (the paper's): snapshot matrix D = [D_1 D_2 D_3] (Section 4.1,
 * eq. (D)), POD basis U (eqs. (SVD), (truncSVD)), reduced system
 * A^M(w) p = r^M(w) (eq. (ReducedA)) with A^M = A0 - i w C_M and
 * r_i^M = i w g_i, tensors R~ = N0 + R and I (eqs. (podprealmpt),
 * (podpimagmpt)), certificate Delta (Lemma 4.1), adaptive selection
 * (Algorithm 1).  The regularised full-order operator is
 * A(w) = K + eps h I - i w C_sigma (eq. (Linear)); X = K + eps h I.
 */
#ifndef MPT_H
#define MPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MPT_OK = 0,
  MPT_E_ARG = 1,         /* invalid argument (shape, pointer, size) */
  MPT_E_HIP = 2,         /* HIP runtime error */
  MPT_E_NOMEM = 3,       /* workspace too small */
  MPT_E_SINGULAR = 4,    /* zero or non-finite pivot in a reduced solve */
  MPT_E_NOTPD = 5,       /* eigen-solver failed to converge */
  MPT_E_UNSUPPORTED = 6  /* size outside what the kernels support */
} mpt_status;

typedef struct mpt_handle_s* mpt_handle;

/* One handle per HIP stream (hip_stream may be NULL for the null stream). */
mpt_status mpt_create(int device, void* hip_stream, mpt_handle* out);
mpt_status mpt_destroy(mpt_handle h);
mpt_status mpt_set_stream(mpt_handle h, void* hip_stream);
const char* mpt_last_error(mpt_handle h);
/* Largest reduced dimension M accepted by the sweep kernels. */
int mpt_max_reduced_dim(void);

/* Real sparse matrix in CSR form (sorted column indices, 0-based).
 * row_blocks is a layout hint for the sparse products: 0 or 1 when the rows
 * have one spatial order; k > 1 when they form k equal consecutive blocks
 * whose members follow one common spatial order (the three edge orientations
 * of a Yee grid, each numbered with the same slowest coordinate).  The
 * products then give each XCD the same slab of every block, so a row's
 * stencil neighbours in the other blocks are read through that XCD's L2.
 * k must divide n (MPT_E_ARG otherwise).  Results do not depend on it. */
typedef struct {
  int64_t n;              /* rows = columns */
  int64_t nnz;
  const int32_t* rowptr;  /* n + 1 */
  const int32_t* colind;  /* nnz */
  const double* val;      /* nnz */
  int32_t row_blocks;
  int32_t pad_;
} mpt_csr;

/*
 * Reduced model of one object (all device pointers, row-major):
 *   KM  M x M     K_M = U^H K U                      (eq. (podprealmpt))
 *   A0  M x M     K_M + eps h U^H U                  (A^M at w = 0)
 *   CM  M x M     C_M = U^H C_sigma U                (eq. (podpimagmpt))
 *   g   3 x M     row i = U^H C_sigma w_i, w_i = x_i + o_i (source, r = i w g)
 *   G   n_ref x (2M+3)^2   residual Grams G_s = Z^H (X + s C_sigma)^{-1} Z,
 *                 one per reference shift s = s_ref[k], with
 *                 Z = [C_sigma w_1..3 | X U | C_sigma U]     (Lemma 4.1)
 *   Dp  n_ref x M x M      conjugation-defect forms D'_s (mpt_project)
 *   s_ref n_ref   reference shifts, ascending, s_ref[0] = 0
 *   E   3 x 3     w_i^T C_sigma w_j                   (the omega-independent
 *                 I terms of (I_tensor_coeffs) under Remark 3.1)
 *   N0  3 x 3     static tensor (eq. (NRI), first line)
 * alpha is the object size (m); alpha_lb the stability constant of Lemma 4.1
 * (2 / (3 + sqrt 10) for these reference norms).  At frequency w the
 * certificate uses the largest s_ref[k] <= w.  KM, A0, CM, G and Dp are
 * Hermitian by definition and must be stored Hermitian: the sweep reads row r
 * of these matrices as the conjugate of column r (one coalesced load per
 * column).  mpt_project stores them exactly Hermitian.  1 <= n_ref <= 64.
 *
 * Per-direction form (one basis per direction, Section 4.1: a TSVD of each
 * D_i; eqs. (podprealmpt), (podpimagmpt) with the cross blocks
 * K^M_ij = U_i^H K U_j, C^M_ij, U_i^H C w_j): dirs = (M_1, M_2, M_3), all
 * >= 1 with sum M, and every matrix above is that of the concatenated basis
 * [U_1 U_2 U_3] (whose diagonal blocks are the per-direction matrices and
 * whose off-diagonal blocks are the cross blocks), except Dp, which then
 * holds n_ref x 3 matrices (mpt_project_dirs).  Direction i is solved in its
 * own basis, (A_ii - i w C_ii) a_i = i w (U_i^H C w_i), and placed in the slots
 * of U_i.  dirs = (0, 0, 0) is the joint form.  Only mpt_sweep takes the
 * per-direction form (M <= 64); the other entry points reject it.
 */
typedef struct {
  int32_t M;
  int32_t n_ref;
  const double* KM;
  const double* A0;
  const double* CM;
  const double* g;
  const double* G;
  const double* Dp;
  const double* s_ref;
  const double* E;
  const double* N0;
  double alpha;
  double alpha_lb;
  int32_t dirs[3];  /* per-direction block sizes, or 0, 0, 0 (joint) */
  int32_t pad_;
} mpt_rom;

/* ----------------------------------------------------------------------
 * a1  POD basis (Section 4.1, eqs. (SVD), (truncSVD); Algorithm 1 steps
 *     "Form D_i" / "obtain the TSVDs").
 * D: N x ncol complex (ldD >= ncol), the joint snapshot matrix
 *    [q_1(w_1..K) | q_2(...) | q_3(...)].
 * Thin SVD by passes of Gram / Hermitian eigen-decomposition / rotation
 * (FP64 MFMA Gram and rotation): pass 1 eigen-decomposes D^H D by Householder
 * tridiagonalisation, multisection and inverse iteration; the columns D V_T
 * of its tail (eigenvalues under 1e-10 of the largest, which pass 1 leaves
 * mixed) get the same treatment on their own Gram, whose eigenvalues under
 * 64 eps of its largest (singular values under ~1.2e-12 s_1) it cannot
 * resolve: those directions leave the basis computation (reported by those
 * eigenvalues); pass 2 diagonalises the Gram of the remaining rotated
 * snapshots by Jacobi (relative accuracy of the small singular values),
 * leaving out columns whose norms are under 1e-13 of the largest (reported
 * by their norms).
 * Then truncation: M = #{s_m/s_1 >= max(tol_sigma, 1e-12)},
 * capped at M_cap, and lowered while s_{M+1}/s_M > 1 - 1e-8 (never splits
 * a cluster).  Relative singular values under 1e-12 are rounding noise of
 * FP64 data, so a fixed-rank request (tol_sigma = 0) stops at the numerical
 * rank.  Writes U (N x M_cap, ldU >= M_cap; columns >= M are zero), sigma
 * (ncol, descending).  *M_out is a HOST pointer: the call synchronises the
 * stream to learn M (as it does twice before to size its steps); U is then
 * formed on the stream, complete in stream order.  ncol <= 192.
 */
size_t mpt_pod_basis_ws_size(int64_t N, int ncol);
mpt_status mpt_pod_basis(mpt_handle h, const double* D, int64_t ldD, int64_t N, int ncol,
                         double tol_sigma, int M_cap, double* U, int64_t ldU,
                         double* sigma, int* M_out, void* ws, size_t ws_bytes);

/* ----------------------------------------------------------------------
 * a2  Galerkin projection (eq. (ReducedA); eqs. (podprealmpt),
 *     (podpimagmpt); residual Gram of Lemma 4.1).
 * K: the full-order curl-curl matrix (N x N).  c: diagonal of C_sigma (N).
 * w: N x 3 real (x_i + o_i).  o: N x 3 real theta~^(0) DOFs or NULL (mu_r=1).
 * vol: 3 values h^3 sum_{faces normal to e_i} (1 - 1/mu_f).
 * U: N x M complex basis (ldU).
 * Conductor data for the certificate (Lemma 4.1): cond (n_c sorted edge
 * indices with c > 0) and the eigen-decomposition of the conductor block of
 * X^{-1}, X = K + eps h I, scaled by the conductivities:
 *   Dc^(1/2) P^T X^{-1} P Dc^(1/2) = Vt^T diag(lam) Vt,   Dc = diag(c[cond]),
 * Vt (n_c x n_c, row-major, row k = eigenvector k), lam (n_c).  With it the
 * residual Gram in the norm of X + s C_sigma needs no solve:
 * Dc^(1/2) P^T (X + s C)^{-1} P Dc^(1/2) = Vt^T diag(lam / (1 + s lam)) Vt
 * (Sherman-Morrison-Woodbury).  s_ref (n_ref, device, ascending, s_ref[0] =
 * 0) lists the reference shifts.
 * Outputs (device, row-major): KM, A0, CM (M x M), g (3 x M),
 * G (n_ref x (2M+3)^2; G_s with Z = [C w | X U | C U]), Dp (n_ref x M x M;
 *   D'_s = D_s / 2 + 4 eps h U^H U, where a^H D_s a is the squared distance
 *   in the norm of X + s C from conj(U a) to span(U):
 *   D_s = A_s - conj(T_s^H A_s^{-1} T_s), A_s = U^H (X + s C) U,
 *   T_s = U^H (X + s C) conj(U)), E (3x3), N0 (3x3; alpha^3 vol_i delta_ij +
 * alpha^3/4 o^T K o).  Y (N x M complex) receives K U when non-NULL (else it
 * lives in ws).  1 <= M <= 96, 1 <= n_ref <= 64.
 */
size_t mpt_project_ws_size(int64_t N, int M, int64_t n_c, int n_ref);
mpt_status mpt_project(mpt_handle h, const mpt_csr* K, const double* c, double eps_h,
                       const double* w, const double* o, const double* vol, double alpha,
                       const double* U, int64_t ldU, int M,
                       const int32_t* cond, int64_t n_c, const double* Vt, const double* lam,
                       int n_ref, const double* s_ref,
                       double* KM, double* A0, double* CM, double* g, double* G, double* Dp,
                       double* E, double* N0, double* Y, void* ws, size_t ws_bytes);

/* The same projection onto a concatenated per-direction basis
 * U = [U_1 U_2 U_3] (dirs: HOST array of the three widths, each >= 1, sum M;
 * the per-direction form of mpt_rom).  Every output is mpt_project's for U,
 * except Dp (n_ref x 3 x M x M): for shift k and target direction i,
 * Dp[k][i] is block diagonal with the blocks D'_{i<-j} = D_{i<-j} / 2 +
 * 4 eps h U_j^H U_j (j = 1..3, M_j x M_j), where a^H D_{i<-j} a is the squared
 * distance in the norm of X + s C from conj(U_j a) to span(U_i):
 *   D_{i<-j} = A_s,jj - conj(T_ij^H A_s,ii^{-1} T_ij),
 *   A_s,ii = U_i^H (X + s C) U_i,  T_ij = U_i^H (X + s C) conj(U_j).
 * Galerkin orthogonality of direction i's error holds against span(U_i)
 * only, so the certificate's linear term for the pair (i, j) uses e_{j->i} =
 * (a_j^H D'_{i<-j} a_j)^(1/2).  ws: mpt_project_ws_size bytes.  1 <= M <= 64. */
mpt_status mpt_project_dirs(mpt_handle h, const mpt_csr* K, const double* c, double eps_h,
                            const double* w, const double* o, const double* vol, double alpha,
                            const double* U, int64_t ldU, int M, const int32_t* dirs,
                            const int32_t* cond, int64_t n_c, const double* Vt,
                            const double* lam, int n_ref, const double* s_ref, double* KM,
                            double* A0, double* CM, double* g, double* G, double* Dp, double* E,
                            double* N0, double* Y, void* ws, size_t ws_bytes);

/* Residual Gram of Lemma 4.1 for one reference shift s from columns prepared
 * by the caller:
 *   G_s = (P + P^H) / 2,  P = Z^H Y over the N rows,
 * where Z (N x (2M+3), ldZ) = [C_sigma w_1..3 | X U | C_sigma U] holds the
 * affine residual's columns (ordered as in mpt_project's G) and
 * Y (N x (2M+3), ldY) = (X + s C_sigma)^{-1} Z comes from the caller's
 * full-order solver, as in the paper's offline stage.  mpt_project builds the
 * same matrices from the conductor block instead, with no solve per basis
 * vector.  The certificate w^H G_s w is a difference of terms larger than
 * itself, so its rounding floor depends on how Y was computed.  Output G:
 * (2M+3)^2 complex, row-major, exactly Hermitian; it may replace slot k of a
 * reduced model's G when s = s_ref[k].  1 <= M <= 96.  Workspace:
 * mpt_residual_gram_ws_size.  Asynchronous on the handle's stream. */
size_t mpt_residual_gram_ws_size(int64_t N, int M);
mpt_status mpt_residual_gram(mpt_handle h, const double* Z, int64_t ldZ, const double* XinvZ,
                             int64_t ldY, int64_t N, int M, double* G, void* ws,
                             size_t ws_bytes);

/* Sparse x tall-skinny product Y = K U (K real CSR, U complex N x M,
 * ldU / ldY >= M).  The bandwidth-bound kernel of the projection. */
mpt_status mpt_spmm(mpt_handle h, const mpt_csr* K, const double* U, int64_t ldU, int M,
                    double* Y, int64_t ldY);

/* ----------------------------------------------------------------------
 * a3+a4  Online sweep (eq. (ReducedA) per frequency; eqs. (podprealmpt),
 *     (podpimagmpt); Lemma 4.1).
 * For each omega[k]: LU with partial pivoting of A0 - i w CM, the three
 * solves a_i for r_i = i w g_i, then out[k*18 + p]:
 *   p = 0..5   R~ (11,12,13,22,23,33)
 *   p = 6..11  I  (same order)
 *   p = 12..17 Delta (same order):
 *     Delta_ij = a^3/(8 alpha_lb) (n_i^2 + n_j^2 + ||r_i - r_j||^2)
 *                + a^3/4 (n_i e_j + n_j e_i),
 *     n_i^2 = w^(i)H G_s w^(i), ||r_i - r_j||^2 = n_i^2 + n_j^2
 *     - 2 Re w^(i)H G_s w^(j), w^(i) = [i w e_i ; -a_i ; i w a_i],
 *     e_i = (max(0, a_i^H D'_s a_i))^(1/2), s = the largest s_ref <= w.
 *   Delta bounds |R~ - R~^PODP|_ij and |I - I^PODP|_ij (the second term
 *   covers the part of the error that Galerkin orthogonality leaves linear in
 *   the residual when span(U) is not closed under conjugation).
 * Per-direction form (rom->dirs set, M <= 64): a_i solves direction i's own
 * system (A0 - i w CM restricted to block i, right-hand side i w g_i
 * restricted to block i) and is zero outside block i; the tensors and the
 * Grams use the full matrices of the concatenated basis, and the linear term
 * is a^3/4 (n_i e_{j->i} + n_j e_{i->j}), e_{j->i} = (a_j^H Dp[s][i] a_j)^(1/2).
 * a_out (n_omega x 3 x M complex) receives a_i when non-NULL.
 * status[k] (device) = 0, or MPT_E_SINGULAR when a pivot was zero or
 * non-finite.  The call does not synchronise: it returns MPT_OK once the work
 * is enqueued, and the caller reads status after the stream.  rom is a HOST
 * struct holding device pointers.  1 <= M <= mpt_max_reduced_dim() (96);
 * M <= 64 runs one frequency per wave segment in registers, larger M one
 * frequency per workgroup with the system in LDS.
 */
mpt_status mpt_sweep(mpt_handle h, const mpt_rom* rom, const double* omega, int64_t n_omega,
                     double* out, double* a_out, int32_t* status);

/* ----------------------------------------------------------------------
 * a5  Snapshot selection (Algorithm 1 selection step).
 * omega (n, ascending), out (n x 18 from mpt_sweep; the Delta columns are
 * used), snap (n_snap ascending).  Intervals snap_j < w < snap_{j+1}
 * (Algorithm 1's snap_j <= w < snap_{j+1} without its left end, a snapshot
 * already: no frequency of the snapshot set is returned again);
 * Lambda_j = max Delta over the interval; the n_star intervals
 * with the largest Lambda_j (ties: lower j) each give one new frequency at
 * their argmax (ties: smaller omega).  Device outputs: new_omega (n_star,
 * rank order; NaN when fewer intervals hold frequencies), lambda (n_snap-1;
 * -inf for empty intervals), Lambda_max (1).  ws: device workspace of
 * mpt_select_snapshots_ws_size(n_snap) bytes (per-interval argmax).
 */
size_t mpt_select_snapshots_ws_size(int n_snap);
mpt_status mpt_select_snapshots(mpt_handle h, const double* omega, int64_t n, const double* out,
                                const double* snap, int n_snap, int n_star,
                                double* new_omega, double* lambda, double* Lambda_max, void* ws,
                                size_t ws_bytes);

/* Allocation-free variant of mpt_select_snapshots, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same inputs, outputs and results
 * without a workspace argument.  Its per-interval scratch is a static device
 * array of the library, MPT_SELECT_STATIC_MAX_SNAP (4096) snapshot
 * frequencies = 32 KiB per GPU, held until the process ends; n_snap above
 * that limit is rejected (MPT_E_ARG).  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (several streams or threads) race.
 * Nothing is allocated: no hipMalloc, hipFree or allocating library routine. */
#define MPT_SELECT_STATIC_MAX_SNAP 4096
mpt_status mpt_select_snapshots_static(mpt_handle h, const double* omega, int64_t n,
                                       const double* out, const double* snap, int n_snap,
                                       int n_star, double* new_omega, double* lambda,
                                       double* Lambda_max);

/* Threshold variant of the selection (the alternative to a fixed N_* that
 * Section 4.4 names, after Hesthaven et al.): every interval whose maximum reaches
 * theta * Lambda (0 < theta <= 1) gives its argmax, at most one per interval,
 * in the rank order of mpt_select_snapshots.  new_omega (n_snap - 1, device;
 * NaN after the last chosen), n_new (1 int32, device) the number chosen;
 * lambda, Lambda_max and ws as in mpt_select_snapshots. */
mpt_status mpt_select_snapshots_threshold(mpt_handle h, const double* omega, int64_t n,
                                          const double* out, const double* snap, int n_snap,
                                          double theta, double* new_omega, int32_t* n_new,
                                          double* lambda, double* Lambda_max, void* ws,
                                          size_t ws_bytes);

/* ----------------------------------------------------------------------
 * a6  Batched dictionary sweep: one persistent launch (captured in a HIP
 * graph when use_graph != 0) over many objects with their own M, omega
 * count and materials.  roms: DEVICE array of n_obj mpt_rom.  omega_off
 * (n_obj + 1, host) indexes omega / out / status: object o owns rows
 * omega_off[o] .. omega_off[o+1]-1.  Results equal mpt_sweep object by
 * object.  tune: NULL for the tuned defaults.  Every object needs M <= 64
 * (MPT_E_UNSUPPORTED otherwise).  ws: device workspace of
 * mpt_sweep_batched_ws_size bytes that holds the work-item plan; the graph of
 * the last call is reused while every argument (ws included) stays the same,
 * and a call that rewrites the plan drops it.  Uploading a new plan
 * synchronises the stream.
 */
typedef struct {
  int32_t omegas_per_item;   /* frequencies per work item (>= 1) */
  int32_t waves_per_group;   /* 1, 2 or 4 */
  int32_t groups_per_cu;     /* persistent groups per compute unit */
  int32_t reserved;
} mpt_tuning;

size_t mpt_sweep_batched_ws_size(const mpt_rom* roms_host, int n_obj, const int64_t* omega_off,
                                 const mpt_tuning* tune);
mpt_status mpt_sweep_batched(mpt_handle h, const mpt_rom* roms_host, const mpt_rom* roms_dev,
                             int n_obj, const int64_t* omega_off, const double* omega,
                             double* out, int32_t* status, const mpt_tuning* tune,
                             int use_graph, void* ws, size_t ws_bytes);

/* ----------------------------------------------------------------------
 * a7  Adjoint of the sweep (differentiated signature).
 * Given upstream gradients dout (n x 18; the Delta columns are ignored) of a
 * scalar L with respect to the sweep outputs, computes dL/domega[k] by an
 * adjoint reduced solve A^H lambda_i = dL/d(conj a_i) re-using the LU of
 * A (recomputed here; nothing is kept between calls), and
 * sig_dsig = sigma_* dL/dsigma_* (one value) for a single conductivity
 * that scales C_sigma, g and E with the basis frozen.
 * Same sizes and rom rules as mpt_sweep, with M <= 64 (MPT_E_UNSUPPORTED
 * otherwise).  No workspace; asynchronous (sig_dsig is a device pointer).
 */
mpt_status mpt_sweep_adjoint(mpt_handle h, const mpt_rom* rom, const double* omega, int64_t n,
                             const double* dout, double* dL_domega, double* sig_dsig,
                             int32_t* status);

/* The differentiable signature of one object at conductivity sigma (device
 * pointer, 1 value) when its reduced model was projected at sigma0: the
 * model depends on w sigma only (C_sigma, g, E proportional to sigma, basis
 * frozen), so
 *   mpt_signature: the outputs of mpt_sweep at w sigma / sigma0;
 *   mpt_signature_adjoint: dL/dw_k at the given w_k (chain rule included)
 *     and dL/dsigma = sum_k w_k dL/dw_k / sigma (one device value), from
 *     upstream gradients dout (n x 18, the Delta columns ignored).
 * M <= 64.  No workspace; asynchronous. */
mpt_status mpt_signature(mpt_handle h, const mpt_rom* rom, const double* omega, int64_t n,
                         const double* sigma, double sigma0, double* out, int32_t* status);
mpt_status mpt_signature_adjoint(mpt_handle h, const mpt_rom* rom, const double* omega, int64_t n,
                                 const double* sigma, double sigma0, const double* dout,
                                 double* dL_domega, double* dL_dsigma, int32_t* status);

/* Per-material sigma sensitivities of an object with two conducting
 * materials (C_sigma = C_1 + C_2, C_m proportional to sigma_m on material
 * m's edges; basis frozen, K_M independent of sigma).  CM1 (M x M), g1
 * (3 x M) and E1 (3 x 3, real) are the parts of C_M, g and E that material 1
 * contributes (mpt_project of material 1's conductivities alone).  The
 * adjoint of each frequency's solve gives
 *   sigma_1 dL/dsigma_1 = sum_k [ -w_k Im sum_i lambda_i^H (g_1,i + C_M1 a_i)
 *                                 + sum_p dL/dI_p (w_k a^3/4)(E_1 + Re(a_i^H C_M1 a_j
 *                                   + a_i^H g_1,j + g_1,i^H a_j))_p ],
 * and sigma_2 dL/dsigma_2 = sum_k w_k dL/dw_k - sigma_1 dL/dsigma_1 (the
 * reduced model depends on sigma w only).  Outputs: dL_domega (n) as in
 * mpt_sweep_adjoint, sig_dsig (2 device doubles: material 1, material 2),
 * status.  M <= 64 (MPT_E_UNSUPPORTED otherwise).  ws: device workspace of
 * mpt_sweep_adjoint_materials_ws_size(n) bytes.  Asynchronous. */
size_t mpt_sweep_adjoint_materials_ws_size(int64_t n);
mpt_status mpt_sweep_adjoint_materials(mpt_handle h, const mpt_rom* rom, const double* CM1,
                                       const double* g1, const double* E1, const double* omega,
                                       int64_t n, const double* dout, double* dL_domega,
                                       double* sig_dsig, int32_t* status, void* ws,
                                       size_t ws_bytes);

/* Batched adjoint over a dictionary (same layout and workspace as
 * mpt_sweep_batched, with tune = NULL); sig_dsig has one value per object. */
mpt_status mpt_sweep_adjoint_batched(mpt_handle h, const mpt_rom* roms_host,
                                     const mpt_rom* roms_dev, int n_obj,
                                     const int64_t* omega_off, const double* omega,
                                     const double* dout, double* dL_domega, double* sig_dsig,
                                     int32_t* status, void* ws, size_t ws_bytes);

/* ----------------------------------------------------------------------
 * Pencil form of the sweep: the shifted-system method of Laub (IEEE TAC
 * 1981) applied to eq. (ReducedA).
 * mpt_pencil_reduce, once per object: unitary Q and Z with
 *   Q^H A0 Z = H (upper Hessenberg),  Q^H C_M Z = T (upper triangular)
 * (Householder QR of C_M, then Givens rotations from both sides), f_i =
 * Q^H g_i, and the quadratic-form matrices of eqs. (podprealmpt),
 * (podpimagmpt) and Lemma 4.1 (one set per reference shift) in MFMA
 * fragment order.  buf (device, >= mpt_pencil_bytes(M, rom->n_ref) bytes,
 * owned by the caller and kept alive while the pencil is used) receives all
 * of it; *out (host struct) receives device
 * pointers into buf.  The rom matrices are only read and may be freed after
 * the stream has passed the call.  1 <= M <= 96 (above 64 the reduction
 * keeps its working copy of A in buf and the sweep holds two rows per lane).
 * mpt_sweep_pencil: per frequency the Hessenberg system
 *   (H - i w T) y_i = i w f_i,   a_i = Z y_i,
 * solved by column elimination with pivoting between adjacent columns
 * (O(M^2)), and the same outputs as mpt_sweep (out n x 18, a_out n x 3 x M
 * when non-NULL, status per frequency: 0 or MPT_E_SINGULAR), equal to them up
 * to rounding.  Asynchronous like mpt_sweep.
 */
typedef struct {
  int32_t M;
  int32_t n_ref;     /* reference shifts of the certificate */
  const double* H;   /* M x M complex, column-major */
  const double* T;   /* M x M complex, column-major */
  const double* f;   /* 3 x M complex */
  const double* Z;   /* M x M complex, row-major */
  const double* W;   /* stacked matrices, MFMA fragment order */
  const double* S;   /* E (3 x 3), N0, then per shift: s, Re G_s[w, w] (3 x 3) */
  double alpha;
  double alpha_lb;
} mpt_pencil;

size_t mpt_pencil_bytes(int M, int n_ref);
mpt_status mpt_pencil_reduce(mpt_handle h, const mpt_rom* rom, void* buf, size_t bytes,
                             mpt_pencil* out);

/* mpt_project followed by mpt_pencil_reduce in one call (joint basis only):
 * the same outputs, bit for bit, as the two calls in a row (the rom matrices
 * as mpt_project writes them, and the pencil in pbuf, pbytes >=
 * mpt_pencil_bytes(M, n_ref), as mpt_pencil_reduce writes it; alpha_lb is the
 * pencil's stability constant, > 0).  The reduction needs A0, C_M and g only,
 * so it runs on a private stream of the handle, forked from and joined back
 * into the handle's stream by events, beside the certificate data (G, D');
 * the call stays asynchronous and stream-ordered for the caller.  Both
 * buffers (ws and pbuf) must stay allocated until the stream has passed the
 * call.  1 <= M <= 96, 1 <= n_ref <= 64; errors as for the two calls. */
mpt_status mpt_project_pencil(mpt_handle h, const mpt_csr* K, const double* c, double eps_h,
                              const double* w, const double* o, const double* vol, double alpha,
                              const double* U, int64_t ldU, int M,
                              const int32_t* cond, int64_t n_c, const double* Vt,
                              const double* lam, int n_ref, const double* s_ref,
                              double* KM, double* A0, double* CM, double* g, double* G,
                              double* Dp, double* E, double* N0, double* Y, void* ws,
                              size_t ws_bytes, void* pbuf, size_t pbytes, double alpha_lb,
                              mpt_pencil* pen);
mpt_status mpt_sweep_pencil(mpt_handle h, const mpt_pencil* pen, const double* omega,
                            int64_t n_omega, double* out, double* a_out, int32_t* status);

/* Pencil form for a dictionary: one call reduces every object (one
 * workgroup per object and stage) and sweeps all objects' frequencies (work
 * items of 16 frequencies of one object, one launch per segment width).
 * roms_host: n_obj host structs (device pointers), 1 <= M <= 96 each;
 * omega_off (n_obj + 1, host, omega_off[0] = 0) indexes omega / out / status
 * as in mpt_sweep_batched; buf (device, >= mpt_pencil_batched_bytes) holds
 * the objects' pencils, packed in order, and the work-item plan.  The plan is
 * uploaded once and reused while the arguments stay the same (the call
 * synchronises the stream when it uploads a new plan).  Results equal
 * mpt_sweep_pencil object by object. */
size_t mpt_pencil_batched_bytes(const mpt_rom* roms_host, int n_obj, const int64_t* omega_off);
mpt_status mpt_sweep_pencil_batched(mpt_handle h, const mpt_rom* roms_host, int n_obj,
                                    const int64_t* omega_off, const double* omega, void* buf,
                                    size_t bytes, double* out, int32_t* status);

/* ----------------------------------------------------------------------
 * Full matrix method (eqs. (Rmatrixmeth), (I_tensor_coeffs)) on the field
 * reconstructed from reduced solutions, q_i = U a_i (§4): per frequency
 *   R~_ij = N0_ij - a^3/4 Re(q_i^H K q_j),
 *   I_ij  = w a^3/4 Re((q_i + w_i)^H C_sigma (q_j + w_j)),
 * with the full-order K (CSR) and C_sigma = diag(c) (nonzero on the n_c
 * conductor edges listed in cond).  Equal to the reduced matrix method of
 * mpt_sweep up to rounding; its cost grows with N (the comparison method).
 * K, c (N), w (N x 3 real, the sources w_i), U (N x M complex, ldU >= M),
 * cond (n_c), a (n x 3 x M complex, e.g. mpt_sweep's a_out), omega (n),
 * N0 (3 x 3) are device pointers; out (n x 12): R~ (11 12 13 22 23 33) then
 * I.  ws: mpt_tensors_fmm_ws_size(N, M) bytes.  Asynchronous.
 */
size_t mpt_tensors_fmm_ws_size(int64_t N, int M);
mpt_status mpt_tensors_fmm(mpt_handle h, const mpt_csr* K, const double* c, const double* w,
                           const double* U, int64_t ldU, int M, const int32_t* cond, int64_t n_c,
                           const double* a, const double* omega, int64_t n, const double* N0,
                           double alpha, double* out, void* ws, size_t ws_bytes);

/* Integration-method analogue of eq. (NRI) on this grid: the same outputs,
 * with R_ij = -a^3/4 Re sum_f face_w[f] conj((C q_i)_f) (C q_j)_f over the
 * faces (curl: n_faces x N face-edge incidence, CSR with curl->n = n_faces
 * rows; face_w = 1/(mu_f h)) and I as in mpt_tensors_fmm.  N is the number of
 * edges (rows of U).  ws: mpt_tensors_im_ws_size(N, n_faces, M) bytes. */
size_t mpt_tensors_im_ws_size(int64_t N, int64_t n_faces, int M);
mpt_status mpt_tensors_im(mpt_handle h, const mpt_csr* curl, const double* face_w,
                          const double* c, const double* w, const double* U, int64_t N,
                          int64_t ldU, int M, const int32_t* cond, int64_t n_c, const double* a,
                          const double* omega, int64_t n, const double* N0, double alpha,
                          double* out, void* ws, size_t ws_bytes);

#ifdef __cplusplus
}
#endif
#endif /* MPT_H */
