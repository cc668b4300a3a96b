// Internal launch entry points of libmpt (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mpt.h"

namespace mpt {

int bucket_of(int M);

// Options of a single-object sweep:
//   material-1 part of a reduced model (C_M1 = U^H C_sigma,1 U, g_1, E_1: the
//   projections of material 1's conducting edges alone) for
//   sigma_1 dL/dsigma_1 in the adjoint sweep; dsig receives one value per
//   frequency.  All NULL: not computed.
//   sigma (device, 1 value) and inv_sigma0: the model was projected at
//   conductivity sigma0 and is evaluated at sigma, i.e. at w sigma / sigma0
//   (it depends on w sigma only); the adjoint then returns dL/dw at the given
//   w.  sigma NULL: no scaling.
struct MatSens {
  const double* CM1 = nullptr;
  const double* g1 = nullptr;
  const double* E1 = nullptr;
  double* dsig = nullptr;
  const double* sigma = nullptr;
  double inv_sigma0 = 1.0;
};

// sweep.hip
hipError_t sweep_launch(const mpt_rom& R, const double* omega, int64_t n, double* out,
                        double* a_out, int32_t* status, const double* dout, double* dom,
                        hipStream_t st, const MatSens& ms = MatSens{});
// out[0] = sum_k dsig[k], out[1] = sum_k omega_k dom[k] - out[0]
hipError_t material_reduce(const double* omega, const double* dom, const double* dsig, int64_t n,
                           double* out, hipStream_t st);
hipError_t persistent_launch(int bucket, bool adj, const mpt_rom* roms, const int4* items,
                             int n_items, unsigned int* counter, const double* omega, double* out,
                             int32_t* status, const double* dout, double* dom, int wpg, int groups,
                             hipStream_t st);
hipError_t reset_counters(unsigned int* c, int n, hipStream_t st);
hipError_t sigma_reduce(const double* omega, const double* dom, const int64_t* off, int n_obj,
                        double* sig, hipStream_t st);
// one object of n frequencies: sig[0] = sum_k omega_k dom_k, divided by
// sigma[0] when sigma is not NULL (then dL/dsigma)
hipError_t sigma_reduce_one(const double* omega, const double* dom, int64_t n,
                            const double* sigma, double* sig, hipStream_t st);

// select.hip
hipError_t select_launch(const double* omega, int64_t n, const double* out, const double* snap,
                         int n_snap, int n_star, double* new_omega, double* lambda,
                         double* Lambda_max, int64_t* arg_ws, hipStream_t st);

hipError_t select_threshold_launch(const double* omega, int64_t n, const double* out,
                                   const double* snap, int n_snap, double theta,
                                   double* new_omega, int32_t* n_new, double* lambda,
                                   double* Lambda_max, int64_t* arg_ws, hipStream_t st);

// spmm.hip
hipError_t spmm_launch(const mpt_csr& K, const double* U, int64_t ldU, int M, double* Y,
                       int64_t ldY, hipStream_t st);

// gram.hip : complex contractions on FP64 MFMA
//   P (m x n) = A^H B over N rows, A: N x m (lda), B: N x n (ldb), complex.
//   Split-N partials in ws then a fixed-order reduction.
size_t gram_ws_size(int64_t N, int m, int n);
size_t gram2c_ws_size(int64_t N, int m, int n);  // for gram2c_launch
hipError_t gram_launch(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t N,
                       int m, int n, double* P, int64_t ldp, void* ws, hipStream_t st);
//   P1 = A^H B (m x n) and P2 = A^H A (m x m) in one pass over the rows
hipError_t gram2_launch(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t N,
                        int m, int n, double* P1, int64_t ldp1, double* P2, int64_t ldp2,
                        void* ws, hipStream_t st);
//   the same, and from the same MFMAs Q1 = A^H conj(B) (m x n) and, with P2,
//   Q2 = A^H conj(A) (may be null).  herm_ab: A^H B is Hermitian and A^H
//   conj(B) complex symmetric by construction (B = S A, S real symmetric), so
//   only the tiles on and above the diagonal are computed; implied when A == B
hipError_t gram2c_launch(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t N,
                         int m, int n, double* P1, int64_t ldp1, double* P2, int64_t ldp2,
                         double* Q1, int64_t ldq1, double* Q2, int64_t ldq2, bool herm_ab,
                         void* ws, hipStream_t st);
//   C (N x n) = A (N x m) * V (m x n), complex, V small (row-major, ldv);
//   columns n .. n_zero-1 of C (when n_zero > n) are set to zero in the same pass.
hipError_t rotate_launch(const double* A, int64_t lda, int64_t N, int m, const double* V,
                         int64_t ldv, int n, double* C, int64_t ldc, hipStream_t st,
                         int n_zero = 0);
//   T (r x n) = S (r x r, real) * Z (r x n, complex); ws of rcgemm_ws_size
size_t rcgemm_ws_size(int64_t r, int n);
hipError_t real_complex_gemm(const double* S, int64_t r, const double* Z, int n, double* T,
                             void* ws, hipStream_t st);

// cert.hip : certificate data per reference shift (Lemma 4.1):
//   G (n_ref x (2M+3)^2) and D' (n_ref x M x M) from the scaled conductor
//   rows Zc = sqrt(c) [w | U] (n_c x (M+3)), the conductor block's eigenpairs
//   (Vt rows, lam), the shifts, the assembled A0, C_M, U^H U, and the
//   conjugation products U^H conj(K U), U^H conj(U) (M x M) and
//   Zc^H conj(Zc) ((M+3) x (M+3)).
size_t cert_ws_size(int M, int64_t nc, int n_ref);
hipError_t cert_launch(int M, const double* Zc, int64_t nc, const double* Vt, const double* lam,
                       int n_ref, const double* s_ref, const double* A0, const double* CM,
                       const double* UhU, const double* TXk, const double* TXu,
                       const double* TCz, double eps_h, const int32_t* dirs, double* G,
                       double* Dp, void* ws, hipStream_t st);

// eig.hip : Hermitian eigen-decomposition of a small n x n matrix (n <= 192)
//   by cyclic two-sided Jacobi in one workgroup; V (n x n)
//   eigenvectors in columns, lam eigenvalues (unsorted); info[0] sweeps used
//   (or -1 when not converged), info[2] sweeps recorded; ws holds the
//   rotation record and a packed copy of A (jacobi_ws_size bytes); A is read
//   only; tol is the relative rotation threshold and floor_rel the absolute
//   one (times max |a_ii|).
size_t jacobi_ws_size(int n, int max_sweeps);
// tridiag.hip : Hermitian eigen-decomposition (n <= 192) by Householder
//   tridiagonalisation, multisection, inverse iteration, Gram-Schmidt and
//   back-transformation; absolute accuracy ~ eps ||A||.  A (n x n) is read
//   only; V (n x n, V[i n + j] = component i of eigenvector j), lam unsorted.
size_t tridiag_ws_size(int n);
hipError_t tridiag_eig_launch(const double* A, int n, double* V, double* lam, void* ws,
                              hipStream_t st);
hipError_t jacobi_launch(double* A, int n, double* V, double* lam, int* info, void* ws,
                         int max_sweeps, double tol, double floor_rel, hipStream_t st);

// fmm.hip : full matrix method on the reconstructed field q = U a
//   Op: K (N x N; wf == nullptr) or the curl (faces x N) with face weights wf
size_t fmm_ws_size(int64_t N, int64_t rows_R, int M);
hipError_t fmm_launch(const mpt_csr& Op, const double* wf, const double* c, const double* w,
                      const double* U, int64_t N, int64_t ldU, int M, const int32_t* cond,
                      int64_t nc, const double* a, const double* omega, int64_t n,
                      const double* N0, double alpha, double* out, void* ws, hipStream_t st);

// pencil.hip : Hessenberg-triangular form of (A0, C_M) and the sweep on it.
//   Byte offsets of the parts of one object's pencil buffer.  The stacked
//   matrices W come last: NTs shared row tiles (K_M, C_M, then a tile with
//   conj(g)) and, per reference shift, NTr tiles (Gxx, H, D', then a tile
//   with the rows of G_s[Cw, XU] and G_s[Cw, CU]).
constexpr int kPenMaxRef = 64;
struct PencilLayout {
  size_t H, T, f, Z, Zf, S, rec, Aw, W;
  int Mp, Kp, NTs, NTr;  // M rounded up to 16 / to 4; MFMA row tiles of W
};
__host__ __device__ inline PencilLayout pencil_layout(int M) {
  PencilLayout L;
  L.Mp = (M + 15) / 16 * 16;
  L.Kp = (M + 3) / 4 * 4;
  L.NTs = 2 * (L.Mp / 16) + 1;
  L.NTr = 3 * (L.Mp / 16) + 1;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o += (bytes + 255) & ~size_t(255);
    return r;
  };
  const size_t mm = (size_t)M * M * 16;
  L.H = take(mm);
  L.T = take(mm);
  L.f = take((size_t)3 * M * 16);
  L.Z = take(mm);
  L.Zf = take((size_t)(L.Mp / 16) * (L.Kp / 4) * 64 * 16);
  L.S = take((18 + 10 * (size_t)kPenMaxRef) * 8);  // E, N0, then (s, Re G_s[w,w]) per shift
  const size_t nrot = M >= 3 ? (size_t)(M - 1) * (M - 2) / 2 : 1;
  L.rec = take(nrot * 3 * 8);
  L.Aw = take(M > 64 ? (size_t)M * (M + 1) * 16 : 16);  // reduction work copy of A (M > 64)
  L.W = o;
  return L;
}
__host__ __device__ inline size_t pencil_tile_bytes(int M) {
  const PencilLayout L = pencil_layout(M);
  return (size_t)(L.Kp / 4) * 64 * 16;
}
__host__ __device__ inline size_t pencil_total_bytes(int M, int n_ref) {
  const PencilLayout L = pencil_layout(M);
  return L.W + (((size_t)(L.NTs + n_ref * L.NTr) * pencil_tile_bytes(M) + 255) & ~size_t(255));
}
// one object of a pencil reduction: the reduced model's matrices and the
// pencil buffer (laid out by pencil_layout(M))
struct PencilJob {
  int M, n_ref;
  const double* A0;
  const double* CM;
  const double* KM;
  const double* G;
  const double* Dp;
  const double* s_ref;
  const double* g;
  const double* E;
  const double* N0;
  char* base;
};
// per-object arguments of the pencil sweep
struct PencilArgs {
  int M, Mp, Kp, NTs, NTr, n_ref;
  const double2* H;
  const double2* T;
  const double2* f;
  const double2* Zf;
  const double2* W;
  const double* S;
  double alpha, alpha_lb;
};
PencilArgs pencil_args(const mpt_pencil& pen);
// jobs == nullptr: the single job `one`; else n_jobs jobs from the device
// array (maxM bounds their M)
hipError_t pencil_reduce_launch(const PencilJob& one, const PencilJob* jobs, int n_jobs, int maxM,
                                int maxRef, hipStream_t st);
// its two parts: the reduction (H, T, Q^H g, Z; reads A0, C_M, g only) and
// the layout of the quadratic-form matrices (reads K_M, C_M, g, E, N0, G, D')
hipError_t pencil_core_launch(const PencilJob& one, const PencilJob* jobs, int n_jobs, int maxM,
                              hipStream_t st);
hipError_t pencil_layout_launch(const PencilJob& one, const PencilJob* jobs, int n_jobs,
                                int maxRef, hipStream_t st);
// items == nullptr: one object (P) over omega[0, n); else n_items work items
// (object, first omega, count <= 16, -) of objects with segment width L
hipError_t pencil_sweep_launch(const PencilArgs& P, const double* omega, int64_t n, double* out,
                               double* a_out, int32_t* status, hipStream_t st);
hipError_t pencil_sweep_items_launch(int L, const PencilArgs* objs, const int4* items,
                                     int n_items, const double* omega, double* out,
                                     int32_t* status, hipStream_t st);

}  // namespace mpt
