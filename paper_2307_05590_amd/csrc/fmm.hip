// Full matrix method (FMM): the tensors of eqs. (Rmatrixmeth) and
// (I_tensor_coeffs) evaluated with the full-order operators on the field
// reconstructed from the reduced solutions, q_i = U a_i (§4).  Up to rounding
// it equals the reduced matrix method; it is the comparison point whose cost
// grows with N instead of M.  The integration-method analogue on this grid
// (sums over faces, eq. (NRI)) takes the same path with the curl: R from
// sum_f w_f Re(conj((C q_i)_f) (C q_j)_f), w_f = 1/(mu_f h).
//
// Per batch of kFmmBatch frequencies (3 kFmmBatch columns):
//   V = the batch's a vectors as an M x 3B matrix (transpose of the n x 3 x M
//       input), Q = U V on FP64 MFMA (rotation kernel), Y = K Q (SpMM);
//   k_fmm_dots: per frequency and pair i <= j, Re(q_i^H y_j) over all rows
//       (row chunks, fixed-order two-stage reduction);
//   k_fmm_cond: per frequency and pair, c_e Re(v_i^H v_j) with v = q + w over
//       the conductor rows only (C_sigma vanishes elsewhere);
//   k_fmm_finish: R~ = N0 - a^3/4 (.), I = w a^3/4 (.).
// Every pass is bound by HBM traffic over the N x 3B panels.
#include "device_util.h"
#include "kernels.h"

namespace mpt {

constexpr int kFmmBatch = 16;      // frequencies per batch
constexpr int kFmmCols = 3 * kFmmBatch;
constexpr int kFmmChunks = 256;    // row chunks of the dot reduction

namespace {
constexpr int kPi6[6] = {0, 0, 0, 1, 1, 2};
constexpr int kPj6[6] = {0, 1, 2, 1, 2, 2};
}  // namespace

// V[m][3b + i] = a[((w0 + b) 3 + i) M + m], zero for b >= nb
__global__ void k_fmm_gather(const double2* __restrict__ a, int64_t w0, int nb, int M,
                             double2* __restrict__ V) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * kFmmCols) return;
  const int m = e / kFmmCols, col = e % kFmmCols, b = col / 3, i = col % 3;
  V[e] = b < nb ? a[((w0 + b) * 3 + i) * M + m] : make_double2(0.0, 0.0);
}

// partial[chunk][b][p] = sum over the chunk's rows of
//   wt[r] Re(conj(Q[r][3b+i]) Y[r][3b+j])   (wt == nullptr: weight 1);
// 256 threads: 16 frequencies x 16 row lanes
__global__ __launch_bounds__(256) void k_fmm_dots(const double2* __restrict__ Q,
                                                  const double2* __restrict__ Y,
                                                  const double* __restrict__ wt, int64_t N,
                                                  int64_t rows_per_chunk,
                                                  double* __restrict__ partial) {
  __shared__ double red[6][256];
  const int b = threadIdx.x & 15, rl = threadIdx.x >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_chunk;
  const int64_t r1 = min(N, r0 + rows_per_chunk);
  double acc[6];
#pragma unroll
  for (int p = 0; p < 6; ++p) acc[p] = 0.0;
  for (int64_t r = r0 + rl; r < r1; r += 16) {
    const double2* q = Q + r * kFmmCols + 3 * b;
    const double2* y = Y + r * kFmmCols + 3 * b;
    double2 qv[3], yv[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      qv[i] = q[i];
      yv[i] = y[i];
    }
    const double f = wt ? wt[r] : 1.0;
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      const double2 x = qv[kPi6[p]], z = yv[kPj6[p]];
      acc[p] = fma(f, fma(x.x, z.x, x.y * z.y), acc[p]);
    }
  }
#pragma unroll
  for (int p = 0; p < 6; ++p) red[p][threadIdx.x] = acc[p];
  __syncthreads();
  if (threadIdx.x < 16 * 6) {
    const int bb = threadIdx.x & 15, p = threadIdx.x >> 4;
    double s = 0.0;
    for (int k = 0; k < 16; ++k) s += red[p][k * 16 + bb];  // fixed order
    partial[((size_t)blockIdx.x * kFmmBatch + bb) * 6 + p] = s;
  }
}

// cpart[b][p] = sum over conductor rows k of c_e Re(conj(v_i) v_j), v = Q + w
// (one workgroup per frequency of the batch)
__global__ __launch_bounds__(256) void k_fmm_cond(const double2* __restrict__ Q,
                                                  const double* __restrict__ w,
                                                  const double* __restrict__ c,
                                                  const int32_t* __restrict__ cond, int64_t nc,
                                                  double* __restrict__ cpart) {
  __shared__ double red[6][256];
  const int b = blockIdx.x;
  double acc[6];
#pragma unroll
  for (int p = 0; p < 6; ++p) acc[p] = 0.0;
  for (int64_t k = threadIdx.x; k < nc; k += blockDim.x) {
    const int64_t e = cond[k];
    const double ce = c[e];
    double2 v[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double2 qq = Q[e * kFmmCols + 3 * b + i];
      v[i] = make_double2(qq.x + w[e * 3 + i], qq.y);
    }
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      const double2 x = v[kPi6[p]], z = v[kPj6[p]];
      acc[p] = fma(ce, fma(x.x, z.x, x.y * z.y), acc[p]);
    }
  }
#pragma unroll
  for (int p = 0; p < 6; ++p) red[p][threadIdx.x] = acc[p];
  __syncthreads();
  for (int s = 128; s >= 1; s >>= 1) {
    if (threadIdx.x < s)
#pragma unroll
      for (int p = 0; p < 6; ++p) red[p][threadIdx.x] += red[p][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 6) cpart[b * 6 + threadIdx.x] = red[threadIdx.x][0];
}

// out[w0 + b][0..5] = N0 - a^3/4 R-sum, out[..][6..11] = w a^3/4 I-sum
__global__ void k_fmm_finish(const double* __restrict__ partial, int chunks,
                             const double* __restrict__ cpart, const double* __restrict__ omega,
                             const double* __restrict__ N0, double a3, int64_t w0, int nb,
                             double* __restrict__ out) {
  const int t = threadIdx.x;
  if (t >= nb * 6) return;
  const int b = t / 6, p = t % 6;
  double s = 0.0;
  for (int k = 0; k < chunks; ++k) s += partial[((size_t)k * kFmmBatch + b) * 6 + p];
  const int i = kPi6[p], j = kPj6[p];
  const double om = omega[w0 + b];
  out[(w0 + b) * 12 + p] = N0[3 * i + j] - 0.25 * a3 * s;
  out[(w0 + b) * 12 + 6 + p] = 0.25 * a3 * om * cpart[b * 6 + p];
}

size_t fmm_ws_size(int64_t N, int64_t rows_R, int M) {
  const size_t panel_q = (((size_t)N * kFmmCols * sizeof(double2)) + 255) & ~size_t(255);
  const size_t panel_y = (((size_t)rows_R * kFmmCols * sizeof(double2)) + 255) & ~size_t(255);
  return panel_q + panel_y + (((size_t)M * kFmmCols * 16 + 255) & ~size_t(255)) +
         (size_t)kFmmChunks * kFmmBatch * 6 * 8 + 256 + kFmmBatch * 6 * 8;
}

// R from Y = Op q: the FMM (Op = K, N x N, rows reduced with q) or the
// integration-method analogue (Op = the curl, faces x N, rows weighted by wf
// and reduced with Y itself)
hipError_t fmm_launch(const mpt_csr& Op, const double* wf, const double* c, const double* w,
                      const double* U, int64_t N, int64_t ldU, int M, const int32_t* cond,
                      int64_t nc, const double* a, const double* omega, int64_t n,
                      const double* N0, double alpha, double* out, void* ws, hipStream_t st) {
  const int64_t rows_R = Op.n;
  const size_t panel_q = (((size_t)N * kFmmCols * sizeof(double2)) + 255) & ~size_t(255);
  const size_t panel_y = (((size_t)rows_R * kFmmCols * sizeof(double2)) + 255) & ~size_t(255);
  char* p = static_cast<char*>(ws);
  double2* Q = reinterpret_cast<double2*>(p);
  double2* Y = reinterpret_cast<double2*>(p + panel_q);
  double2* V = reinterpret_cast<double2*>(p + panel_q + panel_y);
  double* partial = reinterpret_cast<double*>(p + panel_q + panel_y +
                                              (((size_t)M * kFmmCols * 16 + 255) & ~size_t(255)));
  double* cpart = partial + (size_t)kFmmChunks * kFmmBatch * 6;
  const int64_t rpc = (rows_R + kFmmChunks - 1) / kFmmChunks;
  const int chunks = (int)((rows_R + rpc - 1) / rpc);
  const double2* left = wf ? Y : Q;  // IM: |C q|^2 weighted; FMM: q^H (K q)
  const double a3 = alpha * alpha * alpha;
  for (int64_t w0 = 0; w0 < n; w0 += kFmmBatch) {
    const int nb = (int)(n - w0 < kFmmBatch ? n - w0 : kFmmBatch);
    hipLaunchKernelGGL(k_fmm_gather, dim3((M * kFmmCols + 255) / 256), dim3(256), 0, st,
                       reinterpret_cast<const double2*>(a), w0, nb, M, V);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = rotate_launch(U, ldU, N, M, reinterpret_cast<const double*>(V), kFmmCols, kFmmCols,
                      reinterpret_cast<double*>(Q), kFmmCols, st);
    if (e != hipSuccess) return e;
    e = spmm_launch(Op, reinterpret_cast<const double*>(Q), kFmmCols, kFmmCols,
                    reinterpret_cast<double*>(Y), kFmmCols, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fmm_dots, dim3(chunks), dim3(256), 0, st, left, Y, wf, rows_R, rpc,
                       partial);
    hipLaunchKernelGGL(k_fmm_cond, dim3(kFmmBatch), dim3(256), 0, st, Q, w, c, cond, nc, cpart);
    hipLaunchKernelGGL(k_fmm_finish, dim3(1), dim3(kFmmBatch * 6), 0, st, partial, chunks, cpart,
                       omega, N0, a3, w0, nb, out);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace mpt
