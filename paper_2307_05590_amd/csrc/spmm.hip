// Y = K U: real CSR (curl-curl, ~12.6 nonzeros per row) times a complex
// tall-skinny basis (N x M, row-major).  Every nonzero gathers a row segment
// of U, so the kernel is bound by gathers that miss L2.
//   - The columns are processed in chunks of 8 VEC (<= 24) complex values:
//     a narrower gathered segment keeps the stencil neighbourhood of the rows
//     in flight inside an XCD's L2 (measured: about a third of the fetched
//     bytes of a full-width pass at M = 48), at the price of one more read
//     of the CSR arrays per chunk.
//   - Eight lanes share an output row (VEC columns each), so a wave works on
//     eight rows; a row's nonzeros are taken thirteen at a time (the length
//     of a curl-curl row on a Yee grid): the column indices and values
//     first, then all the U gathers, then the FMAs.  A scheduling barrier
//     keeps the gathers together: left alone, the compiler moves each gather
//     next to its FMA to save registers and leaves only a few in flight
//     (measured 12% slower at M = 48).
//   - Workgroups are mapped XCD-aware: each of the 8 XCDs receives a
//     contiguous range of row groups, so the stencil neighbours of its rows
//     share that XCD's L2.  When the rows form k equal blocks in one spatial
//     order (row_blocks = k: the three edge orientations of a Yee grid), the
//     groups of the k blocks are interleaved before the split, so an XCD
//     walks the same slab of every block in step and the neighbours a row
//     finds in the other blocks are in its own L2 too.
#include "device_util.h"
#include "kernels.h"

namespace mpt {

constexpr int kSpmmLanes = 8;                        // lanes per output row
constexpr int kSpmmRowsPerPass = 256 / kSpmmLanes;   // rows in flight per workgroup
constexpr int kSpmmBatch = 13;                       // nonzeros per gather batch

template <int VEC>
__global__ __launch_bounds__(256) void k_spmm(int64_t n, const int32_t* __restrict__ rowptr,
                                              const int32_t* __restrict__ colind,
                                              const double* __restrict__ val,
                                              const double2* __restrict__ U, int64_t ldU, int M,
                                              int c0, double2* __restrict__ Y, int64_t ldY,
                                              int64_t rows_per_group, int nblk) {
  const int64_t nb = gridDim.x;
  const int64_t b = blockIdx.x;
  const int64_t q = nb / 8, rem = nb % 8;
  const int64_t xcd = b % 8, slot = b / 8;
  // XCD x owns q (+1 when x < rem) consecutive logical groups
  const int64_t lb = xcd * q + min(xcd, rem) + slot;
  // logical group lb = group g of row block lb % nblk
  const int64_t nrb = n / nblk;  // rows per block
  const int64_t ob = lb % nblk, g = lb / nblk;
  const int64_t rbeg = ob * nrb + g * rows_per_group;
  const int sub = threadIdx.x / kSpmmLanes;
  const int l = threadIdx.x % kSpmmLanes;
  const int64_t rend = min((ob + 1) * nrb, rbeg + rows_per_group);
  int col[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    const int c = c0 + l + v * kSpmmLanes;
    col[v] = c < M ? c : M - 1;  // clamped: loads stay in the row
  }
  for (int64_t r = rbeg + sub; r < rend; r += kSpmmRowsPerPass) {
    const int e0 = rowptr[r], e1 = rowptr[r + 1];
    double2 acc[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] = make_double2(0.0, 0.0);
    for (int e = e0; e < e1; e += kSpmmBatch) {
      int jj[kSpmmBatch];
      double vv[kSpmmBatch];
#pragma unroll
      for (int t = 0; t < kSpmmBatch; ++t) {
        const int ee = e + t < e1 ? e + t : e1 - 1;  // clamped: loads stay in the row
        jj[t] = colind[ee];
        vv[t] = val[ee];
      }
#pragma unroll
      for (int t = 0; t < kSpmmBatch; ++t)
        if (e + t >= e1) vv[t] = 0.0;  // padding entries add zero
      double2 a[kSpmmBatch][VEC];
#pragma unroll
      for (int t = 0; t < kSpmmBatch; ++t)
#pragma unroll
        for (int v = 0; v < VEC; ++v) a[t][v] = U[(int64_t)jj[t] * ldU + col[v]];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int t = 0; t < kSpmmBatch; ++t)
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          acc[v].x = fma(vv[t], a[t][v].x, acc[v].x);
          acc[v].y = fma(vv[t], a[t][v].y, acc[v].y);
        }
    }
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      const int c = c0 + l + v * kSpmmLanes;
      if (c < M) Y[r * ldY + c] = acc[v];
    }
  }
}

template <int VEC>
static hipError_t spmm_go(const mpt_csr& K, const double2* U, int64_t ldU, int M, int c0,
                          double2* Y, int64_t ldY, hipStream_t st) {
  const int64_t rows_per_group = kSpmmRowsPerPass;
  // the caller has checked that row_blocks divides n
  const int nblk = K.row_blocks > 1 ? K.row_blocks : 1;
  const int64_t nrb = K.n / nblk;
  const int64_t groups = nblk * ((nrb + rows_per_group - 1) / rows_per_group);
  hipLaunchKernelGGL((k_spmm<VEC>), dim3((unsigned)groups), dim3(256), 0, st, K.n, K.rowptr,
                     K.colind, K.val, U, ldU, M, c0, Y, ldY, rows_per_group, nblk);
  return hipGetLastError();
}

hipError_t spmm_launch(const mpt_csr& K, const double* U, int64_t ldU, int M, double* Y,
                       int64_t ldY, hipStream_t st) {
  if (K.n <= 0 || M <= 0) return hipSuccess;
  const double2* Uc = reinterpret_cast<const double2*>(U);
  double2* Yc = reinterpret_cast<double2*>(Y);
  // chunks of 24 columns (8 lanes x 3); a narrower last chunk when M allows
  for (int c0 = 0; c0 < M; c0 += 24) {
    const int w = M - c0 < 24 ? M - c0 : 24;
    const int vec = (w + kSpmmLanes - 1) / kSpmmLanes;
    hipError_t e = vec == 1 ? spmm_go<1>(K, Uc, ldU, M, c0, Yc, ldY, st)
                 : vec == 2 ? spmm_go<2>(K, Uc, ldU, M, c0, Yc, ldY, st)
                            : spmm_go<3>(K, Uc, ldU, M, c0, Yc, ldY, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace mpt
