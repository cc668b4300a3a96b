// Y = K U: real CSR (curl-curl, ~12.6 nonzeros per row) times a complex
// tall-skinny basis (N x M, row-major).  HBM/L2-bandwidth bound: every
// nonzero gathers one 16 M-byte row of U.  Sixteen lanes share an output row,
// each owning VEC = ceil(M/16) complex columns, so a wave keeps the dependent
// load chains (row pointer -> column index -> U row) of four rows in flight
// and every gathered U row is read with coalesced 16-byte loads.  Workgroups
// are mapped XCD-aware: each of the 8 XCDs receives a contiguous range of rows
// so that the stencil neighbours of its rows share that XCD's L2.
#include "device_util.h"
#include "kernels.h"

namespace mpt {

constexpr int kSpmmLanes = 16;                     // lanes per output row
constexpr int kSpmmRowsPerGroup = 256 / kSpmmLanes;  // rows in flight per workgroup

template <int VEC>
__global__ __launch_bounds__(256) void k_spmm(int64_t n, const int32_t* __restrict__ rowptr,
                                              const int32_t* __restrict__ colind,
                                              const double* __restrict__ val,
                                              const double2* __restrict__ U, int64_t ldU, int M,
                                              double2* __restrict__ Y, int64_t ldY,
                                              int64_t rows_per_group) {
  const int64_t nb = gridDim.x;
  const int64_t b = blockIdx.x;
  const int64_t q = nb / 8, rem = nb % 8;
  const int64_t xcd = b % 8, slot = b / 8;
  // XCD x owns q (+1 when x < rem) consecutive logical blocks
  const int64_t lb = xcd * q + min(xcd, rem) + slot;
  const int sub = threadIdx.x / kSpmmLanes;
  const int l = threadIdx.x % kSpmmLanes;
  const int64_t rend = min(n, (lb + 1) * rows_per_group);
  for (int64_t r = lb * rows_per_group + sub; r < rend; r += kSpmmRowsPerGroup) {
    const int e0 = rowptr[r], e1 = rowptr[r + 1];
    double2 acc[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] = make_double2(0.0, 0.0);
    int e = e0;
    for (; e + 1 < e1; e += 2) {
      const int j0 = colind[e], j1 = colind[e + 1];
      const double v0 = val[e], v1 = val[e + 1];
      const double2* u0 = U + (int64_t)j0 * ldU;
      const double2* u1 = U + (int64_t)j1 * ldU;
      double2 a0[VEC], a1[VEC];
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        const int c = l + v * kSpmmLanes;
        a0[v] = c < M ? u0[c] : make_double2(0.0, 0.0);
        a1[v] = c < M ? u1[c] : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        acc[v].x = fma(v0, a0[v].x, acc[v].x);
        acc[v].y = fma(v0, a0[v].y, acc[v].y);
        acc[v].x = fma(v1, a1[v].x, acc[v].x);
        acc[v].y = fma(v1, a1[v].y, acc[v].y);
      }
    }
    if (e < e1) {
      const double v0 = val[e];
      const double2* u0 = U + (int64_t)colind[e] * ldU;
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        const int c = l + v * kSpmmLanes;
        if (c < M) {
          const double2 a = u0[c];
          acc[v].x = fma(v0, a.x, acc[v].x);
          acc[v].y = fma(v0, a.y, acc[v].y);
        }
      }
    }
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      const int c = l + v * kSpmmLanes;
      if (c < M) Y[r * ldY + c] = acc[v];
    }
  }
}

template <int VEC>
static hipError_t spmm_go(const mpt_csr& K, const double2* U, int64_t ldU, int M, double2* Y,
                          int64_t ldY, hipStream_t st) {
  const int64_t rows_per_group = kSpmmRowsPerGroup * 2;
  const int64_t groups = (K.n + rows_per_group - 1) / rows_per_group;
  hipLaunchKernelGGL((k_spmm<VEC>), dim3((unsigned)groups), dim3(256), 0, st, K.n, K.rowptr,
                     K.colind, K.val, U, ldU, M, Y, ldY, rows_per_group);
  return hipGetLastError();
}

hipError_t spmm_launch(const mpt_csr& K, const double* U, int64_t ldU, int M, double* Y,
                       int64_t ldY, hipStream_t st) {
  if (K.n <= 0 || M <= 0) return hipSuccess;
  const double2* Uc = reinterpret_cast<const double2*>(U);
  double2* Yc = reinterpret_cast<double2*>(Y);
  const int vec = (M + kSpmmLanes - 1) / kSpmmLanes;
  switch (vec) {
    case 1: return spmm_go<1>(K, Uc, ldU, M, Yc, ldY, st);
    case 2: return spmm_go<2>(K, Uc, ldU, M, Yc, ldY, st);
    case 3: return spmm_go<3>(K, Uc, ldU, M, Yc, ldY, st);
    case 4: return spmm_go<4>(K, Uc, ldU, M, Yc, ldY, st);
    case 5: return spmm_go<5>(K, Uc, ldU, M, Yc, ldY, st);
    case 6: return spmm_go<6>(K, Uc, ldU, M, Yc, ldY, st);
    case 7: return spmm_go<7>(K, Uc, ldU, M, Yc, ldY, st);
    case 8: return spmm_go<8>(K, Uc, ldU, M, Yc, ldY, st);
    default: {
      // wide bases: process 128 columns at a time
      for (int c0 = 0; c0 < M; c0 += 128) {
        const int m = M - c0 < 128 ? M - c0 : 128;
        hipError_t e = spmm_launch(K, reinterpret_cast<const double*>(Uc + c0), ldU, m,
                                   reinterpret_cast<double*>(Yc + c0), ldY, st);
        if (e != hipSuccess) return e;
      }
      return hipSuccess;
    }
  }
}

}  // namespace mpt
