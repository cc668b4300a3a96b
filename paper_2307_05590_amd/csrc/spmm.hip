// Y = K U: real CSR (curl-curl, ~12.6 nonzeros per row) times a complex
// tall-skinny basis (N x M, row-major).  HBM-bound: every nonzero gathers one
// 16 M-byte row of U; rows of U are contiguous so a group of lanes reads a
// whole row with coalesced 16-byte loads.  A wave handles several output rows;
// lanes map to the M complex columns.  Workgroups are mapped XCD-aware: the
// 8 XCDs receive contiguous row ranges so neighbouring gathers share an L2.
#include "device_util.h"
#include "kernels.h"

namespace mpt {

// LPR lanes per output row (power of two >= M/VEC), VEC complex columns per lane
template <int LPR>
__global__ __launch_bounds__(256) void k_spmm(int64_t n, const int32_t* __restrict__ rowptr,
                                              const int32_t* __restrict__ colind,
                                              const double* __restrict__ val,
                                              const double2* __restrict__ U, int64_t ldU, int M,
                                              double2* __restrict__ Y, int64_t ldY,
                                              int64_t rows_per_group) {
  // XCD-aware remap: consecutive block ids go round-robin over 8 XCDs; give
  // each XCD a contiguous slice of the block range.
  const int64_t nb = gridDim.x;
  const int64_t b = blockIdx.x;
  const int64_t q = nb / 8, rem = nb % 8;
  const int64_t xcd = b % 8, slot = b / 8;
  // XCD x owns q (+1 when x < rem) consecutive logical blocks
  const int64_t lb = xcd * q + min(xcd, rem) + slot;
  const int sub = threadIdx.x / LPR;  // row within the group
  const int l = threadIdx.x % LPR;    // lane within the row
  constexpr int RPG = 256 / LPR;
  for (int64_t r = lb * rows_per_group + sub; r < min(n, (lb + 1) * rows_per_group); r += RPG) {
    const int e0 = rowptr[r], e1 = rowptr[r + 1];
    for (int c0 = 0; c0 < M; c0 += LPR) {
      const int c = c0 + l;
      double2 acc = make_double2(0.0, 0.0);
      if (c < M) {
        int e = e0;
        for (; e + 3 < e1; e += 4) {
          const int j0 = colind[e], j1 = colind[e + 1], j2 = colind[e + 2], j3 = colind[e + 3];
          const double v0 = val[e], v1 = val[e + 1], v2 = val[e + 2], v3 = val[e + 3];
          const double2 u0 = U[(int64_t)j0 * ldU + c];
          const double2 u1 = U[(int64_t)j1 * ldU + c];
          const double2 u2 = U[(int64_t)j2 * ldU + c];
          const double2 u3 = U[(int64_t)j3 * ldU + c];
          acc.x = fma(v0, u0.x, acc.x); acc.y = fma(v0, u0.y, acc.y);
          acc.x = fma(v1, u1.x, acc.x); acc.y = fma(v1, u1.y, acc.y);
          acc.x = fma(v2, u2.x, acc.x); acc.y = fma(v2, u2.y, acc.y);
          acc.x = fma(v3, u3.x, acc.x); acc.y = fma(v3, u3.y, acc.y);
        }
        for (; e < e1; ++e) {
          const double v = val[e];
          const double2 u = U[(int64_t)colind[e] * ldU + c];
          acc.x = fma(v, u.x, acc.x);
          acc.y = fma(v, u.y, acc.y);
        }
        Y[r * ldY + c] = acc;
      }
    }
  }
}

hipError_t spmm_launch(const mpt_csr& K, const double* U, int64_t ldU, int M, double* Y,
                       int64_t ldY, hipStream_t st) {
  if (K.n <= 0 || M <= 0) return hipSuccess;
  const double2* Uc = reinterpret_cast<const double2*>(U);
  double2* Yc = reinterpret_cast<double2*>(Y);
  // rows per workgroup: aim for several thousand groups
  auto go = [&](auto lpr_tag) -> hipError_t {
    constexpr int LPR = decltype(lpr_tag)::value;
    constexpr int RPG = 256 / LPR;
    const int64_t rows_per_group = RPG * 4;
    const int64_t groups = (K.n + rows_per_group - 1) / rows_per_group;
    hipLaunchKernelGGL((k_spmm<LPR>), dim3((unsigned)groups), dim3(256), 0, st, K.n, K.rowptr,
                       K.colind, K.val, Uc, ldU, M, Yc, ldY, rows_per_group);
    return hipGetLastError();
  };
  if (M <= 8) return go(std::integral_constant<int, 8>{});
  if (M <= 16) return go(std::integral_constant<int, 16>{});
  if (M <= 32) return go(std::integral_constant<int, 32>{});
  return go(std::integral_constant<int, 64>{});
}

}  // namespace mpt
