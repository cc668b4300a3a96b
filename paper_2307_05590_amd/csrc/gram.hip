// Dense complex contractions on FP64 MFMA (v_mfma_f64_16x16x4f64):
//   gram:   P = A^H B over N rows (split-N partials + fixed-order reduction)
//   rotate: C = A V  (tall x small)
//   rcgemm: T = S Z  (small real x complex)
// Complex products use four real MFMAs (re.re, im.im, re.im, im.re).
//
// Operand layout of the 16x16x4 f64 MFMA for lane l (0..63):
//   a: A[l % 16][l / 16]   b: B[l / 16][l % 16]
//   d: D[(l / 16) + 4 * v][l % 16], v = 0..3   (checked on gfx950)
#include <type_traits>

#include "device_util.h"
#include "kernels.h"

namespace mpt {

typedef double double4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double4_t mfma(double a, double b, double4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// rows per partial: chosen so that a launch has about a thousand workgroups
// while the partial sums (chunks x m x n) stay small next to the operands
__host__ __device__ inline int64_t gram_rows(int64_t N, int m, int n) {
  const int TI = (m + 15) / 16, TJ = (n + 15) / 16, JG = (TJ + 3) / 4;
  const int64_t groups_per_chunk = (TI * JG + 3) / 4;
  int64_t rows = N * groups_per_chunk / 1024;
  rows = rows < 16 ? 16 : (rows > 8192 ? 8192 : rows);
  return (rows + 3) / 4 * 4;
}

// grid: x = row chunk, y = wave-task group (4 waves per group);
// wave-task t -> tile row I = t / JG, tile column group jg = t % JG (4 tiles)
__global__ __launch_bounds__(256) void k_gram_partial(const double2* __restrict__ A, int64_t lda,
                                                      const double2* __restrict__ B, int64_t ldb,
                                                      int64_t N, int m, int n, int64_t rows,
                                                      int herm, double2* __restrict__ part) {
  const int lane = __lane_id();
  const int TI = (m + 15) / 16, TJ = (n + 15) / 16, JG = (TJ + 3) / 4;
  const int task = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (task >= TI * JG) return;
  const int I = task / JG, jg = task % JG;
  // Hermitian product (A == B): tiles left of the diagonal come from their mirror
  if (herm && jg * 4 + 3 < I) return;
  const int64_t r0 = (int64_t)blockIdx.x * rows;
  const int64_t r1 = min(N, r0 + rows);
  const int ar = I * 16 + (lane & 15);  // column of A feeding this lane
  const bool aok = ar < m;
  double4_t accr[4], acci[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    accr[t] = double4_t{0, 0, 0, 0};
    acci[t] = double4_t{0, 0, 0, 0};
  }
  for (int64_t k0 = r0; k0 < r1; k0 += 4) {
    const int64_t row = k0 + (lane >> 4);
    const bool rok = row < r1;
    const double2 a = (rok && aok) ? A[row * lda + ar] : make_double2(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int J = jg * 4 + t;
      if (J < TJ && !(herm && J < I)) {
        const int bc = J * 16 + (lane & 15);
        const double2 bb = (rok && bc < n) ? B[row * ldb + bc] : make_double2(0.0, 0.0);
        // P = A^H B: re = ar.br + ai.bi ; im = ar.bi - ai.br
        accr[t] = mfma(a.x, bb.x, accr[t]);
        accr[t] = mfma(a.y, bb.y, accr[t]);
        acci[t] = mfma(a.x, bb.y, acci[t]);
        acci[t] = mfma(-a.y, bb.x, acci[t]);
      }
    }
  }
  double2* P = part + (size_t)blockIdx.x * m * n;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int J = jg * 4 + t;
    if (J >= TJ || (herm && J < I)) continue;
    const int col = J * 16 + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int rowo = I * 16 + (lane >> 4) + 4 * v;
      if (rowo < m && col < n) P[(size_t)rowo * n + col] = make_double2(accr[t][v], acci[t][v]);
    }
  }
}

// partial sums: stage 1 sums a slice of the chunks per (entry, slice), stage 2
// sums the slices; both in fixed order (deterministic)
constexpr int kSumSlices = 16;

__global__ void k_sum_partials1(const double2* __restrict__ part, int nparts, int mn,
                                double2* __restrict__ mid) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int sl = blockIdx.y;
  if (idx >= mn) return;
  const int per = (nparts + kSumSlices - 1) / kSumSlices;
  const int p0 = sl * per, p1 = min(nparts, p0 + per);
  double2 s = make_double2(0.0, 0.0);
  for (int p = p0; p < p1; ++p) {
    const double2 v = part[(size_t)p * mn + idx];
    s.x += v.x;
    s.y += v.y;
  }
  mid[(size_t)sl * mn + idx] = s;
}

__global__ void k_sum_partials2(const double2* __restrict__ mid, int mn,
                                double2* __restrict__ P, int n, int64_t ldp, int herm) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= mn) return;
  const int i = idx / n, j = idx % n;
  // mirrored tile of a Hermitian product: conj of the computed (j, i) entry
  const bool mirror = herm && (j / 16) < (i / 16);
  const int src = mirror ? j * n + i : idx;
  double2 s = make_double2(0.0, 0.0);
  for (int sl = 0; sl < kSumSlices; ++sl) {
    const double2 v = mid[(size_t)sl * mn + src];
    s.x += v.x;
    s.y += v.y;
  }
  P[i * ldp + j] = mirror ? make_double2(s.x, -s.y) : s;
}

size_t gram_ws_size(int64_t N, int m, int n) {
  const int64_t rows = gram_rows(N, m, n);
  const int64_t chunks = (N + rows - 1) / rows;
  return (size_t)(chunks + kSumSlices) * m * n * sizeof(double2);
}

hipError_t gram_launch(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t N,
                       int m, int n, double* P, int64_t ldp, void* ws, hipStream_t st) {
  if (m <= 0 || n <= 0) return hipSuccess;
  const int64_t rows = gram_rows(N, m, n);
  const int64_t chunks = N > 0 ? (N + rows - 1) / rows : 0;
  const int TI = (m + 15) / 16, TJ = (n + 15) / 16, JG = (TJ + 3) / 4;
  const int tasks = TI * JG;
  double2* part = reinterpret_cast<double2*>(ws);
  double2* mid = part + (size_t)chunks * m * n;
  const int herm = (A == B && lda == ldb && m == n) ? 1 : 0;
  if (chunks > 0) {
    hipLaunchKernelGGL(k_gram_partial, dim3((unsigned)chunks, (tasks + 3) / 4), dim3(256), 0, st,
                       reinterpret_cast<const double2*>(A), lda,
                       reinterpret_cast<const double2*>(B), ldb, N, m, n, rows, herm, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int mn = m * n;
  hipLaunchKernelGGL(k_sum_partials1, dim3((mn + 255) / 256, kSumSlices), dim3(256), 0, st, part,
                     (int)chunks, mn, mid);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_partials2, dim3((mn + 255) / 256), dim3(256), 0, st, mid, mn,
                     reinterpret_cast<double2*>(P), n, ldp, herm);
  return hipGetLastError();
}

// C (N x n) = A (N x m) V (m x n); one wave per (16-row tile, group of 4
// column tiles)
__global__ __launch_bounds__(256) void k_rotate(const double2* __restrict__ A, int64_t lda,
                                                int64_t N, int m, const double2* __restrict__ V,
                                                int64_t ldv, int n, double2* __restrict__ C,
                                                int64_t ldc) {
  const int lane = __lane_id();
  const int TJ = (n + 15) / 16, JG = (TJ + 3) / 4;
  const int64_t task = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t RT = (N + 15) / 16;
  if (task >= RT * JG) return;
  const int64_t rt = task / JG;
  const int jg = (int)(task % JG);
  const int64_t row = rt * 16 + (lane & 15);
  const bool rok = row < N;
  double4_t accr[4], acci[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    accr[t] = double4_t{0, 0, 0, 0};
    acci[t] = double4_t{0, 0, 0, 0};
  }
  for (int k0 = 0; k0 < m; k0 += 4) {
    const int k = k0 + (lane >> 4);
    const double2 a = (rok && k < m) ? A[row * lda + k] : make_double2(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int J = jg * 4 + t;
      if (J < TJ) {
        const int col = J * 16 + (lane & 15);
        const double2 v = (k < m && col < n) ? V[(int64_t)k * ldv + col] : make_double2(0.0, 0.0);
        accr[t] = mfma(a.x, v.x, accr[t]);
        accr[t] = mfma(-a.y, v.y, accr[t]);
        acci[t] = mfma(a.x, v.y, acci[t]);
        acci[t] = mfma(a.y, v.x, acci[t]);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int J = jg * 4 + t;
    if (J >= TJ) continue;
    const int col = J * 16 + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t r = rt * 16 + (lane >> 4) + 4 * v;
      if (r < N && col < n) C[r * ldc + col] = make_double2(accr[t][v], acci[t][v]);
    }
  }
}

hipError_t rotate_launch(const double* A, int64_t lda, int64_t N, int m, const double* V,
                         int64_t ldv, int n, double* C, int64_t ldc, hipStream_t st) {
  if (N <= 0 || n <= 0) return hipSuccess;
  const int TJ = (n + 15) / 16, JG = (TJ + 3) / 4;
  const int64_t tasks = ((N + 15) / 16) * JG;
  hipLaunchKernelGGL(k_rotate, dim3((unsigned)((tasks + 3) / 4)), dim3(256), 0, st,
                     reinterpret_cast<const double2*>(A), lda, N, m,
                     reinterpret_cast<const double2*>(V), ldv, n, reinterpret_cast<double2*>(C),
                     ldc);
  return hipGetLastError();
}

// T (r x n) = S (r x r real, row-major) Z (r x n complex), split over the
// reduction index in chunks of kRcK (grid.y) with a fixed-order final sum
constexpr int kRcK = 128;

__global__ __launch_bounds__(256) void k_rcgemm(const double* __restrict__ S, int64_t r,
                                                const double2* __restrict__ Z, int n,
                                                double2* __restrict__ part) {
  const int lane = __lane_id();
  const int TJ = (n + 15) / 16, JG = (TJ + 3) / 4;
  const int64_t task = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t RT = (r + 15) / 16;
  if (task >= RT * JG) return;
  const int64_t rt = task / JG;
  const int jg = (int)(task % JG);
  const int64_t row = rt * 16 + (lane & 15);
  const bool rok = row < r;
  const int64_t kb = (int64_t)blockIdx.y * kRcK, ke = min(r, kb + kRcK);
  double4_t accr[4], acci[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    accr[t] = double4_t{0, 0, 0, 0};
    acci[t] = double4_t{0, 0, 0, 0};
  }
  for (int64_t k0 = kb; k0 < ke; k0 += 4) {
    const int64_t k = k0 + (lane >> 4);
    const bool kok = k < ke;
    const double s = (rok && kok) ? S[row * r + k] : 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int J = jg * 4 + t;
      if (J < TJ) {
        const int col = J * 16 + (lane & 15);
        const double2 z = (kok && col < n) ? Z[k * n + col] : make_double2(0.0, 0.0);
        accr[t] = mfma(s, z.x, accr[t]);
        acci[t] = mfma(s, z.y, acci[t]);
      }
    }
  }
  double2* T = part + (size_t)blockIdx.y * r * n;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int J = jg * 4 + t;
    if (J >= TJ) continue;
    const int col = J * 16 + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t rr = rt * 16 + (lane >> 4) + 4 * v;
      if (rr < r && col < n) T[rr * n + col] = make_double2(accr[t][v], acci[t][v]);
    }
  }
}

__global__ void k_rc_sum(const double2* __restrict__ part, int nk, int64_t cnt,
                         double2* __restrict__ T) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  double2 s = make_double2(0.0, 0.0);
  for (int y = 0; y < nk; ++y) {
    const double2 v = part[(size_t)y * cnt + i];
    s.x += v.x;
    s.y += v.y;
  }
  T[i] = s;
}

size_t rcgemm_ws_size(int64_t r, int n) {
  const int64_t nk = (r + kRcK - 1) / kRcK;
  return (size_t)nk * r * n * sizeof(double2);
}

hipError_t real_complex_gemm(const double* S, int64_t r, const double* Z, int n, double* T,
                             void* ws, hipStream_t st) {
  if (r <= 0 || n <= 0) return hipSuccess;
  const int TJ = (n + 15) / 16, JG = (TJ + 3) / 4;
  const int64_t tasks = ((r + 15) / 16) * JG;
  const int nk = (int)((r + kRcK - 1) / kRcK);
  double2* part = reinterpret_cast<double2*>(ws);
  hipLaunchKernelGGL(k_rcgemm, dim3((unsigned)((tasks + 3) / 4), nk), dim3(256), 0, st, S, r,
                     reinterpret_cast<const double2*>(Z), n, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t cnt = r * n;
  hipLaunchKernelGGL(k_rc_sum, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, part, nk,
                     cnt, reinterpret_cast<double2*>(T));
  return hipGetLastError();
}

}  // namespace mpt
