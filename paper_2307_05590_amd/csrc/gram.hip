// Dense complex contractions on FP64 MFMA (v_mfma_f64_16x16x4f64):
//   gram:   P = A^H B over N rows (split-N partials + fixed-order reduction)
//   rotate: C = A V  (tall x small)
//   rcgemm: T = S Z  (small real x complex)
// Complex products use four real MFMAs (re.re, im.im, re.im, im.re).  The
// same four give A^H conj(B) too, so a pass can return both.
//
// Operand layout of the 16x16x4 f64 MFMA for lane l (0..63):
//   a: A[l % 16][l / 16]   b: B[l / 16][l % 16]
//   d: D[(l / 16) + 4 * v][l % 16], v = 0..3   (checked on gfx950)
#include <type_traits>

#include "device_util.h"
#include "kernels.h"

namespace mpt {

// ---------------------------------------------------------------- Gram
// One workgroup owns every output tile of its chunk of rows, so each row is
// read from HBM once and shared by the waves through L1/L2.  The tiles (16x16)
// of up to two products - P1 = A^H B (all tiles, or I <= J when A == B) and
// P2 = A^H A (I <= J) - are grouped in register blocks of RI x RJ tiles; a
// wave works one block at a time: per step of four rows it loads RI + RJ
// fragments (clamped, branch-free) and issues 4 RI RJ MFMAs.  Blocks of a
// Hermitian product that lie entirely below the diagonal are skipped; the
// partial sums of every chunk are reduced in a fixed order (deterministic).
// With 2 x 2 blocks (the POD's large Hermitian Grams) a complex product takes
// three real MFMAs instead of four (Gauss: P1 = ar br, P2 = ai bi,
// P3 = (ar - ai)(br + bi); re = P1 + P2, im = P3 - P1 + P2), on 12 waves.
constexpr int kGramMaxChunks = 512;

struct GramPlan {
  int TI, TJ, RI, RJ, nb1, nb2, waves;
  bool herm1;
  int64_t chunks, rows;
};

// blocks of a TI x TJ tile grid in RI x RJ blocks; herm: only blocks holding
// a tile with I <= J
__host__ __device__ inline int gram_blocks(int TI, int TJ, int RI, int RJ, bool herm) {
  const int BI = (TI + RI - 1) / RI, BJ = (TJ + RJ - 1) / RJ;
  int c = 0;
  for (int bi = 0; bi < BI; ++bi)
    for (int bj = 0; bj < BJ; ++bj)
      if (!herm || bi * RI <= min(TJ - 1, bj * RJ + RJ - 1)) ++c;
  return c;
}
__device__ inline void gram_block_of(int b, int TI, int TJ, int RI, int RJ, bool herm, int& bi,
                                     int& bj) {
  const int BI = (TI + RI - 1) / RI, BJ = (TJ + RJ - 1) / RJ;
  for (bi = 0; bi < BI; ++bi)
    for (bj = 0; bj < BJ; ++bj)
      if (!herm || bi * RI <= min(TJ - 1, bj * RJ + RJ - 1)) {
        if (b == 0) return;
        --b;
      }
}

static GramPlan gram_plan(int64_t N, int m, int n, bool herm1, bool dual) {
  GramPlan g;
  g.TI = (m + 15) / 16;
  g.TJ = (n + 15) / 16;
  g.herm1 = herm1;
  if (g.TI <= 3 && g.TJ <= 3) {
    g.RI = 1;
    g.RJ = dual ? 3 : g.TJ;
  } else {
    g.RI = 2;
    g.RJ = 2;
  }
  g.nb1 = gram_blocks(g.TI, g.TJ, g.RI, g.RJ, herm1);
  g.nb2 = dual ? gram_blocks(g.TI, g.TI, g.RI, g.RJ, true) : 0;
  const int nb = g.nb1 + g.nb2;
  g.waves = nb < 16 ? nb : 16;  // one block per wave where possible
  int64_t ch = (N + 15) / 16;
  if (ch > kGramMaxChunks) ch = kGramMaxChunks;
  if (ch < 1) ch = 1;
  g.rows = ((N + ch - 1) / ch + 3) / 4 * 4;
  g.chunks = N > 0 ? (N + g.rows - 1) / g.rows : 0;
  return g;
}

template <int RI, int RJ, bool G3, bool CJ>
__global__ __launch_bounds__(G3 ? 768 : (CJ ? 512 : 1024)) void k_gram_chunk(
    const double2* __restrict__ A, int64_t lda, const double2* __restrict__ B, int64_t ldb,
    int64_t N, int m, int n, int64_t rows, int flags1, int nb1, int nb2,
    double2* __restrict__ part1, double2* __restrict__ part2, double2* __restrict__ part1c,
    double2* __restrict__ part2c) {
  static_assert(!(G3 && CJ), "one product form at a time");
  const int lane = __lane_id();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), nw = blockDim.x >> 6;
  const int TI = (m + 15) / 16, TJ = (n + 15) / 16;
  const int64_t r0 = (int64_t)blockIdx.x * rows;
  const int64_t r1 = min(N, r0 + rows);
  const int cl = lane & 15;
  const double2 z2 = make_double2(0.0, 0.0);
  for (int bk = wave; bk < nb1 + nb2; bk += nw) {
    const bool second = bk >= nb1;  // wave-uniform
    // flags1: bit 0 the first product is Hermitian (blocks below the diagonal
    // skipped), bit 1 its B is A
    const bool self = second || (flags1 & 2);
    const int ncol = second ? m : n;
    const int tj = second ? TI : TJ;
    int bi, bj;
    gram_block_of(second ? bk - nb1 : bk, TI, tj, RI, RJ, second || (flags1 & 1), bi, bj);
    int ca[RI], cb[RJ];
    bool va[RI], vb[RJ];
#pragma unroll
    for (int r = 0; r < RI; ++r) {
      const int c = (bi * RI + r) * 16 + cl;
      va[r] = c < m;
      ca[r] = va[r] ? c : m - 1;
    }
#pragma unroll
    for (int q = 0; q < RJ; ++q) {
      const int c = (bj * RJ + q) * 16 + cl;
      vb[q] = c < ncol;
      cb[q] = vb[q] ? c : ncol - 1;
    }
    const double2* Bs = self ? A : B;
    const int64_t ldbs = self ? lda : ldb;
    // G3: three real products per complex one (P1 = ar br, P2 = ai bi,
    // P3 = (ar - ai)(br + bi); re = P1 + P2, im = P3 - P1 + P2).
    // CJ: the four real products kept apart (ar br, ai bi, ar bi, ai br), which
    // give both A^H B and A^H conj(B) from the same MFMAs.
    constexpr int R3 = (G3 || CJ) ? RI : 1, C3 = (G3 || CJ) ? RJ : 1;
    constexpr int R4 = CJ ? RI : 1, C4 = CJ ? RJ : 1;
    double4_t accr[RI][RJ], acci[RI][RJ], acc3[R3][C3], acc4[R4][C4];
#pragma unroll
    for (int r = 0; r < RI; ++r)
#pragma unroll
      for (int q = 0; q < RJ; ++q) {
        accr[r][q] = double4_t{0, 0, 0, 0};
        acci[r][q] = double4_t{0, 0, 0, 0};
        if (G3 || CJ) acc3[r % R3][q % C3] = double4_t{0, 0, 0, 0};
        if (CJ) acc4[r % R4][q % C4] = double4_t{0, 0, 0, 0};
      }
    for (int64_t k0 = r0; k0 < r1; k0 += 4) {
      const int64_t row = k0 + (lane >> 4);
      const bool rok = row < r1;
      const int64_t rowc = rok ? row : r1 - 1;
      double2 fa[RI], fb[RJ];
#pragma unroll
      for (int r = 0; r < RI; ++r) {
        const double2 x = A[rowc * lda + ca[r]];
        fa[r] = (rok && va[r]) ? x : z2;
      }
#pragma unroll
      for (int q = 0; q < RJ; ++q) {
        const double2 y = Bs[rowc * ldbs + cb[q]];
        fb[q] = (rok && vb[q]) ? y : z2;
      }
#pragma unroll
      for (int r = 0; r < RI; ++r)
#pragma unroll
        for (int q = 0; q < RJ; ++q) {
          if (G3) {
            accr[r][q] = mfma(fa[r].x, fb[q].x, accr[r][q]);  // P1
            acci[r][q] = mfma(fa[r].y, fb[q].y, acci[r][q]);  // P2
            acc3[r % R3][q % C3] = mfma(fa[r].x - fa[r].y, fb[q].x + fb[q].y, acc3[r % R3][q % C3]);
          } else if (CJ) {
            accr[r][q] = mfma(fa[r].x, fb[q].x, accr[r][q]);
            acci[r][q] = mfma(fa[r].y, fb[q].y, acci[r][q]);
            acc3[r % R3][q % C3] = mfma(fa[r].x, fb[q].y, acc3[r % R3][q % C3]);
            acc4[r % R4][q % C4] = mfma(fa[r].y, fb[q].x, acc4[r % R4][q % C4]);
          } else {
            // conj(a) * b: re = ar br + ai bi, im = ar bi - ai br
            accr[r][q] = mfma(fa[r].x, fb[q].x, accr[r][q]);
            accr[r][q] = mfma(fa[r].y, fb[q].y, accr[r][q]);
            acci[r][q] = mfma(fa[r].x, fb[q].y, acci[r][q]);
            acci[r][q] = mfma(-fa[r].y, fb[q].x, acci[r][q]);
          }
        }
    }
    if (G3) {
#pragma unroll
      for (int r = 0; r < RI; ++r)
#pragma unroll
        for (int q = 0; q < RJ; ++q) {
          const double4_t p1 = accr[r][q], p2 = acci[r][q], p3 = acc3[r % R3][q % C3];
          accr[r][q] = p1 + p2;
          acci[r][q] = (p3 - p1) + p2;
        }
    }
    const size_t poff = second ? (size_t)blockIdx.x * m * m : (size_t)blockIdx.x * m * n;
    if (CJ) {  // A^H conj(B): re = ar br - ai bi, im = -(ar bi + ai br)
      double2* Q = (second ? part2c : part1c) + poff;
#pragma unroll
      for (int r = 0; r < RI; ++r)
#pragma unroll
        for (int q = 0; q < RJ; ++q) {
          const int I = bi * RI + r, J = bj * RJ + q;
          if (I >= TI || J >= tj) continue;
          const int col = J * 16 + cl;
          const double4_t qr = accr[r][q] - acci[r][q];
          const double4_t qi = -(acc3[r % R3][q % C3] + acc4[r % R4][q % C4]);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int rowo = I * 16 + (lane >> 4) + 4 * v;
            if (rowo < m && col < ncol) Q[(size_t)rowo * ncol + col] = make_double2(qr[v], qi[v]);
          }
        }
#pragma unroll
      for (int r = 0; r < RI; ++r)
#pragma unroll
        for (int q = 0; q < RJ; ++q) {  // A^H B: re = ar br + ai bi, im = ar bi - ai br
          const double4_t p1 = accr[r][q], p2 = acci[r][q];
          accr[r][q] = p1 + p2;
          acci[r][q] = acc3[r % R3][q % C3] - acc4[r % R4][q % C4];
        }
    }
    double2* P = (second ? part2 : part1) + poff;
#pragma unroll
    for (int r = 0; r < RI; ++r)
#pragma unroll
      for (int q = 0; q < RJ; ++q) {
        const int I = bi * RI + r, J = bj * RJ + q;
        if (I >= TI || J >= tj) continue;
        const int col = J * 16 + cl;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int rowo = I * 16 + (lane >> 4) + 4 * v;
          if (rowo < m && col < ncol)
            P[(size_t)rowo * ncol + col] = make_double2(accr[r][q][v], acci[r][q][v]);
        }
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

// mirror: 0 every tile computed; 1 Hermitian (tiles below the diagonal are
// the conjugate of the computed (j, i) entry); 2 complex symmetric (its plain
// transpose)
__global__ void k_sum_partials2(const double2* __restrict__ mid, int mn,
                                double2* __restrict__ P, int n, int64_t ldp, int herm) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= mn) return;
  const int i = idx / n, j = idx % n;
  const bool mirror = herm && (j / 16) < (i / 16);
  const int src = mirror ? j * n + i : idx;
  double2 s = make_double2(0.0, 0.0);
  for (int sl = 0; sl < kSumSlices; ++sl) {
    const double2 v = mid[(size_t)sl * mn + src];
    s.x += v.x;
    s.y += v.y;
  }
  P[i * ldp + j] = (mirror && herm == 1) ? make_double2(s.x, -s.y) : s;
}

size_t gram_ws_size(int64_t N, int m, int n) {
  // room for the dual form (P1 m x n and P2 m x m) at the largest chunk count
  const GramPlan g = gram_plan(N, m, n, false, true);
  const size_t mn = (size_t)m * n, mm = (size_t)m * m;
  return ((size_t)g.chunks * (mn + mm) + kSumSlices * (mn > mm ? mn : mm)) * sizeof(double2);
}

size_t gram2c_ws_size(int64_t N, int m, int n) {
  // the dual form and its conjugate-B companions
  const GramPlan g = gram_plan(N, m, n, false, true);
  const size_t mn = (size_t)m * n, mm = (size_t)m * m;
  return ((size_t)g.chunks * (mn + mm) * 2 + kSumSlices * (mn > mm ? mn : mm)) * sizeof(double2);
}

static hipError_t gram_reduce(const double2* part, int64_t chunks, int m, int n, double* P,
                              int64_t ldp, int herm, double2* mid, hipStream_t st) {
  const int mn = m * n;
  hipLaunchKernelGGL(k_sum_partials1, dim3((mn + 255) / 256, kSumSlices), dim3(256), 0, st, part,
                     (int)chunks, mn, mid);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_partials2, dim3((mn + 255) / 256), dim3(256), 0, st, mid, mn,
                     reinterpret_cast<double2*>(P), n, ldp, herm);
  return hipGetLastError();
}

// P1 = A^H B, optionally P2 = A^H A (dual), and with Q1 the companions
// Q1 = A^H conj(B), Q2 = A^H conj(A) from the same MFMAs
static hipError_t gram_run(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t N,
                           int m, int n, double* P1, int64_t ldp1, double* P2, int64_t ldp2,
                           double* Q1, int64_t ldq1, double* Q2, int64_t ldq2, bool herm_ab,
                           void* ws, hipStream_t st) {
  if (m <= 0 || n <= 0) return hipSuccess;
  const bool same = (A == B && lda == ldb && m == n);
  const bool herm1 = same || (herm_ab && m == n);
  const int flags1 = (herm1 ? 1 : 0) | (same ? 2 : 0);
  const bool dual = P2 != nullptr;
  const bool cj = Q1 != nullptr;
  const GramPlan g = gram_plan(N, m, n, herm1, dual);
  double2* part1 = reinterpret_cast<double2*>(ws);
  double2* part2 = part1 + (size_t)g.chunks * m * n;
  double2* part1c = part2 + (dual ? (size_t)g.chunks * m * m : 0);
  double2* part2c = part1c + (cj ? (size_t)g.chunks * m * n : 0);
  double2* mid = part2c + (cj && dual ? (size_t)g.chunks * m * m : 0);
  if (g.chunks > 0) {
    const dim3 grid((unsigned)g.chunks), block(64 * g.waves);
    const double2* Ac = reinterpret_cast<const double2*>(A);
    const double2* Bc = reinterpret_cast<const double2*>(B);
    // the 2 x 2 blocks (the large Hermitian Grams) use three real products
    // per complex one, on 12 waves (their accumulators need 128 registers);
    // the conjugate companions keep four accumulators, on at most 8 waves
    const dim3 grid3((unsigned)g.chunks), block3(64 * (g.waves < 12 ? g.waves : 12));
    const dim3 blockc(64 * (g.waves < 8 ? g.waves : 8));
#define MPT_GC3(RI, RJ)                                                                      \
  hipLaunchKernelGGL((k_gram_chunk<RI, RJ, true, false>), grid3, block3, 0, st, Ac, lda, Bc, ldb, \
                     N, m, n, g.rows, flags1, g.nb1, g.nb2, part1, part2, part1c, part2c)
#define MPT_GC(RI, RJ)                                                                        \
  hipLaunchKernelGGL((k_gram_chunk<RI, RJ, false, false>), grid, block, 0, st, Ac, lda, Bc, ldb, \
                     N, m, n, g.rows, flags1, g.nb1, g.nb2, part1, part2, part1c, part2c)
#define MPT_GCC(RI, RJ)                                                                       \
  hipLaunchKernelGGL((k_gram_chunk<RI, RJ, false, true>), grid, blockc, 0, st, Ac, lda, Bc, ldb, \
                     N, m, n, g.rows, flags1, g.nb1, g.nb2, part1, part2, part1c, part2c)
    if (cj) {
      if (g.RI == 2) MPT_GCC(2, 2);
      else if (g.RJ == 3) MPT_GCC(1, 3);
      else if (g.RJ == 2) MPT_GCC(1, 2);
      else MPT_GCC(1, 1);
    } else {
      if (g.RI == 2) MPT_GC3(2, 2);
      else if (g.RJ == 3) MPT_GC(1, 3);
      else if (g.RJ == 2) MPT_GC(1, 2);
      else MPT_GC(1, 1);
    }
#undef MPT_GC
#undef MPT_GC3
#undef MPT_GCC
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  } else {
    hipError_t e = hipMemsetAsync(part1, 0, (size_t)m * n * sizeof(double2), st);
    if (e == hipSuccess && dual) e = hipMemsetAsync(part2, 0, (size_t)m * m * sizeof(double2), st);
    if (e == hipSuccess && cj) e = hipMemsetAsync(part1c, 0, (size_t)m * n * sizeof(double2), st);
    if (e == hipSuccess && cj && dual)
      e = hipMemsetAsync(part2c, 0, (size_t)m * m * sizeof(double2), st);
    if (e != hipSuccess) return e;
  }
  const int64_t ch = g.chunks > 0 ? g.chunks : 1;
  hipError_t e = gram_reduce(part1, ch, m, n, P1, ldp1, herm1 ? 1 : 0, mid, st);
  if (e == hipSuccess && cj) e = gram_reduce(part1c, ch, m, n, Q1, ldq1, herm1 ? 2 : 0, mid, st);
  if (e != hipSuccess || !dual) return e;
  e = gram_reduce(part2, ch, m, m, P2, ldp2, 1, mid, st);
  if (e == hipSuccess && cj && Q2) e = gram_reduce(part2c, ch, m, m, Q2, ldq2, 2, mid, st);
  return e;
}

hipError_t gram2_launch(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t N,
                        int m, int n, double* P1, int64_t ldp1, double* P2, int64_t ldp2,
                        void* ws, hipStream_t st) {
  return gram_run(A, lda, B, ldb, N, m, n, P1, ldp1, P2, ldp2, nullptr, 0, nullptr, 0, false, ws,
                  st);
}

hipError_t gram2c_launch(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t N,
                         int m, int n, double* P1, int64_t ldp1, double* P2, int64_t ldp2,
                         double* Q1, int64_t ldq1, double* Q2, int64_t ldq2, bool herm_ab,
                         void* ws, hipStream_t st) {
  return gram_run(A, lda, B, ldb, N, m, n, P1, ldp1, P2, ldp2, Q1, ldq1, Q2, ldq2, herm_ab, ws,
                  st);
}

hipError_t gram_launch(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t N,
                       int m, int n, double* P, int64_t ldp, void* ws, hipStream_t st) {
  return gram2_launch(A, lda, B, ldb, N, m, n, P, ldp, nullptr, 0, ws, st);
}

// ------------------------------------------------------------- rotation
// C (N x n) = A (N x m) V (m x n).  A wave owns RT row tiles x CT column tiles
// (register blocking: RT + CT fragment loads feed 4 RT CT MFMAs per k step);
// the waves sharing a row block are adjacent, so A rows are reused in L1/L2.
template <int RT, int CT>
__global__ __launch_bounds__(256) void k_rotate(const double2* __restrict__ A, int64_t lda,
                                                int64_t N, int m, const double2* __restrict__ V,
                                                int64_t ldv, int n, double2* __restrict__ C,
                                                int64_t ldc, int nw) {
  // nw >= n: columns n .. nw-1 of C are written as zeros
  const int lane = __lane_id();
  const int TJ = (nw + 15) / 16, CG = (TJ + CT - 1) / CT;
  const int64_t task = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t RB = (N + 16 * RT - 1) / (16 * RT);
  if (task >= RB * CG) return;
  const int64_t rb = task / CG;
  const int cg = (int)(task % CG);
  const int cl = lane & 15, kl = lane >> 4;
  double4_t accr[RT][CT], acci[RT][CT];
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      accr[r][c] = double4_t{0, 0, 0, 0};
      acci[r][c] = double4_t{0, 0, 0, 0};
    }
  auto load = [&](int k0, double2 (&a)[RT], double2 (&v)[CT]) {
    const int k = k0 + kl;
    const int kc = k < m ? k : m - 1;
    const double2 z2 = make_double2(0.0, 0.0);
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      const int64_t row = rb * 16 * RT + r * 16 + cl;
      const double2 x = A[(row < N ? row : N - 1) * lda + kc];
      a[r] = (row < N && k < m) ? x : z2;
    }
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      const int col = (cg * CT + c) * 16 + cl;
      const double2 x = V[(int64_t)kc * ldv + (col < n ? col : n - 1)];
      v[c] = (k < m && col < n) ? x : z2;
    }
  };
  double2 a[RT], v[CT];
  const bool live = cg * CT * 16 < n;  // wave-uniform: this column group holds columns of V
  if (live) load(0, a, v);
  for (int k0 = 0; live && k0 < m; k0 += 4) {
    double2 na[RT], nv[CT];
    load(k0 + 4, na, nv);  // next step's fragments in flight during the MFMAs
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        accr[r][c] = mfma(a[r].x, v[c].x, accr[r][c]);
        accr[r][c] = mfma(-a[r].y, v[c].y, accr[r][c]);
        acci[r][c] = mfma(a[r].x, v[c].y, acci[r][c]);
        acci[r][c] = mfma(a[r].y, v[c].x, acci[r][c]);
      }
#pragma unroll
    for (int r = 0; r < RT; ++r) a[r] = na[r];
#pragma unroll
    for (int c = 0; c < CT; ++c) v[c] = nv[c];
  }
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      const int col = (cg * CT + c) * 16 + cl;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t row = rb * 16 * RT + r * 16 + kl + 4 * q;
        if (row < N && col < nw) C[row * ldc + col] = make_double2(accr[r][c][q], acci[r][c][q]);
      }
    }
}

hipError_t rotate_launch(const double* A, int64_t lda, int64_t N, int m, const double* V,
                         int64_t ldv, int n, double* C, int64_t ldc, hipStream_t st, int n_zero) {
  const int nw = n_zero > n ? n_zero : n;
  if (N <= 0 || nw <= 0) return hipSuccess;
  constexpr int RT = 2, CT = 3;
  const int TJ = (nw + 15) / 16, CG = (TJ + CT - 1) / CT;
  const int64_t tasks = ((N + 16 * RT - 1) / (16 * RT)) * CG;
  hipLaunchKernelGGL((k_rotate<RT, CT>), dim3((unsigned)((tasks + 3) / 4)), dim3(256), 0, st,
                     reinterpret_cast<const double2*>(A), lda, N, m,
                     reinterpret_cast<const double2*>(V), ldv, n, reinterpret_cast<double2*>(C),
                     ldc, nw);
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
