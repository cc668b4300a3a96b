// Certificate data of Lemma 4.1 in the reference norms of X + s C_sigma
// (X = K + eps h I), one set per reference shift s:
//   * the residual Gram G_s = Z^H (X + s C)^{-1} Z, Z = [C w | X U | C U],
//     from the eigen-decomposition of the conductor block of X^{-1}
//     (Sherman-Morrison-Woodbury: no full-order solve per shift);
//   * the conjugation-defect form D'_s, whose quadratic form bounds the
//     distance from conj(U a) to span(U) in the same norm.
#include <algorithm>

#include "device_util.h"
#include "kernels.h"

namespace mpt {

namespace {
constexpr int kRgRows = 32;  // rows of B staged in LDS per step
}

// Three weighted Grams of B (n_c x L, row-major) per shift s_k:
//   out[((k * 3 + f) * L + p) * L + q] = sum_r wt_f(lam_r) conj(B[r][p]) B[r][q]
//   wt_0 = lam / (1 + s lam), wt_1 = 1 / (1 + s lam), wt_2 = s / (1 + s lam).
// blockIdx.y = shift; each thread owns one (p, q); rows are summed in order.
__global__ __launch_bounds__(256) void k_ref_gram(const double2* __restrict__ B, int64_t nc,
                                                  int L, const double* __restrict__ lam,
                                                  const double* __restrict__ s_ref,
                                                  double2* __restrict__ out) {
  extern __shared__ double2 sB[];  // [kRgRows][L]
  __shared__ double sw[3][kRgRows];
  const int k = blockIdx.y;
  const double s = s_ref[k];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = e < L * L;
  const int p = act ? e / L : 0, q = act ? e % L : 0;
  double2 acc[3];
#pragma unroll
  for (int f = 0; f < 3; ++f) acc[f] = make_double2(0.0, 0.0);
  for (int64_t r0 = 0; r0 < nc; r0 += kRgRows) {
    const int nr = (int)(nc - r0 < kRgRows ? nc - r0 : kRgRows);
    __syncthreads();
    for (int t = threadIdx.x; t < nr * L; t += blockDim.x) sB[t] = B[r0 * L + t];
    if (threadIdx.x < nr) {
      const double l = lam[r0 + threadIdx.x];
      const double chi = 1.0 / (1.0 + s * l);
      sw[0][threadIdx.x] = l * chi;
      sw[1][threadIdx.x] = chi;
      sw[2][threadIdx.x] = s * chi;
    }
    __syncthreads();
    if (act) {
      for (int r = 0; r < nr; ++r) {
        const double2 x = sB[r * L + p], y = sB[r * L + q];
        const double re = fma(x.x, y.x, x.y * y.y);  // conj(x) y
        const double im = fma(x.x, y.y, -x.y * y.x);
#pragma unroll
        for (int f = 0; f < 3; ++f) {
          acc[f].x = fma(sw[f][r], re, acc[f].x);
          acc[f].y = fma(sw[f][r], im, acc[f].y);
        }
      }
    }
  }
  if (act) {
#pragma unroll
    for (int f = 0; f < 3; ++f) out[((size_t)(k * 3 + f) * L + p) * L + q] = acc[f];
  }
}

// G_s ((2M+3)^2 per shift) from the weighted Grams (L = M + 3 columns of B:
// w_1..3 then U).  Unknown order of G: [C w (3) | X U (M) | C U (M)].
//   both indices outside X U:  phi Gram        (C-supported columns)
//   exactly one in X U:        chi Gram        ((X + sC)^{-1} X = I - s (X + sC)^{-1} C)
//   both in X U:               A0 - (s chi) Gram
// Hermitian by definition: the two computed triangles are averaged.
__global__ void k_ref_assemble(int M, int n_ref, const double2* __restrict__ Wg,
                               const double2* __restrict__ A0, double2* __restrict__ G) {
  const int L2 = 2 * M + 3, L = M + 3;
  const int64_t tot = (int64_t)n_ref * L2 * L2;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(e / ((int64_t)L2 * L2));
    const int ab = (int)(e % ((int64_t)L2 * L2));
    const int a = ab / L2, b = ab % L2;
    auto val = [&](int i, int j) {
      const bool xi = i >= 3 && i < 3 + M, xj = j >= 3 && j < 3 + M;
      const int bi = i < 3 ? i : (xi ? i : i - M), bj = j < 3 ? j : (xj ? j : j - M);
      const double2* Wk = Wg + (size_t)k * 3 * L * L;
      if (xi && xj) {
        const double2 g = Wk[(size_t)2 * L * L + bi * L + bj];
        const double2 a0 = A0[(i - 3) * M + (j - 3)];
        return make_double2(a0.x - g.x, a0.y - g.y);
      }
      if (xi || xj) return Wk[(size_t)L * L + bi * L + bj];
      return Wk[bi * L + bj];
    };
    const double2 u = val(a, b), t = val(b, a);
    G[e] = make_double2(0.5 * (u.x + t.x), 0.5 * (u.y - t.y));
  }
}

// D'_s for one shift and one target direction per workgroup (blockIdx.x =
// shift k, blockIdx.y = direction b of nd; nd = 1 for the joint basis):
//   A_s = A0 + s C_M = L L^H (Cholesky), T_s = T_X + s T_C,
//   Y = L^{-1} T_s,  D_s = A_s - conj(Y^H Y),  D'_s = D_s / 2 + 4 eps_h U^H U,
// stored Hermitian.  For the per-direction form the solve is restricted to
// block b of the concatenated basis (rows and columns [e[b], e[b+1])): A_s
// becomes the identity outside that block and T_s loses its other rows, so
// Y^H Y = T_b:^H A_s,bb^{-1} T_b:, and D' is kept on the diagonal blocks only
// (the blocks D'_{b<-j}).  Lw, Yw: M x M work matrices per (shift, b), global
// memory.  TC is read at offset 3 of an (M+3)-column Gram (its U block).
__global__ __launch_bounds__(256) void k_defect(int M, const double* __restrict__ s_ref,
                                                const double2* __restrict__ A0,
                                                const double2* __restrict__ CM,
                                                const double2* __restrict__ TXk,
                                                const double2* __restrict__ TXu,
                                                const double2* __restrict__ TCg,
                                                const double2* __restrict__ UhU, double eps_h,
                                                int4 eb, double2* __restrict__ Lwa,
                                                double2* __restrict__ Ywa,
                                                double2* __restrict__ Dp) {
  const int k = blockIdx.x, b = blockIdx.y, nd = gridDim.y;
  const double s = s_ref[k];
  const int L = M + 3;
  const size_t slot = (size_t)k * nd + b;
  double2* Lw = Lwa + slot * M * M;
  double2* Yw = Ywa + slot * M * M;
  double2* D = Dp + slot * M * M;
  // block bounds eb.x = 0 <= eb.y <= eb.z <= eb.w = M; direction of an index
  auto blk = [&](int r) { return r < eb.y ? 0 : (r < eb.z ? 1 : 2); };
  const int lo = nd == 1 ? 0 : (b == 0 ? 0 : (b == 1 ? eb.y : eb.z));
  const int hi = nd == 1 ? M : (b == 0 ? eb.y : (b == 1 ? eb.z : M));
  const int tid = threadIdx.x, nt = blockDim.x;
  __shared__ double sinv;
  for (int q = tid; q < M * M; q += nt) {
    const int i = q / M, j = q % M;
    const bool in_i = i >= lo && i < hi, in_j = j >= lo && j < hi;
    const double2 a = A0[q], c = CM[q];
    Lw[q] = (in_i && in_j) ? make_double2(fma(s, c.x, a.x), fma(s, c.y, a.y))
                           : make_double2(i == j ? 1.0 : 0.0, 0.0);
    // T_X = U^H X conj(U) = U^H conj(K U) + eps_h U^H conj(U)
    const double2 tk = TXk[q], tu = TXu[q], tc = TCg[(3 + i) * L + 3 + j];
    const double2 tx = make_double2(fma(eps_h, tu.x, tk.x), fma(eps_h, tu.y, tk.y));
    Yw[q] = in_i ? make_double2(fma(s, tc.x, tx.x), fma(s, tc.y, tx.y)) : make_double2(0.0, 0.0);
  }
  // right-looking Cholesky, lower triangle
  for (int c = 0; c < M; ++c) {
    __syncthreads();
    if (tid == 0) {
      const double d = sqrt(Lw[c * M + c].x);  // NaN for a non-positive pivot
      Lw[c * M + c] = make_double2(d, 0.0);
      sinv = 1.0 / d;
    }
    __syncthreads();
    const double inv = sinv;
    for (int i = c + 1 + tid; i < M; i += nt) {
      const double2 v = Lw[i * M + c];
      Lw[i * M + c] = make_double2(v.x * inv, v.y * inv);
    }
    __syncthreads();
    const int rem = M - c - 1;
    for (int e = tid; e < rem * rem; e += nt) {
      const int i = c + 1 + e / rem, j = c + 1 + e % rem;
      if (j <= i) {
        const double2 li = Lw[i * M + c], lj = Lw[j * M + c];
        Lw[i * M + j] = cfms(Lw[i * M + j], li, cconj(lj));
      }
    }
  }
  // forward substitution L Y = T_s, all columns at once
  for (int c = 0; c < M; ++c) {
    __syncthreads();
    const double inv = 1.0 / Lw[c * M + c].x;
    for (int j = tid; j < M; j += nt) {
      const double2 v = Yw[c * M + j];
      Yw[c * M + j] = make_double2(v.x * inv, v.y * inv);
    }
    __syncthreads();
    for (int e = tid; e < (M - c - 1) * M; e += nt) {
      const int i = c + 1 + e / M, j = e % M;
      Yw[i * M + j] = cfms(Yw[i * M + j], Lw[i * M + c], Yw[c * M + j]);
    }
  }
  __syncthreads();
  // X = A_s - conj(Y^H Y), D' = X / 2 + 4 eps_h U^H U, into Lw (no longer needed)
  for (int q0 = tid; q0 < M * M; q0 += nt) {
    const int p = q0 / M, q = q0 % M;
    double2 acc = make_double2(0.0, 0.0);
    for (int r = 0; r < M; ++r) acc = cfma(acc, cconj(Yw[r * M + p]), Yw[r * M + q]);
    const double2 a = A0[q0], c = CM[q0], u = UhU[q0];
    const double xr = fma(s, c.x, a.x) - acc.x, xi = fma(s, c.y, a.y) + acc.y;
    Lw[q0] = make_double2(fma(0.5, xr, 4.0 * eps_h * u.x), fma(0.5, xi, 4.0 * eps_h * u.y));
  }
  __syncthreads();
  for (int q0 = tid; q0 < M * M; q0 += nt) {
    const int p = q0 / M, q = q0 % M;
    const double2 u = Lw[p * M + q], t = Lw[q * M + p];
    D[q0] = (nd == 1 || blk(p) == blk(q)) ? make_double2(0.5 * (u.x + t.x), 0.5 * (u.y - t.y))
                                          : make_double2(0.0, 0.0);
  }
}

size_t cert_ws_size(int M, int64_t nc, int n_ref) {
  const int L = M + 3;
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  return al((size_t)nc * L * 16) +                // B
         al((size_t)n_ref * 3 * L * L * 16) +     // weighted Grams
         al((size_t)n_ref * 3 * M * M * 16) * 2 + // Cholesky / solve work (per direction)
         al(rcgemm_ws_size(nc, L));
}

hipError_t cert_launch(int M, const double* Zc, int64_t nc, const double* Vt, const double* lam,
                       int n_ref, const double* s_ref, const double* A0, const double* CM,
                       const double* UhU, const double* TXk, const double* TXu,
                       const double* TCz, double eps_h, const int32_t* dirs, double* G,
                       double* Dp, void* ws, hipStream_t st) {
  const int L = M + 3;
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  char* p = reinterpret_cast<char*>(ws);
  double2* B = reinterpret_cast<double2*>(p); p += al((size_t)nc * L * 16);
  double2* Wg = reinterpret_cast<double2*>(p); p += al((size_t)n_ref * 3 * L * L * 16);
  double2* Lw = reinterpret_cast<double2*>(p); p += al((size_t)n_ref * 3 * M * M * 16);
  double2* Yw = reinterpret_cast<double2*>(p); p += al((size_t)n_ref * 3 * M * M * 16);
  void* gws = p;
  hipError_t e;
  // B = Vt Zc, then the weighted Grams and G_s per shift
  if ((e = real_complex_gemm(Vt, nc, Zc, L, reinterpret_cast<double*>(B), gws, st)) != hipSuccess)
    return e;
  {
    const dim3 grid((unsigned)((L * L + 255) / 256), (unsigned)n_ref);
    hipLaunchKernelGGL(k_ref_gram, grid, dim3(256), (size_t)kRgRows * L * sizeof(double2), st,
                       B, nc, L, lam, s_ref, Wg);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  {
    const int64_t tot = (int64_t)n_ref * (2 * M + 3) * (2 * M + 3);
    const unsigned blocks = (unsigned)std::min<int64_t>((tot + 255) / 256, 4096);
    hipLaunchKernelGGL(k_ref_assemble, dim3(blocks), dim3(256), 0, st, M, n_ref, Wg,
                       reinterpret_cast<const double2*>(A0), reinterpret_cast<double2*>(G));
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const int nd = dirs ? 3 : 1;
  const int4 eb = dirs ? make_int4(0, dirs[0], dirs[0] + dirs[1], M) : make_int4(0, M, M, M);
  hipLaunchKernelGGL(k_defect, dim3((unsigned)n_ref, (unsigned)nd), dim3(256), 0, st, M, s_ref,
                     reinterpret_cast<const double2*>(A0), reinterpret_cast<const double2*>(CM),
                     reinterpret_cast<const double2*>(TXk), reinterpret_cast<const double2*>(TXu),
                     reinterpret_cast<const double2*>(TCz),
                     reinterpret_cast<const double2*>(UhU), eps_h, eb, Lw, Yw,
                     reinterpret_cast<double2*>(Dp));
  return hipGetLastError();
}

}  // namespace mpt
