// Hermitian eigen-decomposition of a small matrix (n <= 192) to absolute
// accuracy ~ eps ||A||, for the first pass of the POD basis, where the
// eigenvectors only have to rotate the snapshot Gram close to diagonal:
//   1. Householder reduction to tridiagonal form, H_k = I - g_k u_k u_k^H
//      (one workgroup, packed lower triangle in LDS; above the LDS budget the
//      first steps run on a copy in global memory);
//   2. a diagonal unitary that makes the off-diagonal real;
//   3. all eigenvalues of the real tridiagonal by multisection on Sturm
//      counts (every eigenvalue's interval tested at P points per step);
//   4. eigenvectors by inverse iteration with partial pivoting, one wave each;
//   5. two passes of modified Gram-Schmidt in decreasing eigenvalue order;
//   6. back-transformation V = H_0 ... H_{n-3} Phi Z, one wave per column.
// The work is O(n^3) once, against about a dozen O(n^3) sweeps for Jacobi.
#include "device_util.h"
#include "kernels.h"

namespace mpt {

constexpr int kTriMaxN = 192;
constexpr int kTriThreads = 1024;
constexpr size_t kTriLdsBudget = 150 * 1024;
constexpr int kTriWaves = 4;  // waves per workgroup of the per-vector kernels

__device__ __forceinline__ int lpos(int i, int j) { return i * (i + 1) / 2 + j; }  // i >= j

__device__ __forceinline__ double2 lget(const double2* A, int i, int j) {
  return i >= j ? A[lpos(i, j)] : cconj(A[lpos(j, i)]);
}

// 1. + 2.: d (n), e (n-1, >= 0), phases ph (n), reflectors Hv (row k holds
// u_k in columns k+1..n-1) and their scalars g (n-2).
// The packed lower triangle (A[lpos(i - base, j - base)], rows and columns
// >= base held) lives in LDS when it fits; otherwise the first k0 steps work
// on a copy in global memory, and at step k0 the trailing triangle (rows and
// columns >= k0, which then fits) moves into LDS for the remaining steps.
struct HetrdShared {
  double2 u[kTriMaxN], p[kTriMaxN], beta[kTriMaxN];
  double g;
};

// step k on the triangle A (rows and columns >= base stored)
__device__ __forceinline__ void hetrd_step(double2* A, int base, int k, int n, HetrdShared& sh,
                                           double2* __restrict__ Hv, double* __restrict__ gam,
                                           double* __restrict__ dout) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = __lane_id(), wave = tid >> 6;
  auto at = [&](int i, int j) -> double2& { return A[lpos(i - base, j - base)]; };  // i >= j
  const int L = n - k - 1;  // trailing block rows/cols o .. n-1
  const int o = k + 1;
  if (wave == 0) {
    double s = 0.0;
    for (int i = lane; i < L; i += 64) {
      const double2 x = at(o + i, k);
      s += x.x * x.x + x.y * x.y;
    }
    s = wave_sum(s);
    const double alpha = sqrt(s);
    const double2 x0 = at(o, k);
    const double ax0 = sqrt(x0.x * x0.x + x0.y * x0.y);
    const bool refl = alpha > 1e-300;
    double2 th = make_double2(1.0, 0.0);
    if (ax0 > 0.0) th = make_double2(x0.x / ax0, x0.y / ax0);
    const double g = refl ? 1.0 / (alpha * (alpha + ax0)) : 0.0;
    for (int i = lane; i < L; i += 64) {
      double2 x = at(o + i, k);
      if (i == 0) x = make_double2(x.x + th.x * alpha, x.y + th.y * alpha);
      if (!refl) x = make_double2(0.0, 0.0);
      sh.u[i] = x;
      Hv[(size_t)k * n + o + i] = x;
    }
    if (lane == 0) {
      sh.g = g;
      gam[k] = g;
      sh.beta[k] = refl ? make_double2(-th.x * alpha, -th.y * alpha) : x0;
      dout[k] = at(k, k).x;
    }
  }
  __syncthreads();
  const double g = sh.g;
  if (g == 0.0) return;  // uniform: column already reduced
  // p = g A22 u, eight threads per row
  const int s8 = tid & 7;
  for (int i = tid >> 3; i < L; i += nt >> 3) {
    double2 acc = make_double2(0.0, 0.0);
    // the stored row part (j <= i, contiguous), then the mirrored column part
    int j = s8;
    for (; j <= i; j += 8) acc = cfma(acc, at(o + i, o + j), sh.u[j]);
    for (; j < L; j += 8) acc = cfma(acc, cconj(at(o + j, o + i)), sh.u[j]);
    // sum over the 8 lanes of the row group (DPP inside a half-row)
    acc.x += dpp_d<kDppXor1>(acc.x, 0.0);
    acc.y += dpp_d<kDppXor1>(acc.y, 0.0);
    acc.x += dpp_d<kDppXor2>(acc.x, 0.0);
    acc.y += dpp_d<kDppXor2>(acc.y, 0.0);
    acc.x += dpp_d<kDppHalfMirror>(acc.x, 0.0);
    acc.y += dpp_d<kDppHalfMirror>(acc.y, 0.0);
    if (s8 == 0) sh.p[i] = make_double2(g * acc.x, g * acc.y);
  }
  __syncthreads();
  // K = g/2 Re(u^H p) (every wave computes it), w = p - K u,
  // A22 <- A22 - u w^H - w u^H on the lower triangle: thread (r, c) of a
  // 32 x 32 grid takes rows r + 32 a and, in each, columns c + 32 b <= row
  double kk = 0.0;
  for (int i = lane; i < L; i += 64) kk += cmulc(sh.u[i], sh.p[i]).x;
  kk = 0.5 * g * wave_sum(kk);
  const int r0 = tid >> 5, c0 = tid & 31;
  for (int i = r0; i < L; i += nt >> 5) {
    const double2 ui = sh.u[i], pi = sh.p[i];
    const double2 wi = make_double2(pi.x - kk * ui.x, pi.y - kk * ui.y);
    for (int j = c0; j <= i; j += 32) {
      const double2 uj = sh.u[j], pj = sh.p[j];
      const double2 wj = make_double2(pj.x - kk * uj.x, pj.y - kk * uj.y);
      double2& ar = at(o + i, o + j);
      double2 a = ar;
      a = cfms(a, ui, cconj(wj));
      a = cfms(a, wi, cconj(uj));
      ar = a;
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(kTriThreads) void k_hetrd(const double2* __restrict__ Ag, int n,
                                                       int k0, double2* __restrict__ Ap,
                                                       double2* __restrict__ Hv,
                                                       double* __restrict__ gam,
                                                       double* __restrict__ dout,
                                                       double* __restrict__ eout,
                                                       double2* __restrict__ ph) {
  extern __shared__ double2 smem[];
  __shared__ HetrdShared sh;
  const int tid = threadIdx.x, nt = blockDim.x;
  double2* A0 = k0 == 0 ? smem : Ap;
  for (int i = tid; i < n * n; i += nt) {
    const int r = i / n, c = i % n;
    if (r >= c) A0[lpos(r, c)] = Ag[i];
  }
  __syncthreads();
  int k = 0;
  for (; k < k0 && k + 2 < n; ++k) hetrd_step(Ap, 0, k, n, sh, Hv, gam, dout);
  if (k0 > 0) {  // the trailing triangle, rows and columns >= k0, into LDS
    const int m0 = n - k0, cnt = m0 * (m0 + 1) / 2;
    for (int e = tid; e < cnt; e += nt) {
      int i = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
      while ((i + 1) * (i + 2) / 2 <= e) ++i;
      while (i * (i + 1) / 2 > e) --i;
      const int j = e - i * (i + 1) / 2;
      smem[e] = Ap[lpos(k0 + i, k0 + j)];
    }
    __syncthreads();
  }
  for (; k + 2 < n; ++k) hetrd_step(smem, k0, k, n, sh, Hv, gam, dout);
  if (tid == 0) {
    auto at = [&](int i, int j) { return smem[lpos(i - k0, j - k0)]; };
    if (n >= 2) {
      dout[n - 2] = at(n - 2, n - 2).x;
      sh.beta[n - 2] = at(n - 1, n - 2);
    }
    dout[n - 1] = at(n - 1, n - 1).x;
    double2 f = make_double2(1.0, 0.0);
    ph[0] = f;
    for (int kk = 0; kk + 1 < n; ++kk) {
      const double2 b = sh.beta[kk];
      const double ab = sqrt(b.x * b.x + b.y * b.y);
      eout[kk] = ab;
      if (ab > 0.0) f = cmul(f, make_double2(b.x / ab, b.y / ab));
      ph[kk + 1] = f;
    }
  }
}

// 3. eigenvalues (ascending) of the real symmetric tridiagonal (d, e): one
// wave per eigenvalue j tests its interval at 64 points per step (one Sturm
// count per lane); the counts are monotone in the point, so the new interval
// is found by a ballot.  Ten steps shrink the Gershgorin width by 65^10.
__global__ __launch_bounds__(64 * kTriWaves) void k_tri_eigvals(const double* __restrict__ d,
                                                                const double* __restrict__ e,
                                                                int n, double* __restrict__ lam) {
  __shared__ double sd[kTriMaxN], se2[kTriMaxN];
  __shared__ double gb[3];
  const int tid = threadIdx.x, lane = __lane_id(), wave = tid >> 6;
  for (int i = tid; i < n; i += blockDim.x) {
    sd[i] = d[i];
    se2[i] = i + 1 < n ? e[i] * e[i] : 0.0;
  }
  __syncthreads();
  if (wave == 0) {
    double gl = 1e308, gu = -1e308, em = 0.0;
    for (int i = lane; i < n; i += 64) {
      const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
      gl = fmin(gl, sd[i] - r);
      gu = fmax(gu, sd[i] + r);
      em = fmax(em, se2[i]);
    }
    gl = -wave_max(-gl);
    gu = wave_max(gu);
    em = wave_max(em);
    if (lane == 0) {
      const double tn = fmax(fabs(gl), fabs(gu));
      gb[0] = gl - 4.0 * 2.220446049250313e-16 * tn * n;
      gb[1] = gu + 4.0 * 2.220446049250313e-16 * tn * n;
      gb[2] = 1e-290 * fmax(1.0, em);
    }
  }
  __syncthreads();
  const int j = blockIdx.x * kTriWaves + wave;
  if (j >= n) return;
  const double pivmin = gb[2];
  double lo = gb[0], hi = gb[1];
  for (int it = 0; it < 10; ++it) {
    const double x = lo + (hi - lo) * (double)(lane + 1) * (1.0 / 65.0);
    double s = sd[0] - x;
    int c = s < 0.0 ? 1 : 0;
    for (int i = 1; i < n; ++i) {
      if (fabs(s) < pivmin) s = -pivmin;
      double r = __builtin_amdgcn_rcp(s);
      r = fma(r, fma(-s, r, 1.0), r);
      s = (sd[i] - x) - se2[i - 1] * r;
      c += s < 0.0 ? 1 : 0;
    }
    const int k = __popcll(__ballot(c <= j));  // points with count <= j
    const double xl = lo + (hi - lo) * (double)k * (1.0 / 65.0);
    const double xh = lo + (hi - lo) * (double)(k + 1) * (1.0 / 65.0);
    if (k > 0) lo = xl;
    if (k < 64) hi = xh;
  }
  if (lane == 0) lam[j] = 0.5 * (lo + hi);
}

// 4. inverse iteration: three solves of (T - lam_j) x = b with Gaussian
// elimination with partial pivoting (lane 0; factors in LDS), each followed
// by normalisation.  Z row j = eigenvector j.
__global__ __launch_bounds__(64 * kTriWaves) void k_tri_invit(const double* __restrict__ d,
                                                              const double* __restrict__ e,
                                                              const double* __restrict__ lam,
                                                              int n, double* __restrict__ Z) {
  __shared__ double f0[kTriWaves][kTriMaxN], f1[kTriWaves][kTriMaxN], f2[kTriWaves][kTriMaxN],
      fm[kTriWaves][kTriMaxN], bx[kTriWaves][kTriMaxN], yv[kTriWaves][kTriMaxN];
  __shared__ unsigned char fsw[kTriWaves][kTriMaxN];
  const int wave = threadIdx.x >> 6, lane = __lane_id();
  const int j = blockIdx.x * kTriWaves + wave;
  if (j >= n) return;
  double* U0 = f0[wave];
  double* U1 = f1[wave];
  double* U2 = f2[wave];
  double* mm = fm[wave];
  double* b = bx[wave];
  double* y = yv[wave];
  unsigned char* sw = fsw[wave];
  // norm of T for the pivot floor
  double tn = 0.0;
  for (int i = lane; i < n; i += 64)
    tn = fmax(tn, fabs(d[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0));
  tn = wave_max(tn);
  const double tiny = 2.220446049250313e-16 * fmax(tn, 1e-300);
  const double lj = lam[j];
  for (int i = lane; i < n; i += 64) b[i] = 1.0 + 0.01 * (double)((i * 37 + j * 11) % 17);
  if (lane == 0) {
    double xr = d[0] - lj, yr = n > 1 ? e[0] : 0.0;
    for (int i = 0; i + 1 < n; ++i) {
      const double ei = e[i], an = d[i + 1] - lj, en = i + 2 < n ? e[i + 1] : 0.0;
      double mi;
      if (fabs(ei) > fabs(xr)) {
        sw[i] = 1;
        mi = xr / ei;
        U0[i] = ei;
        U1[i] = an;
        U2[i] = en;
        const double nx = yr - mi * an, ny = -mi * en;
        xr = nx;
        yr = ny;
      } else {
        sw[i] = 0;
        const double pv = xr != 0.0 ? xr : tiny;
        mi = ei / pv;
        U0[i] = pv;
        U1[i] = yr;
        U2[i] = 0.0;
        xr = an - mi * yr;
        yr = en;
      }
      mm[i] = mi;
    }
    U0[n - 1] = xr;
    // reciprocal pivots (kept in U0), floored at eps ||T||
    for (int i = 0; i < n; ++i) {
      double u0 = U0[i];
      if (fabs(u0) < tiny) u0 = u0 >= 0.0 ? tiny : -tiny;
      U0[i] = 1.0 / u0;
    }
  }
  for (int s = 0; s < 3; ++s) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane == 0) {
      double bc = b[0];
#pragma unroll 4
      for (int i = 0; i + 1 < n; ++i) {
        if (sw[i]) {
          y[i] = b[i + 1];
          bc = bc - mm[i] * b[i + 1];
        } else {
          y[i] = bc;
          bc = b[i + 1] - mm[i] * bc;
        }
      }
      y[n - 1] = bc;
      double x1 = 0.0, x2 = 0.0;  // x[i+1], x[i+2]
#pragma unroll 4
      for (int i = n - 1; i >= 0; --i) {
        double v = y[i];
        if (i + 1 < n) v -= U1[i] * x1 + U2[i] * x2;
        double xi = v * U0[i];
        if (fabs(xi) > 1e150) {  // rescale what is computed so far
          for (int t = i + 1; t < n; ++t) b[t] *= 1e-150;
          x1 *= 1e-150;
          x2 *= 1e-150;
          xi *= 1e-150;
        }
        b[i] = xi;
        x2 = x1;
        x1 = xi;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double nr = 0.0;
    for (int i = lane; i < n; i += 64) nr += b[i] * b[i];
    nr = wave_sum(nr);
    const double inv = 1.0 / sqrt(nr);
    for (int i = lane; i < n; i += 64) b[i] *= inv;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (int i = lane; i < n; i += 64) Z[(size_t)j * n + i] = b[i];
}

// 5. two passes of modified Gram-Schmidt over the rows of Z in decreasing
// eigenvalue order (lam ascending, so row n-1 first).  Z lives in registers:
// row r belongs to wave r % 16 (slot r / 16), lane l holds its columns l,
// l + 64 and l + 128.  A step normalises the pivot row in its wave, passes
// it through LDS (double-buffered, one barrier per step) and every wave
// removes its projection from its own rows below the pivot, with one wave
// reduction per row.
constexpr int kMgsWaves = 16;
constexpr int kMgsSlots = (kTriMaxN + kMgsWaves - 1) / kMgsWaves;
constexpr int kMgsCols = (kTriMaxN + 63) / 64;

__global__ __launch_bounds__(64 * kMgsWaves) void k_tri_mgs(double* __restrict__ Zg, int n) {
  __shared__ double piv[2][kTriMaxN];
  const int lane = __lane_id();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double z[kMgsSlots][kMgsCols];
#pragma unroll
  for (int s = 0; s < kMgsSlots; ++s)
#pragma unroll
    for (int k = 0; k < kMgsCols; ++k) {
      const int r = s * kMgsWaves + wave, c = k * 64 + lane;
      z[s][k] = (r < n && c < n) ? Zg[(size_t)r * n + c] : 0.0;
    }
  for (int pass = 0; pass < 2; ++pass) {
    for (int j = n - 1; j >= 0; --j) {
      const int buf = j & 1;
      if (wave == j % kMgsWaves) {
        const int sj = j / kMgsWaves;
        double nr = 0.0;
#pragma unroll
        for (int s = 0; s < kMgsSlots; ++s)
          if (s == sj)
#pragma unroll
            for (int k = 0; k < kMgsCols; ++k) nr += z[s][k] * z[s][k];
        const double inv = 1.0 / sqrt(fmax(wave_sum(nr), 1e-300));
#pragma unroll
        for (int s = 0; s < kMgsSlots; ++s)
          if (s == sj)
#pragma unroll
            for (int k = 0; k < kMgsCols; ++k) {
              z[s][k] *= inv;
              const int c = k * 64 + lane;
              if (c < n) piv[buf][c] = z[s][k];
            }
      }
      __syncthreads();
      double pj[kMgsCols];
#pragma unroll
      for (int k = 0; k < kMgsCols; ++k) {
        const int c = k * 64 + lane;
        pj[k] = c < n ? piv[buf][c] : 0.0;
      }
      double d[kMgsSlots];
#pragma unroll
      for (int s = 0; s < kMgsSlots; ++s) {
        d[s] = 0.0;
#pragma unroll
        for (int k = 0; k < kMgsCols; ++k) d[s] += z[s][k] * pj[k];
      }
#pragma unroll
      for (int s = 0; s < kMgsSlots; ++s) {
        const int r = s * kMgsWaves + wave;
        if (r < j) {  // wave-uniform
          const double ds = wave_sum(d[s]);
#pragma unroll
          for (int k = 0; k < kMgsCols; ++k) z[s][k] -= ds * pj[k];
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int s = 0; s < kMgsSlots; ++s)
#pragma unroll
    for (int k = 0; k < kMgsCols; ++k) {
      const int r = s * kMgsWaves + wave, c = k * 64 + lane;
      if (r < n && c < n) Zg[(size_t)r * n + c] = z[s][k];
    }
}

// 6. V[:, j] = H_0 ... H_{n-3} Phi z_j; V row-major n x n (V[i n + j])
__global__ __launch_bounds__(64 * kTriWaves) void k_tri_back(const double* __restrict__ Z,
                                                             const double2* __restrict__ ph,
                                                             const double2* __restrict__ Hv,
                                                             const double* __restrict__ gam, int n,
                                                             double2* __restrict__ V) {
  constexpr int kSlots = (kTriMaxN + 63) / 64;
  __shared__ double gs[kTriMaxN];
  const int wave = threadIdx.x >> 6, lane = __lane_id();
  for (int i = threadIdx.x; i + 2 < n; i += blockDim.x) gs[i] = gam[i];
  __syncthreads();
  const int j = blockIdx.x * kTriWaves + wave;
  if (j >= n) return;
  double2 y[kSlots];
#pragma unroll
  for (int t = 0; t < kSlots; ++t) {
    const int i = lane + 64 * t;
    y[t] = make_double2(0.0, 0.0);
    if (i < n) {
      const double z = Z[(size_t)j * n + i];
      const double2 f = ph[i];
      y[t] = make_double2(f.x * z, f.y * z);
    }
  }
  // reflector k + 1's entries are loaded while reflector k is applied
  auto load_u = [&](int k, double2 (&uu)[kSlots]) {
#pragma unroll
    for (int t = 0; t < kSlots; ++t) {
      const int i = lane + 64 * t;
      uu[t] = (k >= 0 && i > k && i < n) ? Hv[(size_t)k * n + i] : make_double2(0.0, 0.0);
    }
  };
  double2 un[kSlots];
  load_u(n - 3, un);
  for (int k = n - 3; k >= 0; --k) {
    double2 uu[kSlots];
#pragma unroll
    for (int t = 0; t < kSlots; ++t) uu[t] = un[t];
    load_u(k - 1, un);
    const double g = gs[k];
    if (g == 0.0) continue;
    double2 dt = make_double2(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < kSlots; ++t) dt = cfmac(dt, uu[t], y[t]);
    dt.x = wave_sum(dt.x) * g;
    dt.y = wave_sum(dt.y) * g;
#pragma unroll
    for (int t = 0; t < kSlots; ++t) y[t] = cfms(y[t], uu[t], dt);
  }
#pragma unroll
  for (int t = 0; t < kSlots; ++t) {
    const int i = lane + 64 * t;
    if (i < n) V[(size_t)i * n + j] = y[t];
  }
}

struct TriLayout {
  size_t ap, hv, gam, d, e, ph, z, end;
};
static TriLayout tri_layout(int n) {
  TriLayout L;
  size_t o = 0;
  auto take = [&](size_t b) { const size_t r = o; o = (o + b + 255) / 256 * 256; return r; };
  L.ap = take((size_t)n * (n + 1) / 2 * sizeof(double2));
  L.hv = take((size_t)n * n * sizeof(double2));
  L.gam = take((size_t)n * sizeof(double));
  L.d = take((size_t)n * sizeof(double));
  L.e = take((size_t)n * sizeof(double));
  L.ph = take((size_t)n * sizeof(double2));
  L.z = take((size_t)n * n * sizeof(double));
  L.end = o;
  return L;
}

size_t tridiag_ws_size(int n) { return n > 0 ? tri_layout(n).end : 0; }

hipError_t tridiag_eig_launch(const double* A, int n, double* V, double* lam, void* ws,
                              hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (n > kTriMaxN) return hipErrorInvalidValue;
  const TriLayout L = tri_layout(n);
  char* w = reinterpret_cast<char*>(ws);
  double2* Ap = reinterpret_cast<double2*>(w + L.ap);
  double2* Hv = reinterpret_cast<double2*>(w + L.hv);
  double* gam = reinterpret_cast<double*>(w + L.gam);
  double* d = reinterpret_cast<double*>(w + L.d);
  double* e = reinterpret_cast<double*>(w + L.e);
  double2* ph = reinterpret_cast<double2*>(w + L.ph);
  double* Z = reinterpret_cast<double*>(w + L.z);
  const double2* Ag = reinterpret_cast<const double2*>(A);
  // k0: the first step whose trailing triangle (rows and columns >= k0) fits
  // the LDS budget (0: the whole matrix fits)
  int k0 = 0;
  while ((size_t)(n - k0) * (n - k0 + 1) / 2 * sizeof(double2) > kTriLdsBudget) ++k0;
  const size_t lds_a = (size_t)(n - k0) * (n - k0 + 1) / 2 * sizeof(double2);
  hipLaunchKernelGGL(k_hetrd, dim3(1), dim3(kTriThreads), lds_a, st, Ag, n, k0, Ap, Hv, gam, d, e,
                     ph);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  const int nb = (n + kTriWaves - 1) / kTriWaves;
  hipLaunchKernelGGL(k_tri_eigvals, dim3(nb), dim3(64 * kTriWaves), 0, st, d, e, n, lam);
  err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_tri_invit, dim3(nb), dim3(64 * kTriWaves), 0, st, d, e, lam, n, Z);
  err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_tri_mgs, dim3(1), dim3(64 * kMgsWaves), 0, st, Z, n);
  err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_tri_back, dim3(nb), dim3(64 * kTriWaves), 0, st, Z, ph, Hv, gam, n,
                     reinterpret_cast<double2*>(V));
  return hipGetLastError();
}

}  // namespace mpt
