// Hessenberg-triangular form of the reduced pencil (A0, C_M) and the sweep
// built on it: the shifted-system method of Laub (IEEE TAC 1981) applied to
// eq. (ReducedA).
//
// Once per object, unitary Q and Z with
//     Q^H A0 Z = H (upper Hessenberg),   Q^H C_M Z = T (upper triangular)
// (Householder QR of C_M, then Givens rotations from both sides, as in the
// Moler-Stewart reduction), and f_i = Q^H g_i.  Then at every frequency
//     (A0 - i w C_M) a_i = i w g_i   <=>   (H - i w T) y_i = i w f_i,  a_i = Z y_i,
// a Hessenberg system: O(M^2) work instead of the O(M^3) LU of the dense
// reduced matrix.  The quadratic forms of eqs. (podprealmpt), (podpimagmpt)
// and of the certificate (Lemma 4.1) are evaluated at a = Z y with the
// matrices of the reduced model as they are: the certificate is a small
// difference of large terms, and its rounding floor |w|^T |G| |w| is a
// property of the basis it is evaluated in (in the rotated coordinates it can
// be orders of magnitude higher).
//
// Sweep kernel, per workgroup of 256 threads and a batch of 16 frequencies:
//   1. every frequency is solved by a segment of L = 16/32/64 lanes (row r in
//      lane r): column elimination from the right with pivoting between two
//      adjacent columns, the back substitution interleaved with it, then the
//      column transforms applied to the solution (a chain over the lanes);
//   2. a = Z y for the 48 solutions of the batch, then the products W A of the
//      stacked matrices W = [K_M; C_M; A0; G_cc; conj(g); F] (4 Mp + 16 rows)
//      with them, on FP64 MFMA; each output tile is contracted at once with
//      the solutions (the quadratic forms);
//   3. one thread per frequency combines the sums into R~, I and Delta.
#include "device_util.h"
#include "kernels.h"

namespace mpt {

constexpr int kPenBatch = 16;  // frequencies per workgroup batch

PencilLayout pencil_layout(int M) {
  PencilLayout L;
  L.Mp = (M + 15) / 16 * 16;
  L.Kp = (M + 3) / 4 * 4;
  L.NT = 4 * (L.Mp / 16) + 1;
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
  L.W = take((size_t)L.NT * (L.Kp / 4) * 64 * 16);
  L.S = take(27 * 8);
  const size_t nrot = M >= 3 ? (size_t)(M - 1) * (M - 2) / 2 : 1;
  L.rec = take(nrot * 3 * 8);
  L.total = o;
  return L;
}

namespace {

// Givens rotation [[c, s], [-conj(s), c]] (c real) with
//   [[c, s], [-conj(s), c]] [x; y] = [*; 0]
__device__ __forceinline__ void givens_left(double2 x, double2 y, double& c, double2& s) {
  const double ax = sqrt(x.x * x.x + x.y * x.y);
  const double ay2 = y.x * y.x + y.y * y.y;
  if (ay2 == 0.0) {
    c = 1.0;
    s = make_double2(0.0, 0.0);
    return;
  }
  if (ax == 0.0) {
    c = 0.0;
    s = make_double2(1.0, 0.0);
    return;
  }
  const double r = sqrt(ax * ax + ay2);
  c = ax / r;
  // s = (x / |x|) conj(y) / r
  const double2 u = make_double2(x.x / ax, x.y / ax);
  const double2 sy = cmul(u, cconj(y));
  s = make_double2(sy.x / r, sy.y / r);
}

// column rotation S = [[c, s], [-conj(s), c]] with [w, u] S = [0, *]
__device__ __forceinline__ void givens_right(double2 w, double2 u, double& c, double2& s) {
  const double au = sqrt(u.x * u.x + u.y * u.y);
  const double aw2 = w.x * w.x + w.y * w.y;
  if (aw2 == 0.0) {
    c = 1.0;
    s = make_double2(0.0, 0.0);
    return;
  }
  if (au == 0.0) {
    c = 0.0;
    s = make_double2(1.0, 0.0);
    return;
  }
  const double r = sqrt(au * au + aw2);
  c = au / r;
  // s = conj(w) (u / |u|) / r
  const double2 sw = cmul(cconj(w), make_double2(u.x / au, u.y / au));
  s = make_double2(sw.x / r, sw.y / r);
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace

// ------------------------------------------------------------ reduction
// One workgroup (256 threads) per object.  LDS: A, B (M x (M+1) each, padded
// rows), F (3 x M), v (M), beta.  The Givens chain runs in wave 0 (rotations
// are sequential; each is applied by up to 64 lanes at once); the right
// rotations are recorded for the accumulation of Z.
__global__ __launch_bounds__(256) void k_pencil_reduce(int M, const double2* __restrict__ A0,
                                                       const double2* __restrict__ CM,
                                                       const double2* __restrict__ g,
                                                       double2* __restrict__ H,
                                                       double2* __restrict__ T,
                                                       double2* __restrict__ f,
                                                       double* __restrict__ rec) {
  extern __shared__ double2 lds[];
  const int ld = M + 1;
  double2* sA = lds;
  double2* sB = sA + M * ld;
  double2* sF = sB + M * ld;
  double2* sV = sF + 3 * M;
  __shared__ double sBeta;
  const int tid = threadIdx.x, lane = __lane_id(), wave = tid >> 6;
  for (int e = tid; e < M * M; e += blockDim.x) {
    const int r = e / M, c = e % M;
    sA[r * ld + c] = A0[e];
    sB[r * ld + c] = CM[e];
  }
  for (int e = tid; e < 3 * M; e += blockDim.x) sF[e] = g[e];
  __syncthreads();

  // ---- Householder QR of B; the reflections are applied to A and F -----
  for (int k = 0; k + 1 < M; ++k) {
    const int len = M - k;
    if (wave == 0) {
      const double2 x = lane < len ? sB[(k + lane) * ld + k] : make_double2(0.0, 0.0);
      const double nrm2 = wave_sum(x.x * x.x + x.y * x.y);
      const double2 x0 = sB[k * ld + k];
      const double ax0 = sqrt(x0.x * x0.x + x0.y * x0.y);
      const double nrm = sqrt(nrm2);
      // alpha = -(x0 / |x0|) ||x||, v = x - alpha e_1, beta = 2 / ||v||^2
      const double2 ph = ax0 > 0.0 ? make_double2(x0.x / ax0, x0.y / ax0) : make_double2(1.0, 0.0);
      const double2 alpha = make_double2(-ph.x * nrm, -ph.y * nrm);
      const double2 v0 = make_double2(x0.x - alpha.x, x0.y - alpha.y);
      const double vn2 = nrm2 - ax0 * ax0 + (v0.x * v0.x + v0.y * v0.y);
      if (lane < len) sV[lane] = lane == 0 ? v0 : x;
      if (lane == 0) sBeta = (nrm2 > 0.0 && vn2 > 0.0) ? 2.0 / vn2 : 0.0;
    }
    __syncthreads();
    const double beta = sBeta;
    const int ncol = len + M + 3;
    if (beta != 0.0) {
      for (int t = tid; t < ncol; t += blockDim.x) {
        double2* col;
        int stride;
        if (t < len) {
          col = sB + k * ld + (k + t);
          stride = ld;
        } else if (t < len + M) {
          col = sA + k * ld + (t - len);
          stride = ld;
        } else {
          col = sF + (t - len - M) * M + k;
          stride = 1;
        }
        double2 s = make_double2(0.0, 0.0);
        for (int u = 0; u < len; ++u) s = cfmac(s, sV[u], col[u * stride]);
        s.x *= beta;
        s.y *= beta;
        for (int u = 0; u < len; ++u) col[u * stride] = cfms(col[u * stride], sV[u], s);
      }
    }
    __syncthreads();
    for (int u = 1 + tid; u < len; u += blockDim.x) sB[(k + u) * ld + k] = make_double2(0.0, 0.0);
    __syncthreads();
  }

  // ---- Givens chain: A to Hessenberg form, B kept triangular ------------
  if (wave == 0) {
    int nrec = 0;
    for (int j = 0; j + 2 < M; ++j) {
      for (int i = M - 1; i >= j + 2; --i) {
        // left rotation of rows i-1, i: zero A[i][j]
        double c;
        double2 s;
        givens_left(sA[(i - 1) * ld + j], sA[i * ld + j], c, s);
        const double2 ms = make_double2(-s.x, s.y);  // -conj(s)
        {
          const int col = j + lane;
          if (col < M) {
            const double2 x1 = sA[(i - 1) * ld + col], x2 = sA[i * ld + col];
            double2 n1 = cmul(s, x2), n2 = cmul(ms, x1);
            n1.x = fma(c, x1.x, n1.x);
            n1.y = fma(c, x1.y, n1.y);
            n2.x = fma(c, x2.x, n2.x);
            n2.y = fma(c, x2.y, n2.y);
            sA[(i - 1) * ld + col] = n1;
            sA[i * ld + col] = col == j ? make_double2(0.0, 0.0) : n2;
          }
          const int cb = i - 1 + lane;
          if (cb < M) {
            const double2 x1 = sB[(i - 1) * ld + cb], x2 = sB[i * ld + cb];
            double2 n1 = cmul(s, x2), n2 = cmul(ms, x1);
            n1.x = fma(c, x1.x, n1.x);
            n1.y = fma(c, x1.y, n1.y);
            n2.x = fma(c, x2.x, n2.x);
            n2.y = fma(c, x2.y, n2.y);
            sB[(i - 1) * ld + cb] = n1;
            sB[i * ld + cb] = n2;
          }
          if (lane < 3) {
            const double2 x1 = sF[lane * M + i - 1], x2 = sF[lane * M + i];
            double2 n1 = cmul(s, x2), n2 = cmul(ms, x1);
            n1.x = fma(c, x1.x, n1.x);
            n1.y = fma(c, x1.y, n1.y);
            n2.x = fma(c, x2.x, n2.x);
            n2.y = fma(c, x2.y, n2.y);
            sF[lane * M + i - 1] = n1;
            sF[lane * M + i] = n2;
          }
        }
        wave_sync_lds();
        // right rotation of columns i-1, i: zero the fill B[i][i-1]
        double c2;
        double2 s2;
        givens_right(sB[i * ld + i - 1], sB[i * ld + i], c2, s2);
        const double2 ms2 = make_double2(-s2.x, s2.y);  // -conj(s2)
        if (lane < M) {
          const int r = lane;
          {
            const double2 x1 = sA[r * ld + i - 1], x2 = sA[r * ld + i];
            // [x1, x2] S = [c x1 - conj(s) x2, s x1 + c x2]
            double2 n1 = cmul(ms2, x2), n2 = cmul(s2, x1);
            n1.x = fma(c2, x1.x, n1.x);
            n1.y = fma(c2, x1.y, n1.y);
            n2.x = fma(c2, x2.x, n2.x);
            n2.y = fma(c2, x2.y, n2.y);
            sA[r * ld + i - 1] = n1;
            sA[r * ld + i] = n2;
          }
          if (r <= i) {
            const double2 x1 = sB[r * ld + i - 1], x2 = sB[r * ld + i];
            double2 n1 = cmul(ms2, x2), n2 = cmul(s2, x1);
            n1.x = fma(c2, x1.x, n1.x);
            n1.y = fma(c2, x1.y, n1.y);
            n2.x = fma(c2, x2.x, n2.x);
            n2.y = fma(c2, x2.y, n2.y);
            sB[r * ld + i - 1] = r == i ? make_double2(0.0, 0.0) : n1;
            sB[r * ld + i] = n2;
          }
        }
        if (lane == 0) {
          rec[3 * nrec + 0] = c2;
          rec[3 * nrec + 1] = s2.x;
          rec[3 * nrec + 2] = s2.y;
        }
        ++nrec;
        wave_sync_lds();
      }
    }
  }
  __syncthreads();
  // H and T column-major with exact zeros below the (sub)diagonal
  for (int e = tid; e < M * M; e += blockDim.x) {
    const int c = e / M, r = e % M;
    H[e] = r <= c + 1 ? sA[r * ld + c] : make_double2(0.0, 0.0);
    T[e] = r <= c ? sB[r * ld + c] : make_double2(0.0, 0.0);
  }
  for (int e = tid; e < 3 * M; e += blockDim.x) f[e] = sF[e];
}

// ------------------------------------------------- accumulation of Z
// Z = product of the recorded right rotations, row by row (thread r owns row
// r in LDS); the rotations of one column sweep move leftwards, so the column
// they share is carried in registers.
__device__ __forceinline__ size_t wfrag_index(int row, int col, int Kp);

__global__ __launch_bounds__(64) void k_pencil_z(int M, int Mp, int Kp,
                                                 const double* __restrict__ rec,
                                                 double2* __restrict__ Z,
                                                 double2* __restrict__ Zf) {
  extern __shared__ double2 sZ[];
  const int ld = M + 1;
  const int r = threadIdx.x;
  if (r < M) {
    for (int c = 0; c < M; ++c) sZ[r * ld + c] = make_double2(c == r ? 1.0 : 0.0, 0.0);
    int idx = 0;
    for (int j = 0; j + 2 < M; ++j) {
      double2 carry = sZ[r * ld + M - 1];
      for (int i = M - 1; i >= j + 2; --i) {
        const double c = rec[3 * idx], sx = rec[3 * idx + 1], sy = rec[3 * idx + 2];
        ++idx;
        const double2 s = make_double2(sx, sy), ms = make_double2(-sx, sy);
        const double2 x1 = sZ[r * ld + i - 1], x2 = carry;
        double2 n1 = cmul(ms, x2), n2 = cmul(s, x1);
        n1.x = fma(c, x1.x, n1.x);
        n1.y = fma(c, x1.y, n1.y);
        n2.x = fma(c, x2.x, n2.x);
        n2.y = fma(c, x2.y, n2.y);
        sZ[r * ld + i] = n2;
        carry = n1;
      }
      sZ[r * ld + j + 1] = carry;
    }
    for (int c = 0; c < M; ++c) Z[(size_t)r * M + c] = sZ[r * ld + c];
  }
  // the same matrix in MFMA A-fragment order, zero padded to Mp x Kp
  __syncthreads();
  for (int e = threadIdx.x; e < Mp * Kp; e += blockDim.x) {
    const int rr = e / Kp, c = e % Kp;
    Zf[wfrag_index(rr, c, Kp)] = (rr < M && c < M) ? sZ[rr * ld + c] : make_double2(0.0, 0.0);
  }
}

// ------------------------------------------- stacked matrices for MFMA
// blockIdx.x = 0..3: K_M, C_M, A0, G_cc into rows b Mp .. of W; blockIdx.x =
// 4: the last tile of W (rows conj(g_i) and F_i = G[i][c block]) and the
// 3 x 3 constants (Re G_ee, E, N0).  W is stored in MFMA A-fragment order:
// W_frag[(tile * Kp/4 + kk) * 64 + l] = W[16 tile + l % 16][4 kk + l / 16].
__device__ __forceinline__ size_t wfrag_index(int row, int col, int Kp) {
  const int rt = row >> 4, kk = col >> 2;
  const int l = (row & 15) + 16 * (col & 3);
  return ((size_t)rt * (Kp / 4) + kk) * 64 + l;
}

__global__ __launch_bounds__(256) void k_pencil_layout(
    int M, int Mp, int Kp, const double2* __restrict__ KM, const double2* __restrict__ CM,
    const double2* __restrict__ A0, const double2* __restrict__ G, const double2* __restrict__ g,
    const double* __restrict__ E, const double* __restrict__ N0, double2* __restrict__ W,
    double* __restrict__ S) {
  const int tid = threadIdx.x, b = blockIdx.x;
  const int ldG = 2 * M + 3;
  if (b < 4) {
    for (int e = tid; e < Mp * Kp; e += blockDim.x) {
      const int r = e / Kp, c = e % Kp;
      double2 v = make_double2(0.0, 0.0);
      if (r < M && c < M) {
        if (b == 0) v = KM[r * M + c];
        else if (b == 1) v = CM[r * M + c];
        else if (b == 2) v = A0[r * M + c];
        else v = G[(size_t)(3 + M + r) * ldG + 3 + M + c];
      }
      W[wfrag_index(b * Mp + r, c, Kp)] = v;
    }
  } else {
    for (int e = tid; e < 16 * Kp; e += blockDim.x) {
      const int q = e / Kp, c = e % Kp;
      double2 v = make_double2(0.0, 0.0);
      if (c < M) {
        if (q < 3) v = cconj(g[q * M + c]);                            // g_q^H a = conj(g_q) . a
        else if (q < 6) v = G[(size_t)(q - 3) * ldG + 3 + M + c];      // (F a)_i
      }
      W[wfrag_index(4 * Mp + q, c, Kp)] = v;
    }
    if (tid < 9) {
      S[tid] = G[(size_t)(tid / 3) * ldG + tid % 3].x;
      S[9 + tid] = E[tid];
      S[18 + tid] = N0[tid];
    }
  }
}

hipError_t pencil_reduce_launch(int M, const double* A0, const double* CM, const double* KM,
                                const double* G, const double* g, const double* E,
                                const double* N0, void* buf, hipStream_t st) {
  const PencilLayout L = pencil_layout(M);
  char* base = static_cast<char*>(buf);
  double2* H = reinterpret_cast<double2*>(base + L.H);
  double2* T = reinterpret_cast<double2*>(base + L.T);
  double2* f = reinterpret_cast<double2*>(base + L.f);
  double2* Z = reinterpret_cast<double2*>(base + L.Z);
  double2* Zf = reinterpret_cast<double2*>(base + L.Zf);
  double2* W = reinterpret_cast<double2*>(base + L.W);
  double* S = reinterpret_cast<double*>(base + L.S);
  double* rec = reinterpret_cast<double*>(base + L.rec);
  const size_t lds1 = ((size_t)2 * M * (M + 1) + 4 * M) * sizeof(double2);
  hipLaunchKernelGGL(k_pencil_reduce, dim3(1), dim3(256), lds1, st, M,
                     reinterpret_cast<const double2*>(A0), reinterpret_cast<const double2*>(CM),
                     reinterpret_cast<const double2*>(g), H, T, f, rec);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds2 = (size_t)M * (M + 1) * sizeof(double2);
  hipLaunchKernelGGL(k_pencil_z, dim3(1), dim3(64), lds2, st, M, L.Mp, L.Kp, rec, Z, Zf);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pencil_layout, dim3(5), dim3(256), 0, st, M, L.Mp, L.Kp,
                     reinterpret_cast<const double2*>(KM), reinterpret_cast<const double2*>(CM),
                     reinterpret_cast<const double2*>(A0), reinterpret_cast<const double2*>(G),
                     reinterpret_cast<const double2*>(g), E, N0, W, S);
  return hipGetLastError();
}

// ------------------------------------------------------------ the sweep
namespace {

template <int L>
__device__ __forceinline__ double seg_bc(double v, int src) {
  if constexpr (L == 64) return bcast(v, __builtin_amdgcn_readfirstlane(src));
  else return shfl_d(v, src);
}
template <int L>
__device__ __forceinline__ double2 seg_bc2(double2 v, int src) {
  return make_double2(seg_bc<L>(v.x, src), seg_bc<L>(v.y, src));
}
// value of the lane 16 / 32 lanes away (permlane swaps)
__device__ __forceinline__ double other16(double x, int wl) {
  double a, b;
  swap16_d(x, a, b);
  return (wl & 16) ? a : b;
}
__device__ __forceinline__ double other32(double x, int wl) {
  double a, b;
  swap32_d(x, a, b);
  return (wl & 32) ? a : b;
}

constexpr int kPairI[6] = {0, 0, 0, 1, 1, 2};
constexpr int kPairJ[6] = {0, 1, 2, 1, 2, 2};

__device__ __forceinline__ int pair_of(int i, int j) {
  if (i > j) {
    const int t = i;
    i = j;
    j = t;
  }
  return i == 0 ? j : (i == 1 ? 2 + j : 5);
}

}  // namespace

struct PencilArgs {
  int M, Mp, Kp, NT;
  const double2* H;
  const double2* T;
  const double2* f;
  const double2* Zf;
  const double2* W;
  const double* S;
  double alpha, alpha_lb;
};

template <int L>
__global__ __launch_bounds__(256) void k_sweep_pencil(PencilArgs P, const double* __restrict__ omega,
                                                      int64_t n, double* __restrict__ out,
                                                      double* __restrict__ a_out,
                                                      int32_t* __restrict__ status) {
  extern __shared__ double2 lds[];
  const int M = P.M, Kp = P.Kp, NT = P.NT;
  double2* sY = lds;                                                  // [3][Kp][16]
  double2* sEt = sY + 3 * Kp * kPenBatch;                             // [3][6][16]
  double* sPart = reinterpret_cast<double*>(sEt + 18 * kPenBatch);    // [NT][6][16]
  int* sStat = reinterpret_cast<int*>(sPart + (size_t)NT * 6 * kPenBatch);
  const int tid = threadIdx.x, wl = __lane_id(), wave = tid >> 6;
  const int ll = wl & (L - 1), base = wl - ll;
  constexpr int kSegs = 64 / L;
  const int64_t b0 = (int64_t)blockIdx.x * kPenBatch;

  // ---- 1. Hessenberg solves, one frequency per segment ------------------
  for (int rnd = 0; rnd < L / 16; ++rnd) {
    const int wloc = rnd * 4 * kSegs + wave * kSegs + wl / L;
    const int64_t gi = b0 + wloc;
    const bool valid = gi < n;
    const double om = valid ? omega[gi] : 0.0;
    const bool act = ll < M;
    auto colval = [&](int k) -> double2 {  // (H - i w T)[ll][k]
      if (!act) return make_double2(0.0, 0.0);
      const double2 h = P.H[(size_t)k * M + ll], t = P.T[(size_t)k * M + ll];
      return make_double2(fma(om, t.y, h.x), fma(-om, t.x, h.y));
    };
    double2 c = colval(M - 1);
    double2 b[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double2 fi = act ? P.f[i * M + ll] : make_double2(0.0, 0.0);
      b[i] = make_double2(-om * fi.y, om * fi.x);  // i w f_i
    }
    double2 my_l = make_double2(0.0, 0.0), my_z[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) my_z[i] = make_double2(0.0, 0.0);
    bool my_sw = false;
    bool bad = false;
    double2 a1 = M >= 2 ? colval(M - 2) : make_double2(0.0, 0.0);
    double2 a2 = M >= 3 ? colval(M - 3) : make_double2(0.0, 0.0);
    for (int k = M - 2; k >= 0; --k) {
      const double2 a = a1;
      a1 = a2;
      if (k >= 2) a2 = colval(k - 2);
      const int q = k + 1;
      double code = 0.0;
      double2 l = make_double2(0.0, 0.0), z[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) z[i] = make_double2(0.0, 0.0);
      if (ll == q) {
        // pivot between column k (a) and the carried column k+1 (c) on row
        // k+1: the larger |re| + |im| (the carried column on ties)
        const bool sw = fabs(a.x) + fabs(a.y) > fabs(c.x) + fabs(c.y);
        const double2 p = sw ? a : c, o = sw ? c : a;
        const double d = p.x * p.x + p.y * p.y;
        const bool bd = !(d > 0.0) || !isfinite(d);
        const double2 inv = crecip(p);
        l = cmul(o, inv);
#pragma unroll
        for (int i = 0; i < 3; ++i) z[i] = cmul(b[i], inv);
        code = (sw ? 1.0 : 0.0) + (bd ? 2.0 : 0.0);
        my_sw = sw;
        my_l = l;
#pragma unroll
        for (int i = 0; i < 3; ++i) my_z[i] = z[i];
      }
      const int src = base + q;
      code = seg_bc<L>(code, src);
      l = seg_bc2<L>(l, src);
#pragma unroll
      for (int i = 0; i < 3; ++i) z[i] = seg_bc2<L>(z[i], src);
      const bool sw = code == 1.0 || code == 3.0;
      bad = bad || code >= 2.0;
      if (ll < q) {
        const double2 p = sw ? a : c, o = sw ? c : a;
        c = cfms(o, l, p);
#pragma unroll
        for (int i = 0; i < 3; ++i) b[i] = cfms(b[i], p, z[i]);
      }
    }
    // z_0 in lane 0, then y = (column transforms) z by a chain over the lanes
    double2 t[3];
    {
      double code = 0.0;
      if (ll == 0) {
        const double d = c.x * c.x + c.y * c.y;
        code = (!(d > 0.0) || !isfinite(d)) ? 2.0 : 0.0;
      }
      const double2 inv = crecip(c);
#pragma unroll
      for (int i = 0; i < 3; ++i) t[i] = cmul(b[i], inv);
      bad = bad || seg_bc<L>(code, base) >= 2.0;
    }
    double2 yprev[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) yprev[i] = make_double2(0.0, 0.0);
    for (int k = 0; k + 1 < M; ++k) {
      double2 tin[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) tin[i] = seg_bc2<L>(t[i], base + k);
      if (ll == k + 1) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const double2 v = cfms(my_z[i], my_l, tin[i]);
          yprev[i] = my_sw ? v : tin[i];
          t[i] = my_sw ? tin[i] : v;
        }
      }
    }
    double2 y[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int src = base + (ll + 1 < L ? ll + 1 : ll);
      const double2 yn = make_double2(shfl_d(yprev[i].x, src), shfl_d(yprev[i].y, src));
      y[i] = ll == M - 1 ? t[i] : yn;
    }
    if (ll < Kp) {
#pragma unroll
      for (int i = 0; i < 3; ++i)
        sY[(i * Kp + ll) * kPenBatch + wloc] = (valid && act) ? y[i] : make_double2(0.0, 0.0);
    }
    if (ll == 0) sStat[wloc] = bad ? 1 : 0;
  }
  __syncthreads();

  // ---- 2a. a = Z y (MFMA), written back over y -----------------------------
  const int KB = Kp / 4, tpb = P.Mp / 16;
  {
    constexpr int kMaxJobs = 3;  // (row tiles x 3 right-hand sides) / 4 waves, M <= 64
    double4_t zr[kMaxJobs], zi[kMaxJobs];
#pragma unroll
    for (int q = 0; q < kMaxJobs; ++q) {
      const int job = wave + 4 * q;  // job = rt * 3 + j
      zr[q] = double4_t{0, 0, 0, 0};
      zi[q] = double4_t{0, 0, 0, 0};
      if (job < 3 * tpb) {
        const int rt = job / 3, j = job % 3;
        const double2* Zt = P.Zf + (size_t)rt * KB * 64 + wl;
        for (int kk = 0; kk < KB; ++kk) {
          const double2 z = Zt[(size_t)kk * 64];
          const double2 yv = sY[(j * Kp + kk * 4 + (wl >> 4)) * kPenBatch + (wl & 15)];
          zr[q] = mfma(z.x, yv.x, zr[q]);
          zr[q] = mfma(-z.y, yv.y, zr[q]);
          zi[q] = mfma(z.x, yv.y, zi[q]);
          zi[q] = mfma(z.y, yv.x, zi[q]);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kMaxJobs; ++q) {
      const int job = wave + 4 * q;
      if (job < 3 * tpb) {
        const int rt = job / 3, j = job % 3;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = rt * 16 + (wl >> 4) + 4 * v;
          if (row < Kp)
            sY[(j * Kp + row) * kPenBatch + (wl & 15)] = make_double2(zr[q][v], zi[q][v]);
        }
      }
    }
    __syncthreads();
  }

  // ---- 2b. MFMA products with the stacked matrices, contracted at once ----
  for (int rt = wave; rt < NT; rt += 4) {
    double4_t ar[3], ai[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      ar[j] = double4_t{0, 0, 0, 0};
      ai[j] = double4_t{0, 0, 0, 0};
    }
    const double2* Wt = P.W + (size_t)rt * KB * 64 + wl;
    for (int kk = 0; kk < KB; ++kk) {
      const double2 w = Wt[(size_t)kk * 64];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double2 yv = sY[(j * Kp + kk * 4 + (wl >> 4)) * kPenBatch + (wl & 15)];
        ar[j] = mfma(w.x, yv.x, ar[j]);
        ar[j] = mfma(-w.y, yv.y, ar[j]);
        ai[j] = mfma(w.x, yv.y, ai[j]);
        ai[j] = mfma(w.y, yv.x, ai[j]);
      }
    }
    if (rt < NT - 1) {
      // Re y_i^H (P y_j) for the six pairs i <= j, rows of this tile
      const int row0 = (rt % tpb) * 16;
      double part[6];
#pragma unroll
      for (int p = 0; p < 6; ++p) part[p] = 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = row0 + (wl >> 4) + 4 * v;
        if (row < M) {
          double2 yi[3];
#pragma unroll
          for (int i = 0; i < 3; ++i) yi[i] = sY[(i * Kp + row) * kPenBatch + (wl & 15)];
#pragma unroll
          for (int p = 0; p < 6; ++p) {
            const int i = kPairI[p], j = kPairJ[p];
            part[p] = fma(yi[i].x, ar[j][v], part[p]);
            part[p] = fma(yi[i].y, ai[j][v], part[p]);
          }
        }
      }
#pragma unroll
      for (int p = 0; p < 6; ++p) {
        double s = part[p] + other16(part[p], wl);
        s = s + other32(s, wl);
        if (wl < 16) sPart[(rt * 6 + p) * kPenBatch + wl] = s;
      }
    } else {
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const int row = (wl >> 4) + 4 * v;
        if (row < 6) {
#pragma unroll
          for (int j = 0; j < 3; ++j)
            sEt[(j * 6 + row) * kPenBatch + (wl & 15)] = make_double2(ar[j][v], ai[j][v]);
        }
      }
    }
  }
  __syncthreads();

  // ---- 3. tensors and certificates, one thread per frequency ---------------
  if (tid < kPenBatch && b0 + tid < n) {
    const int w = tid;
    const int64_t gi = b0 + w;
    const double om = omega[gi];
    double Q[4][6];
#pragma unroll
    for (int blk = 0; blk < 4; ++blk)
#pragma unroll
      for (int p = 0; p < 6; ++p) {
        double s = 0.0;
        for (int tb = 0; tb < tpb; ++tb) s += sPart[((blk * tpb + tb) * 6 + p) * kPenBatch + w];
        Q[blk][p] = s;
      }
    auto GA = [&](int i, int j) { return sEt[(j * 6 + i) * kPenBatch + w]; };      // g_i^H a_j
    auto FA = [&](int i, int j) { return sEt[(j * 6 + 3 + i) * kPenBatch + w]; };  // (F a_j)_i
    const double* Wee = P.S;
    const double* E = P.S + 9;
    const double* N0 = P.S + 18;
    const double a3 = P.alpha * P.alpha * P.alpha;
    double* o = out + gi * 18;
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      const int i = kPairI[p], j = kPairJ[p];
      o[p] = N0[3 * i + j] - 0.25 * a3 * Q[0][p];
      o[6 + p] = 0.25 * a3 * om * (E[3 * i + j] + Q[1][p] + GA(i, j).x + GA(j, i).x);
      double cr[3];
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const int a = u == 0 ? i : (u == 1 ? j : i);
        const int bb = u == 0 ? i : j;
        const int q = pair_of(a, bb);
        cr[u] = om * om * (Wee[3 * a + bb] + FA(a, bb).x + FA(bb, a).x + Q[3][q]) -
                om * (GA(a, bb).y + GA(bb, a).y) + Q[2][q];
      }
      o[12 + p] = a3 / (8.0 * P.alpha_lb) * (2.0 * cr[0] + 2.0 * cr[1] - 2.0 * cr[2]);
    }
    status[gi] = sStat[w] ? MPT_E_SINGULAR : 0;
  }
  if (a_out != nullptr) {
    for (int it = tid; it < kPenBatch * 3 * M; it += blockDim.x) {
      const int w = it / (3 * M), rem = it % (3 * M), i = rem / M, r = rem % M;
      const int64_t gi = b0 + w;
      if (gi < n)
        reinterpret_cast<double2*>(a_out)[(gi * 3 + i) * M + r] = sY[(i * Kp + r) * kPenBatch + w];
    }
  }
}

hipError_t pencil_sweep_launch(const mpt_pencil& pen, const double* omega, int64_t n,
                               double* out, double* a_out, int32_t* status, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int M = pen.M;
  const PencilLayout Lo = pencil_layout(M);
  PencilArgs P;
  P.M = M;
  P.Mp = Lo.Mp;
  P.Kp = Lo.Kp;
  P.NT = Lo.NT;
  P.H = reinterpret_cast<const double2*>(pen.H);
  P.T = reinterpret_cast<const double2*>(pen.T);
  P.f = reinterpret_cast<const double2*>(pen.f);
  P.Zf = reinterpret_cast<const double2*>(pen.Z) + (Lo.Zf - Lo.Z) / sizeof(double2);
  P.W = reinterpret_cast<const double2*>(pen.W);
  P.S = pen.S;
  P.alpha = pen.alpha;
  P.alpha_lb = pen.alpha_lb;
  const size_t lds = ((size_t)3 * Lo.Kp * kPenBatch + 18 * kPenBatch) * sizeof(double2) +
                     (size_t)Lo.NT * 6 * kPenBatch * sizeof(double) + kPenBatch * sizeof(int);
  const dim3 grid((unsigned)((n + kPenBatch - 1) / kPenBatch)), block(256);
  if (M <= 16)
    hipLaunchKernelGGL((k_sweep_pencil<16>), grid, block, lds, st, P, omega, n, out, a_out, status);
  else if (M <= 32)
    hipLaunchKernelGGL((k_sweep_pencil<32>), grid, block, lds, st, P, omega, n, out, a_out, status);
  else
    hipLaunchKernelGGL((k_sweep_pencil<64>), grid, block, lds, st, P, omega, n, out, a_out, status);
  return hipGetLastError();
}

}  // namespace mpt
