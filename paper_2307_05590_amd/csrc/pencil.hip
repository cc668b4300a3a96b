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
//      stacked matrices with them, on FP64 MFMA: the shared W = [K_M; C_M;
//      conj(g)] and, for each reference shift used by a frequency of the
//      batch, W_s = [Gxx; H; D'; B; F] (blocks of the residual Gram G_s of
//      Lemma 4.1 and the defect form); each output tile is contracted at once
//      with the solutions (the quadratic forms), the tiles of a shift only for
//      the frequencies that use it;
//   3. one thread per frequency combines the sums into R~, I and Delta.
#include "device_util.h"
#include "kernels.h"

namespace mpt {

constexpr int kPenBatch = 16;  // frequencies per workgroup batch
constexpr int kPenLdsM = 64;   // above this M the reduction keeps A in global memory

namespace {

// 1 / sqrt(x) for a positive normal x: v_rsq_f64 and two Newton steps
__device__ __forceinline__ double rsqrt_d(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-x * y, y, 1.0);  // 1 - x y^2
    y = fma(0.5 * y, e, y);
  }
  return y;
}

// Givens rotation [[c, s], [-conj(s), c]] (c real) with
//   [[c, s], [-conj(s), c]] [x; y] = [*; 0]:
//   c = |x| / r,  s = (x / |x|) conj(y) / r,  r^2 = |x|^2 + |y|^2;
// with t = 1 / (|x| r):  c = |x|^2 t,  s = x conj(y) t
__device__ __forceinline__ void givens_left(double2 x, double2 y, double& c, double2& s) {
  const double ax2 = x.x * x.x + x.y * x.y;
  const double ay2 = y.x * y.x + y.y * y.y;
  if (ay2 == 0.0) {
    c = 1.0;
    s = make_double2(0.0, 0.0);
    return;
  }
  if (ax2 == 0.0) {
    c = 0.0;
    s = make_double2(1.0, 0.0);
    return;
  }
  const double t = rsqrt_d(ax2 * (ax2 + ay2));
  c = ax2 * t;
  const double2 sy = cmul(x, cconj(y));
  s = make_double2(sy.x * t, sy.y * t);
}

// column rotation S = [[c, s], [-conj(s), c]] with [w, u] S = [0, *]:
//   c = |u| / r,  s = conj(w) (u / |u|) / r;  with t = 1 / (|u| r):
//   c = |u|^2 t,  s = conj(w) u t
__device__ __forceinline__ void givens_right(double2 w, double2 u, double& c, double2& s) {
  const double au2 = u.x * u.x + u.y * u.y;
  const double aw2 = w.x * w.x + w.y * w.y;
  if (aw2 == 0.0) {
    c = 1.0;
    s = make_double2(0.0, 0.0);
    return;
  }
  if (au2 == 0.0) {
    c = 0.0;
    s = make_double2(1.0, 0.0);
    return;
  }
  const double t = rsqrt_d(au2 * (au2 + aw2));
  c = au2 * t;
  const double2 sw = cmul(cconj(w), u);
  s = make_double2(sw.x * t, sw.y * t);
}

// Applies the rotations i = M-1 down to j+2 of one sweep to a vector p
// (entries j+1 .. M-1, stride `stride`) with the shared entry carried in
// registers:
//   LEFT:  [p_{i-1}; p_i] <- [[c, s], [-conj(s), c]] [p_{i-1}; p_i]
//   RIGHT: [p_{i-1}, p_i] <- [p_{i-1}, p_i] [[c, s], [-conj(s), c]]
// Four entries are loaded per LDS round trip.  rot(i, c, s) supplies the
// parameters; entries with index < zero_below are written as exact zeros.
template <bool LEFT, class Rot>
__device__ __forceinline__ void rot_chain(double2* p, int stride, int M, int j, Rot rot,
                                          int zero_below) {
  double2 carry = p[(M - 1) * stride];
  int i = M - 1;
  while (i >= j + 2) {
    const int cnt = min(4, i - (j + 1));
    double2 x[4], o[4], sv[4];
    double cv[4];
    // all loads of the group first: one LDS round trip per four rotations
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t < cnt) {
        x[t] = p[(i - 1 - t) * stride];
        rot(i - t, cv[t], sv[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t < cnt) {
        const double c = cv[t];
        const double2 s = sv[t];
        const double2 ms = make_double2(-s.x, s.y);  // -conj(s)
        double2 n1, n2;
        if (LEFT) {
          n1 = cmul(s, carry);
          n2 = cmul(ms, x[t]);
        } else {
          n1 = cmul(ms, carry);
          n2 = cmul(s, x[t]);
        }
        n1.x = fma(c, x[t].x, n1.x);
        n1.y = fma(c, x[t].y, n1.y);
        n2.x = fma(c, carry.x, n2.x);
        n2.y = fma(c, carry.y, n2.y);
        o[t] = n2;
        carry = n1;
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (t < cnt) p[(i - t) * stride] = (i - t < zero_below) ? make_double2(0.0, 0.0) : o[t];
    i -= cnt;
  }
  p[(j + 1) * stride] = (j + 1 < zero_below) ? make_double2(0.0, 0.0) : carry;
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
template <int RR>  // rows (columns) per lane of wave 0: 1 for M <= 64, 2 for M <= 128
__global__ __launch_bounds__(256) void k_pencil_reduce(PencilJob one,
                                                       const PencilJob* __restrict__ jobs) {
  const PencilJob J = jobs ? jobs[blockIdx.x] : one;
  const int M = J.M;
  const PencilLayout Lo = pencil_layout(M);
  const double2* A0 = reinterpret_cast<const double2*>(J.A0);
  const double2* CM = reinterpret_cast<const double2*>(J.CM);
  const double2* g = reinterpret_cast<const double2*>(J.g);
  double2* H = reinterpret_cast<double2*>(J.base + Lo.H);
  double2* T = reinterpret_cast<double2*>(J.base + Lo.T);
  double2* f = reinterpret_cast<double2*>(J.base + Lo.f);
  double* rec = reinterpret_cast<double*>(J.base + Lo.rec);
  extern __shared__ double2 lds[];
  const int ld = M + 1;
  // above M = 64 the two working matrices do not both fit in LDS: A is kept
  // in the pencil buffer (global memory, visible across the workgroup's
  // barriers), B in LDS
  const bool a_global = M > kPenLdsM;
  double2* sA = a_global ? reinterpret_cast<double2*>(J.base + Lo.Aw) : lds;
  double2* sB = a_global ? lds : sA + M * ld;
  double2* sF = sB + M * ld;
  double2* sV = sF + 3 * M;
  __shared__ double sBeta;
  __shared__ double2 sAlpha;
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
      double2 x[RR];
      double part = 0.0;
#pragma unroll
      for (int sl = 0; sl < RR; ++sl) {
        const int u = lane + 64 * sl;
        x[sl] = u < len ? sB[(k + u) * ld + k] : make_double2(0.0, 0.0);
        part += x[sl].x * x[sl].x + x[sl].y * x[sl].y;
      }
      const double nrm2 = wave_sum(part);
      const double2 x0 = sB[k * ld + k];
      const double ax0 = sqrt(x0.x * x0.x + x0.y * x0.y);
      const double nrm = sqrt(nrm2);
      // alpha = -(x0 / |x0|) ||x||, v = x - alpha e_1, beta = 2 / ||v||^2
      const double2 ph = ax0 > 0.0 ? make_double2(x0.x / ax0, x0.y / ax0) : make_double2(1.0, 0.0);
      const double2 alpha = make_double2(-ph.x * nrm, -ph.y * nrm);
      const double2 v0 = make_double2(x0.x - alpha.x, x0.y - alpha.y);
      const double vn2 = nrm2 - ax0 * ax0 + (v0.x * v0.x + v0.y * v0.y);
#pragma unroll
      for (int sl = 0; sl < RR; ++sl) {
        const int u = lane + 64 * sl;
        if (u < len) sV[u] = u == 0 ? v0 : x[sl];
      }
      if (lane == 0) {
        const bool refl = nrm2 > 0.0 && vn2 > 0.0;
        sBeta = refl ? 2.0 / vn2 : 0.0;
        sAlpha = refl ? alpha : x0;
      }
    }
    __syncthreads();
    const double beta = sBeta;
    const int ncol = len + M + 3;
    if (beta != 0.0) {
      for (int t = tid; t < ncol; t += blockDim.x) {
        if (t == 0) {  // the column being reduced: alpha e_1
          sB[k * ld + k] = sAlpha;
          for (int u = 1; u < len; ++u) sB[(k + u) * ld + k] = make_double2(0.0, 0.0);
          continue;
        }
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
        // v^H col with four independent partial sums
        double2 p0 = make_double2(0.0, 0.0), p1 = p0, p2 = p0, p3 = p0;
        int u = 0;
        for (; u + 3 < len; u += 4) {
          p0 = cfmac(p0, sV[u], col[u * stride]);
          p1 = cfmac(p1, sV[u + 1], col[(u + 1) * stride]);
          p2 = cfmac(p2, sV[u + 2], col[(u + 2) * stride]);
          p3 = cfmac(p3, sV[u + 3], col[(u + 3) * stride]);
        }
        for (; u < len; ++u) p0 = cfmac(p0, sV[u], col[u * stride]);
        double2 sdot = make_double2((p0.x + p1.x) + (p2.x + p3.x), (p0.y + p1.y) + (p2.y + p3.y));
        sdot.x *= beta;
        sdot.y *= beta;
        for (u = 0; u < len; ++u) col[u * stride] = cfms(col[u * stride], sV[u], sdot);
      }
    }
    __syncthreads();
  }

  // ---- Givens sweeps: A to Hessenberg form, B kept triangular ------------
  // Sweep j zeroes A[j+2.., j] by left rotations of rows (i-1, i), i = M-1
  // down to j+2; each fills B[i][i-1], which the right rotation of columns
  // (i-1, i) removes.  Left and right rotations commute as operators, so a
  // sweep is (1) its rotation parameters, then (2) A <- L A R, B <- L B R and
  // F <- L F in bulk.  The parameters need little: the left ones follow from
  // column j of A alone, and the right one of step i from three entries of B
  // as the sweep has left them,
  //   B[i-1][i-1] (untouched so far), B[i-1][i] = (B R)[i-1][i] (row i-1 is
  //   untouched by the left rotations before step i) and B[i][i], which a
  //   short scalar recursion carries from step to step;
  // so wave 0 holds, per lane r, row r of B times the right rotations so far
  // at the current column (the rows' carries), and everything moves between
  // lanes by v_readlane: no LDS round trip on the sequential path.
  // The right rotations are recorded in order for the accumulation of Z.
  double* sRot = reinterpret_cast<double*>(sV);  // recL (3 x M) then recR (3 x M)
  int nrec = 0;
  for (int j = 0; j + 2 < M; ++j) {
    // rotation i is held by lane i % 64 in slot i / 64
    double myc[RR], myc2[RR];
    double2 mys[RR], mys2[RR];
#pragma unroll
    for (int sl = 0; sl < RR; ++sl) {
      myc[sl] = myc2[sl] = 1.0;
      mys[sl] = mys2[sl] = make_double2(0.0, 0.0);
    }
    if (wave == 0) {
      double2 colj[RR], bd[RR], carry[RR], nx[RR];
#pragma unroll
      for (int sl = 0; sl < RR; ++sl) {
        const int r = lane + 64 * sl;
        const bool act = r < M;
        colj[sl] = act ? sA[r * ld + j] : make_double2(0.0, 0.0);
        bd[sl] = act ? sB[r * ld + r] : make_double2(0.0, 0.0);  // diagonal of B
        carry[sl] = act ? sB[r * ld + M - 1] : make_double2(0.0, 0.0);
        nx[sl] = act ? sB[r * ld + M - 2] : make_double2(0.0, 0.0);
      }
      // value of row r (uniform) from the lane and slot that hold it
      auto rowv = [&](const double2 (&v)[RR], int r) -> double2 {
        const int sl = r >> 6;
        double2 x = v[0];
#pragma unroll
        for (int t = 1; t < RR; ++t)
          if (sl == t) x = v[t];
        return bcast2(x, r & 63);
      };
      double2 y = rowv(colj, M - 1);
      double c1 = 1.0, c21 = 1.0;
      double2 s1 = make_double2(0.0, 0.0), s21 = make_double2(0.0, 0.0);
      double2 e_prev = make_double2(0.0, 0.0), b_prev = make_double2(0.0, 0.0);
      for (int i = M - 1; i >= j + 2; --i) {
        // left rotation i (rows i-1, i) from column j
        const double2 x = rowv(colj, i - 1);
        double c;
        double2 s;
        givens_left(x, y, c, s);
        {
          double2 ny = cmul(s, y);
          ny.x = fma(c, x.x, ny.x);
          ny.y = fma(c, x.y, ny.y);
          y = ny;
        }
        // B[i][i] before step i
        const double2 bii = rowv(bd, i);
        double2 b_i;
        if (i == M - 1) {
          b_i = bii;
        } else {
          // after left i+1: B[i][i] = c1 Bo[i][i], B[i][i+1] = c1 e_prev + s1 b_prev;
          // after right i+1: B[i][i] = c21 B[i][i] - conj(s21) B[i][i+1]
          double2 t = cmul(s1, b_prev);
          t.x = fma(c1, e_prev.x, t.x);
          t.y = fma(c1, e_prev.y, t.y);
          b_i = cmul(make_double2(-s21.x, s21.y), t);
          b_i.x = fma(c21 * c1, bii.x, b_i.x);
          b_i.y = fma(c21 * c1, bii.y, b_i.y);
        }
        const double2 F = rowv(carry, i - 1);  // B[i-1][i] before step i
        // after left i: fill w = B[i][i-1] = -conj(s) B[i-1][i-1], u = B[i][i]
        const double2 ms = make_double2(-s.x, s.y);  // -conj(s)
        const double2 w = cmul(ms, rowv(bd, i - 1));
        double2 u = cmul(ms, F);
        u.x = fma(c, b_i.x, u.x);
        u.y = fma(c, b_i.y, u.y);
        double c2;
        double2 s2;
        givens_right(w, u, c2, s2);
        if (lane == (i & 63)) {
#pragma unroll
          for (int sl = 0; sl < RR; ++sl) {
            if (sl == (i >> 6)) {
              myc[sl] = c;
              mys[sl] = s;
              myc2[sl] = c2;
              mys2[sl] = s2;
            }
          }
        }
        c1 = c;
        s1 = s;
        c21 = c2;
        s21 = s2;
        e_prev = F;
        b_prev = b_i;
        // the rows' carries: right rotation i on columns (i-1, i)
#pragma unroll
        for (int sl = 0; sl < RR; ++sl) {
          const int r = lane + 64 * sl;
          const double2 x1 = nx[sl];
          if (r < M && i - 2 >= 0) nx[sl] = sB[r * ld + i - 2];
          double2 nc = cmul(make_double2(-s2.x, s2.y), carry[sl]);
          nc.x = fma(c2, x1.x, nc.x);
          nc.y = fma(c2, x1.y, nc.y);
          carry[sl] = nc;
        }
      }
#pragma unroll
      for (int sl = 0; sl < RR; ++sl) {
        const int r = lane + 64 * sl;
        // column j done: A[j+1][j] = y, zeros below
        if (r == j + 1) sA[(j + 1) * ld + j] = y;
        if (r >= j + 2 && r < M) {
          sA[r * ld + j] = make_double2(0.0, 0.0);
          // publish the rotations of this sweep
          sRot[3 * r] = myc[sl];
          sRot[3 * r + 1] = mys[sl].x;
          sRot[3 * r + 2] = mys[sl].y;
          sRot[3 * M + 3 * r] = myc2[sl];
          sRot[3 * M + 3 * r + 1] = mys2[sl].x;
          sRot[3 * M + 3 * r + 2] = mys2[sl].y;
          const int kk = nrec + (M - 1 - r);  // recorded in the order applied
          rec[3 * kk] = myc2[sl];
          rec[3 * kk + 1] = mys2[sl].x;
          rec[3 * kk + 2] = mys2[sl].y;
        }
      }
    }
    nrec += M - 2 - j;
    __syncthreads();
    // ---- left rotations: columns j+1.. of A (wave 0, then wave 3 beyond 64
    // columns), of B (wave 1, then wave 2), F (wave 2)
    auto ldsL = [&](int i, double& c, double2& s) {
      c = sRot[3 * i];
      s = make_double2(sRot[3 * i + 1], sRot[3 * i + 2]);
    };
    auto ldsR = [&](int i, double& c, double2& s) {
      c = sRot[3 * M + 3 * i];
      s = make_double2(sRot[3 * M + 3 * i + 1], sRot[3 * M + 3 * i + 2]);
    };
    // wave 0 reads rotations 0..63 from its registers (v_readlane ignores the
    // execution mask, and slot 0 was written with the whole wave active);
    // rotations 64.. come from their published copy
    auto regL = [&](int i, double& c, double2& s) {
      if (RR > 1 && i >= 64) {
        ldsL(i, c, s);
      } else {
        c = bcast(myc[0], i);
        s = bcast2(mys[0], i);
      }
    };
    auto regR = [&](int i, double& c, double2& s) {
      if (RR > 1 && i >= 64) {
        ldsR(i, c, s);
      } else {
        c = bcast(myc2[0], i);
        s = bcast2(mys2[0], i);
      }
    };
    if (wave == 0) {
      if (j + 1 + lane < M) rot_chain<true>(sA + (j + 1 + lane), ld, M, j, regL, -1);
    } else if (wave == 1) {
      if (j + 1 + lane < M) rot_chain<true>(sB + (j + 1 + lane), ld, M, j, ldsL, -1);
    } else if (wave == 2) {
      if (lane < 3) rot_chain<true>(sF + lane * M, 1, M, j, ldsL, -1);
      if (RR > 1 && j + 65 + lane < M) rot_chain<true>(sB + (j + 65 + lane), ld, M, j, ldsL, -1);
    } else if (RR > 1) {
      if (j + 65 + lane < M) rot_chain<true>(sA + (j + 65 + lane), ld, M, j, ldsL, -1);
    }
    __syncthreads();
    // ---- right rotations: rows of A (waves 0, 2) and of B (waves 1, 3),
    // columns j+1..; B stays upper triangular: entries below the diagonal
    // are written as exact zeros (the fills, cancelled to rounding by the
    // bulk products)
    if (wave == 0) {
      if (lane < M) rot_chain<false>(sA + lane * ld, 1, M, j, regR, -1);
    } else if (wave == 1) {
      if (lane < M) rot_chain<false>(sB + lane * ld, 1, M, j, ldsR, lane);
    } else if (RR > 1 && wave == 2) {
      if (lane + 64 < M) rot_chain<false>(sA + (lane + 64) * ld, 1, M, j, ldsR, -1);
    } else if (RR > 1 && wave == 3) {
      if (lane + 64 < M) rot_chain<false>(sB + (lane + 64) * ld, 1, M, j, ldsR, lane + 64);
    }
    __syncthreads();
  }

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

__global__ __launch_bounds__(128) void k_pencil_z(PencilJob one, const PencilJob* __restrict__ jobs) {
  const PencilJob J = jobs ? jobs[blockIdx.x] : one;
  const int M = J.M;
  const PencilLayout Lo = pencil_layout(M);
  const int Mp = Lo.Mp, Kp = Lo.Kp;
  const double* rec = reinterpret_cast<const double*>(J.base + Lo.rec);
  double2* Z = reinterpret_cast<double2*>(J.base + Lo.Z);
  double2* Zf = reinterpret_cast<double2*>(J.base + Lo.Zf);
  extern __shared__ double2 sZ[];
  const int ld = M + 1;
  const int r = threadIdx.x;
  const int nrot = M >= 3 ? (M - 1) * (M - 2) / 2 : 0;
  // the rotation record in LDS when it fits beside Z, else read from global
  double* sRec = reinterpret_cast<double*>(sZ + M * ld);
  if (M <= kPenLdsM)
    for (int e = r; e < 3 * nrot; e += blockDim.x) sRec[e] = rec[e];
  const double* rsrc = M <= kPenLdsM ? sRec : rec;
  __syncthreads();
  if (r < M) {
    for (int c = 0; c < M; ++c) sZ[r * ld + c] = make_double2(c == r ? 1.0 : 0.0, 0.0);
    int idx0 = 0;
    for (int j = 0; j + 2 < M; ++j) {
      auto rotz = [&](int i, double& c, double2& s) {
        const int k = idx0 + (M - 1 - i);
        c = rsrc[3 * k];
        s = make_double2(rsrc[3 * k + 1], rsrc[3 * k + 2]);
      };
      rot_chain<false>(sZ + r * ld, 1, M, j, rotz, -1);
      idx0 += M - 2 - j;
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
// W is stored in MFMA A-fragment order, one 16-row tile after the other:
// W_frag[(tile * Kp/4 + kk) * 64 + l] = W[16 tile + l % 16][4 kk + l / 16].
// blockIdx.x = 0, 1: K_M, C_M (shared tiles); 2: the shared last tile (rows
// conj(g_i)) and the constants (E, N0, per shift s and Re G_s[w, w]);
// 3 + 4 k + m: shift k, m = 0..2 the blocks Gxx = G_s[XU, XU], H = G_s[CU, CU]
// and D'_s, m = 3 its last tile (rows G_s[Cw_i, XU], then G_s[Cw_i, CU]).
__device__ __forceinline__ size_t wfrag_index(int row, int col, int Kp) {
  const int rt = row >> 4, kk = col >> 2;
  const int l = (row & 15) + 16 * (col & 3);
  return ((size_t)rt * (Kp / 4) + kk) * 64 + l;
}

__global__ __launch_bounds__(256) void k_pencil_layout(PencilJob one,
                                                       const PencilJob* __restrict__ jobs) {
  const PencilJob J = jobs ? jobs[blockIdx.y] : one;
  const int M = J.M;
  const PencilLayout Lo = pencil_layout(M);
  const int Mp = Lo.Mp, Kp = Lo.Kp, tpb = Mp / 16;
  const int b = blockIdx.x;
  if (b >= 3 + 4 * J.n_ref) return;
  const double2* KM = reinterpret_cast<const double2*>(J.KM);
  const double2* CM = reinterpret_cast<const double2*>(J.CM);
  const double2* g = reinterpret_cast<const double2*>(J.g);
  double2* W = reinterpret_cast<double2*>(J.base + Lo.W);
  double* S = reinterpret_cast<double*>(J.base + Lo.S);
  const int tid = threadIdx.x;
  const int ldG = 2 * M + 3;
  if (b < 2) {
    for (int e = tid; e < Mp * Kp; e += blockDim.x) {
      const int r = e / Kp, c = e % Kp;
      double2 v = make_double2(0.0, 0.0);
      if (r < M && c < M) v = b == 0 ? KM[r * M + c] : CM[r * M + c];
      W[wfrag_index(b * Mp + r, c, Kp)] = v;
    }
  } else if (b == 2) {
    for (int e = tid; e < 16 * Kp; e += blockDim.x) {
      const int q = e / Kp, c = e % Kp;
      const double2 v = (c < M && q < 3) ? cconj(g[q * M + c]) : make_double2(0.0, 0.0);
      W[wfrag_index(2 * Mp + q, c, Kp)] = v;  // g_q^H a = conj(g_q) . a
    }
    if (tid < 9) {
      S[tid] = J.E[tid];
      S[9 + tid] = J.N0[tid];
    }
    for (int k = tid; k < J.n_ref; k += blockDim.x) {
      const double2* G = reinterpret_cast<const double2*>(J.G) + (size_t)k * ldG * ldG;
      S[18 + 10 * k] = J.s_ref[k];
      for (int t = 0; t < 9; ++t) S[18 + 10 * k + 1 + t] = G[(size_t)(t / 3) * ldG + t % 3].x;
    }
  } else {
    const int k = (b - 3) / 4, m = (b - 3) % 4;
    const double2* G = reinterpret_cast<const double2*>(J.G) + (size_t)k * ldG * ldG;
    const double2* Dq = reinterpret_cast<const double2*>(J.Dp) + (size_t)k * M * M;
    // first row of shift k's tiles (rows of 16 per tile)
    const int row0 = (Lo.NTs + k * Lo.NTr) * 16;
    if (m < 3) {
      for (int e = tid; e < Mp * Kp; e += blockDim.x) {
        const int r = e / Kp, c = e % Kp;
        double2 v = make_double2(0.0, 0.0);
        if (r < M && c < M) {
          if (m == 0) v = G[(size_t)(3 + r) * ldG + 3 + c];
          else if (m == 1) v = G[(size_t)(3 + M + r) * ldG + 3 + M + c];
          else v = Dq[r * M + c];
        }
        W[wfrag_index(row0 + m * Mp + r, c, Kp)] = v;
      }
    } else {
      for (int e = tid; e < 16 * Kp; e += blockDim.x) {
        const int q = e / Kp, c = e % Kp;
        double2 v = make_double2(0.0, 0.0);
        if (c < M) {
          if (q < 3) v = G[(size_t)q * ldG + 3 + c];              // (B a)_q
          else if (q < 6) v = G[(size_t)(q - 3) * ldG + 3 + M + c];  // (F a)_q
        }
        W[wfrag_index(row0 + 3 * Mp + q, c, Kp)] = v;
      }
    }
    (void)tpb;
  }
}

static size_t reduce_lds(int M) {
  const size_t mats = M > kPenLdsM ? 1 : 2;  // B only, or A and B
  return (mats * M * (M + 1) + 6 * (size_t)M) * sizeof(double2);
}
static size_t z_lds(int M) {
  const size_t nrot = M >= 3 ? (size_t)(M - 1) * (M - 2) / 2 : 0;
  return (size_t)M * (M + 1) * sizeof(double2) + (M > kPenLdsM ? 0 : nrot * 3 * sizeof(double));
}

hipError_t pencil_core_launch(const PencilJob& one, const PencilJob* jobs, int n_jobs, int maxM,
                              hipStream_t st) {
  // LDS for the largest requirement among M <= maxM (not monotonic at kPenLdsM)
  const int Ml = maxM < kPenLdsM ? maxM : kPenLdsM;
  size_t lds1 = reduce_lds(Ml), lds2 = z_lds(Ml);
  if (maxM > kPenLdsM) {
    lds1 = lds1 > reduce_lds(maxM) ? lds1 : reduce_lds(maxM);
    lds2 = lds2 > z_lds(maxM) ? lds2 : z_lds(maxM);
  }
  if (maxM > 64)
    hipLaunchKernelGGL((k_pencil_reduce<2>), dim3(n_jobs), dim3(256), lds1, st, one, jobs);
  else
    hipLaunchKernelGGL((k_pencil_reduce<1>), dim3(n_jobs), dim3(256), lds1, st, one, jobs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // one thread per row of Z
  hipLaunchKernelGGL(k_pencil_z, dim3(n_jobs), dim3(maxM > 64 ? 128 : 64), lds2, st, one, jobs);
  return hipGetLastError();
}

hipError_t pencil_layout_launch(const PencilJob& one, const PencilJob* jobs, int n_jobs,
                                int maxRef, hipStream_t st) {
  hipLaunchKernelGGL(k_pencil_layout, dim3(3 + 4 * maxRef, n_jobs), dim3(256), 0, st, one, jobs);
  return hipGetLastError();
}

hipError_t pencil_reduce_launch(const PencilJob& one, const PencilJob* jobs, int n_jobs, int maxM,
                                int maxRef, hipStream_t st) {
  hipError_t e = pencil_core_launch(one, jobs, n_jobs, maxM, st);
  if (e != hipSuccess) return e;
  return pencil_layout_launch(one, jobs, n_jobs, maxRef, st);
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


template <int L, int R>
__global__ __launch_bounds__(256, 3) void k_sweep_pencil(PencilArgs one,
                                                      const PencilArgs* __restrict__ objs,
                                                      const int4* __restrict__ items,
                                                      const double* __restrict__ omega, int64_t n,
                                                      double* __restrict__ out,
                                                      double* __restrict__ a_out,
                                                      int32_t* __restrict__ status) {
  extern __shared__ double2 lds[];
  int64_t b0;
  int cnt;
  PencilArgs P;
  if (items) {
    const int4 it = items[blockIdx.x];
    P = objs[it.x];
    b0 = it.y;
    cnt = it.z;
  } else {
    P = one;
    b0 = (int64_t)blockIdx.x * kPenBatch;
    cnt = (int)(n - b0 < kPenBatch ? n - b0 : kPenBatch);
  }
  const int M = P.M, Kp = P.Kp, NTs = P.NTs, NTr = P.NTr;
  double2* sY = lds;                                                  // [3][Kp][16]
  double2* sEt = sY + 3 * Kp * kPenBatch;                             // [3][12][16]
  double* sPart = reinterpret_cast<double*>(sEt + 36 * kPenBatch);    // [5][6][16]
  int* sStat = reinterpret_cast<int*>(sPart + (size_t)5 * 6 * kPenBatch);
  int* sRef = sStat + kPenBatch;   // reference shift of each frequency
  int* sList = sRef + kPenBatch;   // the distinct shifts of the batch, ascending
  int* sNList = sList + kPenBatch;
  const int tid = threadIdx.x, wl = __lane_id(), wave = tid >> 6;
  const int ll = wl & (L - 1), base = wl - ll;
  constexpr int kSegs = 64 / L;

  // ---- 1. Hessenberg solves, one frequency per segment of L lanes; lane ll
  //         holds rows ll + L s, s < R (R = 2 only with L = 64) -------------
  for (int rnd = 0; rnd < L / 16; ++rnd) {
    const int wloc = rnd * 4 * kSegs + wave * kSegs + wl / L;
    const int64_t gi = b0 + wloc;
    const bool valid = wloc < cnt;
    const double om = valid ? omega[gi] : 0.0;
    auto colval = [&](int k, int sl) -> double2 {  // (H - i w T)[row][k]
      const int row = ll + L * sl;
      if (row >= M) return make_double2(0.0, 0.0);
      const double2 h = P.H[(size_t)k * M + row], t = P.T[(size_t)k * M + row];
      return make_double2(fma(om, t.y, h.x), fma(-om, t.x, h.y));
    };
    double2 c[R], b[R][3], my_l[R], my_z[R][3], a1[R], a2[R];
    bool my_sw[R];
#pragma unroll
    for (int sl = 0; sl < R; ++sl) {
      const int row = ll + L * sl;
      c[sl] = colval(M - 1, sl);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double2 fi = row < M ? P.f[i * M + row] : make_double2(0.0, 0.0);
        b[sl][i] = make_double2(-om * fi.y, om * fi.x);  // i w f_i
        my_z[sl][i] = make_double2(0.0, 0.0);
      }
      my_l[sl] = make_double2(0.0, 0.0);
      my_sw[sl] = false;
      a1[sl] = M >= 2 ? colval(M - 2, sl) : make_double2(0.0, 0.0);
      a2[sl] = M >= 3 ? colval(M - 3, sl) : make_double2(0.0, 0.0);
    }
    bool bad = false;
    for (int k = M - 2; k >= 0; --k) {
      double2 a[R];
#pragma unroll
      for (int sl = 0; sl < R; ++sl) {
        a[sl] = a1[sl];
        a1[sl] = a2[sl];
        if (k >= 2) a2[sl] = colval(k - 2, sl);
      }
      const int q = k + 1, qs = q / L, ql = q % L;  // row q: lane ql, slot qs
      double code = 0.0;
      double2 l = make_double2(0.0, 0.0), z[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) z[i] = make_double2(0.0, 0.0);
      if (ll == ql) {
        double2 aq = a[0], cq = c[0], bq[3] = {b[0][0], b[0][1], b[0][2]};
        if (R == 2 && qs == 1) {
          aq = a[R - 1];
          cq = c[R - 1];
#pragma unroll
          for (int i = 0; i < 3; ++i) bq[i] = b[R - 1][i];
        }
        // pivot between column k (a) and the carried column k+1 (c) on row
        // k+1: the larger |re| + |im| (the carried column on ties)
        const bool sw = fabs(aq.x) + fabs(aq.y) > fabs(cq.x) + fabs(cq.y);
        const double2 p = sw ? aq : cq, o = sw ? cq : aq;
        const double d = p.x * p.x + p.y * p.y;
        const bool bd = !(d > 0.0) || !isfinite(d);
        const double2 inv = crecip(p);
        l = cmul(o, inv);
#pragma unroll
        for (int i = 0; i < 3; ++i) z[i] = cmul(bq[i], inv);
        code = (sw ? 1.0 : 0.0) + (bd ? 2.0 : 0.0);
#pragma unroll
        for (int sl = 0; sl < R; ++sl) {
          if (sl == qs) {
            my_sw[sl] = sw;
            my_l[sl] = l;
#pragma unroll
            for (int i = 0; i < 3; ++i) my_z[sl][i] = z[i];
          }
        }
      }
      const int src = base + ql;
      code = seg_bc<L>(code, src);
      l = seg_bc2<L>(l, src);
#pragma unroll
      for (int i = 0; i < 3; ++i) z[i] = seg_bc2<L>(z[i], src);
      const bool sw = code == 1.0 || code == 3.0;
      bad = bad || code >= 2.0;
#pragma unroll
      for (int sl = 0; sl < R; ++sl) {
        if (ll + L * sl < q) {
          const double2 p = sw ? a[sl] : c[sl], o = sw ? c[sl] : a[sl];
          c[sl] = cfms(o, l, p);
#pragma unroll
          for (int i = 0; i < 3; ++i) b[sl][i] = cfms(b[sl][i], p, z[i]);
        }
      }
    }
    // z_0 at row 0 (lane 0, slot 0), then y = (column transforms) z by a
    // chain over the rows
    double2 t[R][3];
    {
      double code = 0.0;
      if (ll == 0) {
        const double d = c[0].x * c[0].x + c[0].y * c[0].y;
        code = (!(d > 0.0) || !isfinite(d)) ? 2.0 : 0.0;
      }
      const double2 inv = crecip(c[0]);
#pragma unroll
      for (int i = 0; i < 3; ++i) t[0][i] = cmul(b[0][i], inv);
#pragma unroll
      for (int sl = 1; sl < R; ++sl)
#pragma unroll
        for (int i = 0; i < 3; ++i) t[sl][i] = make_double2(0.0, 0.0);
      bad = bad || seg_bc<L>(code, base) >= 2.0;
    }
    double2 yprev[R][3];
#pragma unroll
    for (int sl = 0; sl < R; ++sl)
#pragma unroll
      for (int i = 0; i < 3; ++i) yprev[sl][i] = make_double2(0.0, 0.0);
    for (int k = 0; k + 1 < M; ++k) {
      const int ks = k / L, kl = k % L;
      const int q = k + 1, qs = q / L, ql = q % L;
      double2 tin[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double2 tsel = (R == 2 && ks == 1) ? t[R - 1][i] : t[0][i];
        tin[i] = seg_bc2<L>(tsel, base + kl);
      }
      if (ll == ql) {
#pragma unroll
        for (int sl = 0; sl < R; ++sl) {
          if (sl == qs) {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
              const double2 v = cfms(my_z[sl][i], my_l[sl], tin[i]);
              yprev[sl][i] = my_sw[sl] ? v : tin[i];
              t[sl][i] = my_sw[sl] ? tin[i] : v;
            }
          }
        }
      }
    }
    // row r takes y_r from row r + 1's yprev; row M - 1 its own t
    double2 y[R][3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if constexpr (R == 1) {
        const int src = base + (ll + 1 < L ? ll + 1 : ll);
        const double2 yn = make_double2(shfl_d(yprev[0][i].x, src), shfl_d(yprev[0][i].y, src));
        y[0][i] = ll == M - 1 ? t[0][i] : yn;
      } else {
        const int src = (ll + 1) & 63;
        const double2 ya = make_double2(shfl_d(yprev[0][i].x, src), shfl_d(yprev[0][i].y, src));
        const double2 yb = make_double2(shfl_d(yprev[R - 1][i].x, src),
                                        shfl_d(yprev[R - 1][i].y, src));
        y[0][i] = ll < 63 ? ya : yb;
        y[R - 1][i] = yb;
#pragma unroll
        for (int sl = 0; sl < R; ++sl)
          if (ll + L * sl == M - 1) y[sl][i] = t[sl][i];
      }
    }
#pragma unroll
    for (int sl = 0; sl < R; ++sl) {
      const int row = ll + L * sl;
      if (row < Kp) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
          sY[(i * Kp + row) * kPenBatch + wloc] =
              (valid && row < M) ? y[sl][i] : make_double2(0.0, 0.0);
      }
    }
    if (ll == 0) {
      sStat[wloc] = bad ? 1 : 0;
      // reference shift: the largest s_k <= w (s_0 = 0)
      int kr = 0;
      for (int k = 1; k < P.n_ref; ++k)
        if (P.S[18 + 10 * k] <= om) kr = k;
      sRef[wloc] = valid ? kr : -1;
    }
  }
  __syncthreads();
  if (tid == 0) {
    int nl = 0, last = -1;
    for (;;) {  // ascending distinct shifts of the valid frequencies
      int nxt = 1 << 30;
      for (int w = 0; w < cnt; ++w)
        if (sRef[w] > last && sRef[w] < nxt) nxt = sRef[w];
      if (nxt == (1 << 30)) break;
      sList[nl++] = nxt;
      last = nxt;
    }
    *sNList = nl;
  }
  __syncthreads();

  // ---- 2a. a = Z y (MFMA), written back over y -----------------------------
  const int KB = Kp / 4, tpb = P.Mp / 16;
  {
    constexpr int kMaxJobs = R == 2 ? 5 : 3;  // (row tiles x 3 right-hand sides) / 4 waves
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

  // ---- 2b. MFMA products with the stacked matrices, contracted at once.
  // Jobs: one per quadratic-form block (K_M, C_M; then Gxx, H, D' for each
  // shift of the batch), which takes the block's row tiles in order and sums
  // their contractions in registers, and one per remaining tile (g; B and F
  // for each shift); a shift's results are kept only for the frequencies
  // that use it. --------
  const int nlist = *sNList;
  const int njobs = 3 + 4 * nlist;
  for (int job = wave; job < njobs; job += 4) {
    int rt0, blk, kr = -1;  // first W tile; quadratic-form block, or -1 for a single tile
    if (job < 3) {
      blk = job < 2 ? job : -1;
      rt0 = job < 2 ? job * tpb : NTs - 1;
    } else {
      const int u = (job - 3) / 4, q = (job - 3) % 4;
      kr = sList[u];
      blk = q < 3 ? 2 + q : -1;
      rt0 = NTs + kr * NTr + q * tpb;
    }
    const int col = wl & 15;
    const bool keep = kr < 0 || (col < cnt && sRef[col] == kr);
    const int ntile = blk >= 0 ? tpb : 1;
    double acc[6];
#pragma unroll
    for (int p = 0; p < 6; ++p) acc[p] = 0.0;
    for (int tt = 0; tt < ntile; ++tt) {
      double4_t ar[3], ai[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        ar[j] = double4_t{0, 0, 0, 0};
        ai[j] = double4_t{0, 0, 0, 0};
      }
      const double2* Wt = P.W + (size_t)(rt0 + tt) * KB * 64 + wl;
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
      if (blk >= 0) {
        // Re y_i^H (P y_j) for the six pairs i <= j, rows of this tile
        const int row0 = tt * 16;
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
          acc[p] += s;
        }
      } else if (keep) {
        const int rb = kr < 0 ? 0 : 6;  // rows of sEt: shared tile, then the shift's
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          const int row = (wl >> 4) + 4 * v;
          if (row < 6) {
#pragma unroll
            for (int j = 0; j < 3; ++j)
              sEt[(j * 12 + rb + row) * kPenBatch + (wl & 15)] = make_double2(ar[j][v], ai[j][v]);
          }
        }
      }
    }
    if (blk >= 0 && wl < 16 && keep) {
#pragma unroll
      for (int p = 0; p < 6; ++p) sPart[(blk * 6 + p) * kPenBatch + wl] = acc[p];
    }
  }
  __syncthreads();

  // ---- 3. tensors and certificates, one thread per frequency ---------------
  if (tid < cnt) {
    const int w = tid;
    const int64_t gi = b0 + w;
    const double om = omega[gi];
    double Q[5][6];  // K_M, C_M, Gxx, H, D'
#pragma unroll
    for (int blk = 0; blk < 5; ++blk)
#pragma unroll
      for (int p = 0; p < 6; ++p) Q[blk][p] = sPart[(blk * 6 + p) * kPenBatch + w];
    auto GA = [&](int i, int j) { return sEt[(j * 12 + i) * kPenBatch + w]; };      // g_i^H a_j
    auto BA = [&](int i, int j) { return sEt[(j * 12 + 6 + i) * kPenBatch + w]; };  // (B a_j)_i
    auto FA = [&](int i, int j) { return sEt[(j * 12 + 9 + i) * kPenBatch + w]; };  // (F a_j)_i
    const double* E = P.S;
    const double* N0 = P.S + 9;
    const double* Wee = P.S + 18 + 10 * sRef[w] + 1;
    const double a3 = P.alpha * P.alpha * P.alpha;
    double* o = out + gi * 18;
    double nn[3], ee[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) ee[i] = sqrt(fmax(Q[4][pair_of(i, i)], 0.0));
    double crd[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int q = pair_of(i, i);
      crd[i] = om * om * (Wee[4 * i] + 2.0 * FA(i, i).x + Q[3][q]) - 2.0 * om * BA(i, i).y +
               Q[2][q];
      nn[i] = sqrt(fmax(crd[i], 0.0));
    }
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      const int i = kPairI[p], j = kPairJ[p];
      o[p] = N0[3 * i + j] - 0.25 * a3 * Q[0][p];
      o[6 + p] = 0.25 * a3 * om * (E[3 * i + j] + Q[1][p] + GA(i, j).x + GA(j, i).x);
      // Re c_ij = w^2 [W_ij + Re(F a_j)_i + Re(F a_i)_j + Re a_i^H H a_j]
      //           - w [Im (B a_j)_i + Im (B a_i)_j] + Re a_i^H Gxx a_j
      const double cij = om * om * (Wee[3 * i + j] + FA(i, j).x + FA(j, i).x + Q[3][p]) -
                         om * (BA(i, j).y + BA(j, i).y) + Q[2][p];
      o[12 + p] = a3 / (8.0 * P.alpha_lb) * (2.0 * crd[i] + 2.0 * crd[j] - 2.0 * cij) +
                  0.25 * a3 * (nn[i] * ee[j] + nn[j] * ee[i]);
    }
    status[gi] = sStat[w] ? MPT_E_SINGULAR : 0;
  }
  if (a_out != nullptr) {
    for (int it = tid; it < kPenBatch * 3 * M; it += blockDim.x) {
      const int w = it / (3 * M), rem = it % (3 * M), i = rem / M, r = rem % M;
      const int64_t gi = b0 + w;
      if (w < cnt)
        reinterpret_cast<double2*>(a_out)[(gi * 3 + i) * M + r] = sY[(i * Kp + r) * kPenBatch + w];
    }
  }
}

PencilArgs pencil_args(const mpt_pencil& pen) {
  const PencilLayout Lo = pencil_layout(pen.M);
  const char* base = reinterpret_cast<const char*>(pen.H);  // the buffer starts with H
  PencilArgs P;
  P.M = pen.M;
  P.Mp = Lo.Mp;
  P.Kp = Lo.Kp;
  P.NTs = Lo.NTs;
  P.NTr = Lo.NTr;
  P.n_ref = pen.n_ref;
  P.H = reinterpret_cast<const double2*>(base + Lo.H);
  P.T = reinterpret_cast<const double2*>(base + Lo.T);
  P.f = reinterpret_cast<const double2*>(base + Lo.f);
  P.Zf = reinterpret_cast<const double2*>(base + Lo.Zf);
  P.W = reinterpret_cast<const double2*>(base + Lo.W);
  P.S = reinterpret_cast<const double*>(base + Lo.S);
  P.alpha = pen.alpha;
  P.alpha_lb = pen.alpha_lb;
  return P;
}

// Kp: rows of the solutions
static size_t sweep_lds(int Kp) {
  return ((size_t)3 * Kp * kPenBatch + 36 * kPenBatch) * sizeof(double2) +
         (size_t)5 * 6 * kPenBatch * sizeof(double) + (3 * kPenBatch + 1) * sizeof(int);
}

hipError_t pencil_sweep_launch(const PencilArgs& P, const double* omega, int64_t n, double* out,
                               double* a_out, int32_t* status, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const size_t lds = sweep_lds(P.Kp);
  const dim3 grid((unsigned)((n + kPenBatch - 1) / kPenBatch)), block(256);
  const PencilArgs* no = nullptr;
  const int4* ni = nullptr;
  if (P.M <= 16)
    hipLaunchKernelGGL((k_sweep_pencil<16, 1>), grid, block, lds, st, P, no, ni, omega, n, out,
                       a_out, status);
  else if (P.M <= 32)
    hipLaunchKernelGGL((k_sweep_pencil<32, 1>), grid, block, lds, st, P, no, ni, omega, n, out,
                       a_out, status);
  else if (P.M <= 64)
    hipLaunchKernelGGL((k_sweep_pencil<64, 1>), grid, block, lds, st, P, no, ni, omega, n, out,
                       a_out, status);
  else
    hipLaunchKernelGGL((k_sweep_pencil<64, 2>), grid, block, lds, st, P, no, ni, omega, n, out,
                       a_out, status);
  return hipGetLastError();
}

hipError_t pencil_sweep_items_launch(int L, const PencilArgs* objs, const int4* items,
                                     int n_items, const double* omega, double* out,
                                     int32_t* status, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  // LDS for the largest object of the bucket: Kp <= bucket, tiles <= bucket / 16
  const size_t lds = sweep_lds(L);
  const dim3 grid((unsigned)n_items), block(256);
  PencilArgs none{};
  double* no_a = nullptr;
  if (L == 16)
    hipLaunchKernelGGL((k_sweep_pencil<16, 1>), grid, block, lds, st, none, objs, items, omega,
                       (int64_t)0, out, no_a, status);
  else if (L == 32)
    hipLaunchKernelGGL((k_sweep_pencil<32, 1>), grid, block, lds, st, none, objs, items, omega,
                       (int64_t)0, out, no_a, status);
  else if (L == 64)
    hipLaunchKernelGGL((k_sweep_pencil<64, 1>), grid, block, lds, st, none, objs, items, omega,
                       (int64_t)0, out, no_a, status);
  else  // 64 < M <= 96: two rows per lane
    hipLaunchKernelGGL((k_sweep_pencil<64, 2>), grid, block, lds, st, none, objs, items, omega,
                       (int64_t)0, out, no_a, status);
  return hipGetLastError();
}

}  // namespace mpt
