// Online reduced sweep for 64 < M <= 96 (eq. (ReducedA); tensors by eqs.
// (podprealmpt), (podpimagmpt); certificates by Lemma 4.1).  The M x M system
// no longer fits in the registers of one wave, so one workgroup per frequency
// holds it in LDS:
//   - LU with partial pivoting (max |re| + |im| over the rows not yet
//     pivoted, lowest row on ties) without row swaps: pivot search and the
//     column of multipliers by wave 0, the trailing update by all waves;
//   - forward and back substitution of the three right-hand sides by wave 0
//     (wave-level LDS ordering, no workgroup barriers);
//   - the five reduced mat-vecs with one thread per (row, vector), reading
//     the Hermitian matrices column-wise (coalesced) and conjugating;
//   - the 54 quadratic-form sums in fixed order, one thread per slot.
#include "device_util.h"
#include "kernels.h"

namespace mpt {

constexpr int kBigMaxM = 96;
constexpr int kBigThreads = 256;
constexpr int kBigLd = kBigMaxM + 1;  // padded LDS row

__constant__ int kBPi[6] = {0, 0, 0, 1, 1, 2};
__constant__ int kBPj[6] = {0, 1, 2, 1, 2, 2};

__device__ __forceinline__ int bpair(int i, int j) {
  if (i > j) { const int t = i; i = j; j = t; }
  return i == 0 ? j : (i == 1 ? 2 + j : 5);
}

__global__ __launch_bounds__(kBigThreads) void k_sweep_big(const mpt_rom R,
                                                           const double* __restrict__ omega,
                                                           int64_t n, double* __restrict__ out,
                                                           double* __restrict__ a_out,
                                                           int32_t* __restrict__ status) {
  extern __shared__ double2 sA[];  // M rows x kBigLd; reused for the mat-vec results
  __shared__ double2 sB[3][kBigMaxM];
  __shared__ double2 sX[3][kBigMaxM];
  __shared__ double2 sL[kBigMaxM];     // multipliers of the current step
  __shared__ int sPiv[kBigMaxM];       // pivot row of step k
  __shared__ int sDone[kBigMaxM];
  __shared__ int sBad;
  __shared__ double sQ[64];
  const int tid = threadIdx.x, lane = __lane_id(), wave = tid >> 6;
  const int M = R.M;
  const int ldG = 2 * M + 3;
  const double2* A0 = reinterpret_cast<const double2*>(R.A0);
  const double2* CM = reinterpret_cast<const double2*>(R.CM);
  const double2* KM = reinterpret_cast<const double2*>(R.KM);
  const double2* gv = reinterpret_cast<const double2*>(R.g);
  const double a3 = R.alpha * R.alpha * R.alpha;

  for (int64_t k_om = blockIdx.x; k_om < n; k_om += gridDim.x) {
    const double om = omega[k_om];
    // reference shift of this frequency: the largest s_ref[k] <= om
    int kref = 0;
    for (int j = 1; j < R.n_ref; ++j)
      if (R.s_ref[j] <= om) kref = j;
    const double2* G = reinterpret_cast<const double2*>(R.G) + (size_t)kref * ldG * ldG;
    const double2* Dq = reinterpret_cast<const double2*>(R.Dp) + (size_t)kref * M * M;
    // ---- A = A0 - i w C_M (row r = conj of column r), rhs i w g_i -------
    for (int e = tid; e < M * M; e += kBigThreads) {
      const int j = e / M, r = e % M;  // consecutive threads: consecutive r
      const double2 a0 = cconj(A0[j * M + r]);
      const double2 c = cconj(CM[j * M + r]);
      sA[r * kBigLd + j] = make_double2(fma(om, c.y, a0.x), fma(-om, c.x, a0.y));
    }
    for (int e = tid; e < 3 * M; e += kBigThreads) {
      const int i = e / M, r = e % M;
      const double2 gg = gv[i * M + r];
      sB[i][r] = make_double2(-om * gg.y, om * gg.x);
    }
    for (int r = tid; r < M; r += kBigThreads) sDone[r] = 0;
    if (tid == 0) sBad = 0;
    __syncthreads();
    // ---- LU: step k eliminates column k below the (virtual) pivot row ----
    for (int k = 0; k < M; ++k) {
      if (wave == 0) {
        double best = -1.0;
        int bi = M;
        for (int r = lane; r < M; r += 64) {
          if (!sDone[r]) {
            const double2 v = sA[r * kBigLd + k];
            const double val = fabs(v.x) + fabs(v.y);
            if (val > best || (val == best && r < bi) || val != val) {
              best = val != val ? 1e308 : val;  // NaN: take it and flag below
              bi = r;
            }
          }
        }
        const double wbest = wave_max(best);
        const uint64_t mk = __ballot(best == wbest && bi < M);
        // lowest row among the lanes holding the maximum
        int p = M;
        for (uint64_t m2 = mk; m2; m2 &= m2 - 1) {
          const int ln = __ffsll((unsigned long long)m2) - 1;
          const int cand = __builtin_amdgcn_readlane(bi, ln);
          p = cand < p ? cand : p;
        }
        const double2 piv = sA[p * kBigLd + k];
        const double d = piv.x * piv.x + piv.y * piv.y;
        const bool bad = !(d > 0.0) || !isfinite(d);
        const double2 inv = crecip(piv);
        for (int r = lane; r < M; r += 64) {
          if (!sDone[r] && r != p) {
            const double2 l = cmul(sA[r * kBigLd + k], inv);
            sL[r] = l;
            sA[r * kBigLd + k] = l;  // L factor kept in place
          }
        }
        if (lane == 0) {
          sPiv[k] = p;
          sDone[p] = 1;
          if (bad) sBad = 1;
        }
      }
      __syncthreads();
      const int p = sPiv[k];
      const int W = M - k - 1 + 3;  // trailing columns and the three rhs
      for (int e = tid; e < M * W; e += kBigThreads) {
        const int r = e / W, c = e % W;
        if (sDone[r]) continue;  // pivot rows (including p) stay
        const double2 l = sL[r];
        if (c < M - k - 1) {
          const int j = k + 1 + c;
          sA[r * kBigLd + j] = cfms(sA[r * kBigLd + j], l, sA[p * kBigLd + j]);
        } else {
          const int i = c - (M - k - 1);
          sB[i][r] = cfms(sB[i][r], l, sB[i][p]);
        }
      }
      __syncthreads();
    }
    // ---- back substitution (wave 0): unknown k from pivot row sPiv[k] ----
    if (wave == 0) {
      for (int k = M - 1; k >= 0; --k) {
        const int p = sPiv[k];
        const double2 inv = crecip(sA[p * kBigLd + k]);
        double2 xk[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) xk[i] = cmul(sB[i][p], inv);
        if (lane == 0)
#pragma unroll
          for (int i = 0; i < 3; ++i) sX[i][k] = xk[i];
        // rows pivoted before step k hold U entries in column k
        for (int kk = lane; kk < k; kk += 64) {
          const int q = sPiv[kk];
          const double2 u = sA[q * kBigLd + k];
#pragma unroll
          for (int i = 0; i < 3; ++i) sB[i][q] = cfms(sB[i][q], u, xk[i]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    __syncthreads();
    // ---- mat-vecs: K_M a_i, C_M a_i, Gxx a_i, H a_i, D' a_i into the A region
    // (Gxx = G_s[XU, XU], H = G_s[CU, CU]) ----------------------------------
    double2* sKa = sA;              // [3][M]
    double2* sCa = sA + 3 * kBigMaxM;
    double2* sAa = sA + 6 * kBigMaxM;
    double2* sHa = sA + 9 * kBigMaxM;
    double2* sDa = sA + 12 * kBigMaxM;
    for (int e = tid; e < 3 * M; e += kBigThreads) {
      const int i = e / M, r = e % M;
      double2 ka = make_double2(0.0, 0.0), ca = ka, aa = ka, ha = ka, da = ka;
      for (int j = 0; j < M; ++j) {
        const double2 xj = sX[i][j];
        ka = cfma(ka, cconj(KM[j * M + r]), xj);
        ca = cfma(ca, cconj(CM[j * M + r]), xj);
        aa = cfma(aa, cconj(G[(size_t)(3 + j) * ldG + 3 + r]), xj);
        ha = cfma(ha, cconj(G[(size_t)(3 + M + j) * ldG + 3 + M + r]), xj);
        da = cfma(da, cconj(Dq[j * M + r]), xj);
      }
      sKa[i * kBigMaxM + r] = ka;
      sCa[i * kBigMaxM + r] = ca;
      sAa[i * kBigMaxM + r] = aa;
      sHa[i * kBigMaxM + r] = ha;
      sDa[i * kBigMaxM + r] = da;
    }
    __syncthreads();
    // ---- 54 quadratic-form slots (the register kernel's order), one thread
    // each, fixed order ---------------------------------------------------
    if (tid < 54) {
      const int sl = tid;
      double acc = 0.0;
      if (sl < 24) {
        const int q = sl % 6, kind = sl / 6;
        const int i = kBPi[q], j = kBPj[q];
        const double2* Y = kind == 0 ? sKa : (kind == 1 ? sCa : (kind == 2 ? sAa : sHa));
        for (int r = 0; r < M; ++r) acc += cmulc(sX[i][r], Y[j * kBigMaxM + r]).x;
      } else if (sl < 33) {  // Re g_i^H a_j
        const int u = sl - 24, i = u / 3, j = u % 3;
        double2 s2 = make_double2(0.0, 0.0);
        for (int r = 0; r < M; ++r) s2 = cfmac(s2, gv[i * M + r], sX[j][r]);
        acc = s2.x;
      } else if (sl < 42) {  // Re (F a_j)_i
        const int u = sl - 33, i = u / 3, j = u % 3;
        double2 s2 = make_double2(0.0, 0.0);
        for (int r = 0; r < M; ++r) s2 = cfma(s2, G[(size_t)i * ldG + 3 + M + r], sX[j][r]);
        acc = s2.x;
      } else if (sl < 51) {  // Im (B a_j)_i
        const int u = sl - 42, i = u / 3, j = u % 3;
        double2 s2 = make_double2(0.0, 0.0);
        for (int r = 0; r < M; ++r) s2 = cfma(s2, G[(size_t)i * ldG + 3 + r], sX[j][r]);
        acc = s2.y;
      } else {  // Re a_i^H D' a_i
        const int i = sl - 51;
        for (int r = 0; r < M; ++r) acc += cmulc(sX[i][r], sDa[i * kBigMaxM + r]).x;
      }
      sQ[sl] = acc;
    }
    __syncthreads();
    // ---- outputs (same formulas as the register kernel) -----------------
    if (tid < 18) {
      const int po = tid, pp = po % 6, i = kBPi[pp], j = kBPj[pp];
      double v;
      if (po < 6) {
        v = R.N0[3 * i + j] - 0.25 * a3 * sQ[pp];
      } else if (po < 12) {
        v = 0.25 * a3 * om * (R.E[3 * i + j] + sQ[6 + pp] + sQ[24 + 3 * i + j] + sQ[24 + 3 * j + i]);
      } else {
        double cr[3];
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          const int a = t == 0 ? i : (t == 1 ? j : i);
          const int b = t == 0 ? i : (t == 1 ? j : j);
          const int q = bpair(a, b);
          const double Wab = G[(size_t)a * ldG + b].x;
          cr[t] = om * om * (Wab + sQ[33 + 3 * a + b] + sQ[33 + 3 * b + a] + sQ[18 + q]) -
                  om * (sQ[42 + 3 * a + b] + sQ[42 + 3 * b + a]) + sQ[12 + q];
        }
        const double ni = sqrt(fmax(cr[0], 0.0)), nj = sqrt(fmax(cr[1], 0.0));
        const double ei = sqrt(fmax(sQ[51 + i], 0.0)), ej = sqrt(fmax(sQ[51 + j], 0.0));
        v = a3 / (8.0 * R.alpha_lb) * (2.0 * cr[0] + 2.0 * cr[1] - 2.0 * cr[2]) +
            0.25 * a3 * (ni * ej + nj * ei);
      }
      out[18 * k_om + po] = v;
    }
    if (a_out != nullptr)
      for (int e = tid; e < 3 * M; e += kBigThreads) {
        const int i = e / M, r = e % M;
        reinterpret_cast<double2*>(a_out)[(size_t)k_om * 3 * M + i * M + r] = sX[i][r];
      }
    if (tid == 0) status[k_om] = sBad ? 4 : 0;
    __syncthreads();
  }
}

size_t sweep_big_lds_bytes(int M) { return (size_t)M * kBigLd * sizeof(double2); }

hipError_t sweep_big_launch(const mpt_rom& R, const double* omega, int64_t n, double* out,
                            double* a_out, int32_t* status, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (R.M > kBigMaxM) return hipErrorInvalidValue;
  // the mat-vec results (15 vectors of kBigMaxM) reuse the matrix region
  const size_t lds = std::max(sweep_big_lds_bytes(R.M), (size_t)15 * kBigMaxM * sizeof(double2));
  // one workgroup per CU fits (about 160 KB of LDS at M = 96); a grid-stride
  // loop over the frequencies
  const int64_t groups = std::min<int64_t>(n, 1024);
  hipLaunchKernelGGL(k_sweep_big, dim3((unsigned)groups), dim3(kBigThreads), lds, st, R, omega, n,
                     out, a_out, status);
  return hipGetLastError();
}

}  // namespace mpt
