// Hermitian eigen-decomposition of a small matrix (n <= 192) by cyclic
// two-sided Jacobi with the parallel round-robin ordering: every round
// rotates n/2 disjoint index pairs at once, so one workgroup applies all
// column rotations, then all row rotations, with a barrier between.
// The rotation threshold |a_pq| <= tol sqrt(|a_pp a_qq|) keeps the relative
// accuracy of the small eigenvalues of graded Gram matrices.
#include "device_util.h"
#include "kernels.h"

namespace mpt {

constexpr int kJacobiMaxN = 192;

__device__ __forceinline__ int rr_index(int j, int r, int ne) {
  return j == 0 ? 0 : 1 + ((j - 1 + r) % (ne - 1));
}

template <bool SHARED_A>
__global__ __launch_bounds__(256) void k_jacobi(double2* __restrict__ Ag, int n,
                                                double2* __restrict__ V, double* __restrict__ lam,
                                                int* __restrict__ info, int max_sweeps) {
  extern __shared__ double2 smem[];
  __shared__ double rc[kJacobiMaxN / 2];
  __shared__ double2 rs[kJacobiMaxN / 2];  // s
  __shared__ double2 rph[kJacobiMaxN / 2];  // e^{-i phi}
  __shared__ int rp[kJacobiMaxN / 2], rq[kJacobiMaxN / 2];
  __shared__ int nrot;
  __shared__ double dmax;
  double2* A = SHARED_A ? smem : Ag;
  const int tid = threadIdx.x, nt = blockDim.x;
  if (SHARED_A) {
    for (int i = tid; i < n * n; i += nt) A[i] = Ag[i];
  }
  for (int i = tid; i < n * n; i += nt) V[i] = make_double2((i / n) == (i % n) ? 1.0 : 0.0, 0.0);
  const int ne = n + (n & 1);
  const int np = ne / 2;
  // rotation threshold: 4 n eps relative to sqrt(|a_pp a_qq|) (keeps the
  // relative accuracy of graded matrices), with an absolute floor 1e-30 of
  // the largest diagonal entry (below double precision for sigma^2)
  const double tol = 4.0 * n * 2.220446049250313e-16;
  int sweep = 0;
  bool converged = false;
  __syncthreads();
  for (; sweep < max_sweeps; ++sweep) {
    if (tid == 0) {
      nrot = 0;
      double m = 0.0;
      for (int i = 0; i < n; ++i) m = fmax(m, fabs(A[i * n + i].x));
      dmax = m;
    }
    __syncthreads();
    const double floor_abs = 1e-30 * dmax;
    for (int r = 0; r < ne - 1; ++r) {
      // rotations of this round
      for (int t = tid; t < np; t += nt) {
        int p = rr_index(t, r, ne), q = rr_index(ne - 1 - t, r, ne);
        if (p > q) { const int tmp = p; p = q; q = tmp; }
        double c = 1.0;
        double2 s = make_double2(0.0, 0.0), ph = make_double2(1.0, 0.0);
        if (q < n) {
          const double a = A[p * n + p].x, d = A[q * n + q].x;
          const double2 b = A[p * n + q];
          const double ab = sqrt(b.x * b.x + b.y * b.y);
          if (ab > floor_abs && ab > 1e-300 && ab > tol * sqrt(fabs(a * d))) {
            const double tau = (d - a) / (2.0 * ab);
            const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = make_double2(tt * c, 0.0);
            ph = make_double2(b.x / ab, -b.y / ab);  // e^{-i phi}
            atomicAdd(&nrot, 1);
          }
        }
        rc[t] = c;
        rs[t] = s;
        rph[t] = ph;
        rp[t] = p;
        rq[t] = q;
      }
      __syncthreads();
      // A <- A Q and V <- V Q (column pairs)
      for (int w = tid; w < np * n; w += nt) {
        const int t = w / n, k = w % n;
        const int q = rq[t];
        if (q >= n || (rs[t].x == 0.0)) continue;
        const int p = rp[t];
        const double c = rc[t], s = rs[t].x;
        const double2 ph = rph[t];
        {
          const double2 akp = A[k * n + p], akq = A[k * n + q];
          const double2 t2 = cmul(akq, ph);  // a_kq e^{-i phi}
          A[k * n + p] = make_double2(c * akp.x - s * t2.x, c * akp.y - s * t2.y);
          A[k * n + q] = make_double2(s * akp.x + c * t2.x, s * akp.y + c * t2.y);
        }
        {
          const double2 vkp = V[k * n + p], vkq = V[k * n + q];
          const double2 t2 = cmul(vkq, ph);
          V[k * n + p] = make_double2(c * vkp.x - s * t2.x, c * vkp.y - s * t2.y);
          V[k * n + q] = make_double2(s * vkp.x + c * t2.x, s * vkp.y + c * t2.y);
        }
      }
      __syncthreads();
      // A <- Q^H A (row pairs)
      for (int w = tid; w < np * n; w += nt) {
        const int t = w / n, k = w % n;
        const int q = rq[t];
        if (q >= n || (rs[t].x == 0.0)) continue;
        const int p = rp[t];
        const double c = rc[t], s = rs[t].x;
        const double2 phc = cconj(rph[t]);  // e^{+i phi}
        const double2 apk = A[p * n + k], aqk = A[q * n + k];
        const double2 t2 = cmul(aqk, phc);
        A[p * n + k] = make_double2(c * apk.x - s * t2.x, c * apk.y - s * t2.y);
        A[q * n + k] = make_double2(s * apk.x + c * t2.x, s * apk.y + c * t2.y);
      }
      __syncthreads();
    }
    if (nrot == 0) {
      converged = true;
      break;
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += nt) lam[i] = A[i * n + i].x;
  if (SHARED_A) {
    for (int i = tid; i < n * n; i += nt) Ag[i] = A[i];
  }
  if (tid == 0) info[0] = converged ? sweep + 1 : -1;
}

hipError_t jacobi_launch(double* A, int n, double* V, double* lam, int* info, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (n > kJacobiMaxN) return hipErrorInvalidValue;
  const size_t lds = (size_t)n * n * sizeof(double2);
  if (lds <= 150 * 1024) {
    hipLaunchKernelGGL((k_jacobi<true>), dim3(1), dim3(256), lds, st,
                       reinterpret_cast<double2*>(A), n, reinterpret_cast<double2*>(V), lam, info,
                       60);
  } else {
    hipLaunchKernelGGL((k_jacobi<false>), dim3(1), dim3(256), 0, st,
                       reinterpret_cast<double2*>(A), n, reinterpret_cast<double2*>(V), lam, info,
                       60);
  }
  return hipGetLastError();
}

}  // namespace mpt
