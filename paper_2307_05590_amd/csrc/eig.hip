// Hermitian eigen-decomposition of a small matrix (n <= 192) by cyclic
// two-sided Jacobi with the parallel round-robin ordering.
//
// Each round rotates n/2 disjoint index pairs at once.  With the rotations of
// a round fixed, every 2x2 block A[{p1,q1},{p2,q2}] transforms independently
// (Q1^H B Q2), so one pass over the upper block triangle (mirrored into the
// lower one) applies the whole round: one read and one write of A per round,
// A held in LDS when it fits.  The rotations of every round are recorded and a
// second, row-parallel kernel accumulates the eigenvector matrix V = prod Q
// (rows of V are independent), keeping the sequential kernel's work to A.
// The rotation threshold |a_pq| <= tol sqrt(|a_pp a_qq|) keeps the relative
// accuracy of the small eigenvalues of graded Gram matrices.
#include "device_util.h"
#include "kernels.h"

namespace mpt {

constexpr int kJacobiMaxN = 192;
constexpr int kJacobiThreads = 1024;

struct Rot {
  double c, s;   // real cosine / sine
  double2 ph;    // e^{-i phi}, phi = arg a_pq
};

__device__ __forceinline__ int rr_index(int j, int r, int ne) {
  return j == 0 ? 0 : 1 + ((j - 1 + r) % (ne - 1));
}

// pair t of round r (p < q); q == n marks the idle slot of an odd n
__device__ __forceinline__ void rr_pair(int t, int r, int ne, int& p, int& q) {
  p = rr_index(t, r, ne);
  q = rr_index(ne - 1 - t, r, ne);
  if (p > q) { const int tmp = p; p = q; q = tmp; }
}

template <bool SHARED_A>
__global__ __launch_bounds__(kJacobiThreads) void k_jacobi(double2* __restrict__ Ag, int n,
                                                           double* __restrict__ lam,
                                                           Rot* __restrict__ rec,
                                                           int* __restrict__ info, int max_sweeps,
                                                           double tol) {
  extern __shared__ double2 smem[];
  __shared__ Rot rot[kJacobiMaxN / 2];
  __shared__ int rp[kJacobiMaxN / 2], rq[kJacobiMaxN / 2];
  __shared__ int nrot;
  __shared__ double dmax;
  // LDS copy with a padded row stride (n+1 complex) against bank conflicts
  const int ld = SHARED_A ? n + 1 : n;
  double2* A = SHARED_A ? smem : Ag;
  const int tid = threadIdx.x, nt = blockDim.x;
  if (SHARED_A)
    for (int i = tid; i < n * n; i += nt) A[(i / n) * ld + i % n] = Ag[i];
  const int ne = n + (n & 1);
  const int np = ne / 2;
  const int nblk = np * (np + 1) / 2;
  // block table: e -> (ta, tb), ta <= tb, packed in the LDS tail
  unsigned short* tab = reinterpret_cast<unsigned short*>(SHARED_A ? smem + (size_t)n * ld : smem);
  for (int e = tid; e < nblk; e += nt) {
    int t1 = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
    while ((t1 + 1) * (t1 + 2) / 2 <= e) ++t1;
    while (t1 * (t1 + 1) / 2 > e) --t1;
    tab[2 * e] = (unsigned short)(e - t1 * (t1 + 1) / 2);
    tab[2 * e + 1] = (unsigned short)t1;
  }
  int sweep = 0;
  bool converged = false;
  __syncthreads();
  for (; sweep < max_sweeps; ++sweep) {
    if (tid == 0) {
      nrot = 0;
      double m = 0.0;
      for (int i = 0; i < n; ++i) m = fmax(m, fabs(A[i * ld + i].x));
      dmax = m;
    }
    __syncthreads();
    const double floor_abs = 1e-30 * dmax;
    for (int r = 0; r < ne - 1; ++r) {
      for (int t = tid; t < np; t += nt) {
        int p, q;
        rr_pair(t, r, ne, p, q);
        Rot R = {1.0, 0.0, make_double2(1.0, 0.0)};
        if (q < n) {
          const double a = A[p * ld + p].x, d = A[q * ld + q].x;
          const double2 b = A[p * ld + q];
          const double ab = sqrt(b.x * b.x + b.y * b.y);
          if (ab > floor_abs && ab > 1e-300 && ab > tol * sqrt(fabs(a * d))) {
            const double tau = (d - a) / (2.0 * ab);
            const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            R.c = 1.0 / sqrt(1.0 + tt * tt);
            R.s = tt * R.c;
            R.ph = make_double2(b.x / ab, -b.y / ab);
            nrot = 1;  // any rotation this sweep (benign same-value race)
          }
        }
        rot[t] = R;
        rp[t] = p;
        rq[t] = q;
        rec[((size_t)sweep * (ne - 1) + r) * np + t] = R;
      }
      __syncthreads();
      // 2x2 blocks (t1 <= t2): B <- Q1^H B Q2, Q = [[c, s], [-s ph, c ph]]
      for (int e = tid; e < nblk; e += nt) {
        const int ta = tab[2 * e], tb = tab[2 * e + 1];  // ta <= tb
        const int p1 = rp[ta], q1 = rq[ta], p2 = rp[tb], q2 = rq[tb];
        const Rot R1 = rot[ta], R2 = rot[tb];
        if (R1.s == 0.0 && R2.s == 0.0) continue;
        const bool v1 = q1 < n, v2 = q2 < n;
        double2 b00 = A[p1 * ld + p2];
        double2 b01 = v2 ? A[p1 * ld + q2] : make_double2(0.0, 0.0);
        double2 b10 = v1 ? A[q1 * ld + p2] : make_double2(0.0, 0.0);
        double2 b11 = (v1 && v2) ? A[q1 * ld + q2] : make_double2(0.0, 0.0);
        // right: B Q2 (columns p2, q2)
        if (R2.s != 0.0) {
          const double c = R2.c, s = R2.s;
          const double2 t0 = cmul(b01, R2.ph), t1v = cmul(b11, R2.ph);
          const double2 n00 = make_double2(c * b00.x - s * t0.x, c * b00.y - s * t0.y);
          const double2 n01 = make_double2(s * b00.x + c * t0.x, s * b00.y + c * t0.y);
          const double2 n10 = make_double2(c * b10.x - s * t1v.x, c * b10.y - s * t1v.y);
          const double2 n11 = make_double2(s * b10.x + c * t1v.x, s * b10.y + c * t1v.y);
          b00 = n00; b01 = n01; b10 = n10; b11 = n11;
        }
        // left: Q1^H B (rows p1, q1)
        if (R1.s != 0.0) {
          const double c = R1.c, s = R1.s;
          const double2 phc = cconj(R1.ph);
          const double2 t0 = cmul(b10, phc), t1v = cmul(b11, phc);
          const double2 n00 = make_double2(c * b00.x - s * t0.x, c * b00.y - s * t0.y);
          const double2 n01 = make_double2(c * b01.x - s * t1v.x, c * b01.y - s * t1v.y);
          const double2 n10 = make_double2(s * b00.x + c * t0.x, s * b00.y + c * t0.y);
          const double2 n11 = make_double2(s * b01.x + c * t1v.x, s * b01.y + c * t1v.y);
          b00 = n00; b01 = n01; b10 = n10; b11 = n11;
        }
        if (ta == tb) {  // diagonal block: exactly diagonal after the rotation
          A[p1 * ld + p1] = make_double2(b00.x, 0.0);
          if (v1) {
            A[q1 * ld + q1] = make_double2(b11.x, 0.0);
            A[p1 * ld + q1] = make_double2(0.0, 0.0);
            A[q1 * ld + p1] = make_double2(0.0, 0.0);
          }
        } else {
          A[p1 * ld + p2] = b00;
          A[p2 * ld + p1] = cconj(b00);
          if (v2) {
            A[p1 * ld + q2] = b01;
            A[q2 * ld + p1] = cconj(b01);
          }
          if (v1) {
            A[q1 * ld + p2] = b10;
            A[p2 * ld + q1] = cconj(b10);
          }
          if (v1 && v2) {
            A[q1 * ld + q2] = b11;
            A[q2 * ld + q1] = cconj(b11);
          }
        }
      }
      __syncthreads();
    }
    if (nrot == 0) {
      converged = true;
      break;
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += nt) lam[i] = A[i * ld + i].x;
  if (SHARED_A)
    for (int i = tid; i < n * n; i += nt) Ag[i] = A[(i / n) * ld + i % n];
  if (tid == 0) {
    info[0] = converged ? sweep + 1 : -1;
    info[2] = converged ? sweep + 1 : max_sweeps;  // recorded sweeps
  }
}

// V = prod of the recorded rotations; one workgroup per row of V, the row in
// LDS, the disjoint pairs of a round applied in parallel by the lanes.
__global__ __launch_bounds__(128) void k_jacobi_vectors(int n, const Rot* __restrict__ rec,
                                                        const int* __restrict__ info,
                                                        double2* __restrict__ V) {
  __shared__ double2 row[kJacobiMaxN];
  const int k = blockIdx.x;
  const int tid = threadIdx.x;
  for (int j = tid; j < n; j += blockDim.x) row[j] = make_double2(j == k ? 1.0 : 0.0, 0.0);
  const int ne = n + (n & 1);
  const int np = ne / 2;
  const int sweeps = info[2];
  __syncthreads();
  for (int sw = 0; sw < sweeps; ++sw) {
    for (int r = 0; r < ne - 1; ++r) {
      const Rot* rr = rec + ((size_t)sw * (ne - 1) + r) * np;
      for (int t = tid; t < np; t += blockDim.x) {
        const Rot R = rr[t];
        if (R.s == 0.0) continue;
        int p, q;
        rr_pair(t, r, ne, p, q);
        if (q >= n) continue;
        const double2 vp = row[p], vq = row[q];
        const double2 t2 = cmul(vq, R.ph);
        row[p] = make_double2(R.c * vp.x - R.s * t2.x, R.c * vp.y - R.s * t2.y);
        row[q] = make_double2(R.s * vp.x + R.c * t2.x, R.s * vp.y + R.c * t2.y);
      }
      __syncthreads();
    }
  }
  for (int j = tid; j < n; j += blockDim.x) V[k * n + j] = row[j];
}

size_t jacobi_ws_size(int n, int max_sweeps) {
  const int ne = n + (n & 1);
  return (size_t)max_sweeps * (ne - 1) * (ne / 2) * sizeof(Rot);
}

hipError_t jacobi_launch(double* A, int n, double* V, double* lam, int* info, void* ws,
                         int max_sweeps, double tol, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (n > kJacobiMaxN) return hipErrorInvalidValue;
  Rot* rec = reinterpret_cast<Rot*>(ws);
  const int ne = n + (n & 1), np = ne / 2;
  const size_t tab = (size_t)np * (np + 1) * sizeof(unsigned short) + 16;
  const size_t lds = (size_t)n * (n + 1) * sizeof(double2) + tab;
  if (lds <= 156 * 1024) {  // plus ~4 KB static: within the 160 KB of a CU
    hipLaunchKernelGGL((k_jacobi<true>), dim3(1), dim3(kJacobiThreads), lds, st,
                       reinterpret_cast<double2*>(A), n, lam, rec, info, max_sweeps, tol);
  } else {
    hipLaunchKernelGGL((k_jacobi<false>), dim3(1), dim3(kJacobiThreads), tab, st,
                       reinterpret_cast<double2*>(A), n, lam, rec, info, max_sweeps, tol);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_jacobi_vectors, dim3(n), dim3(128), 0, st, n, rec, info,
                     reinterpret_cast<double2*>(V));
  return hipGetLastError();
}

}  // namespace mpt
