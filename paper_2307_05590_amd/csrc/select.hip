// Snapshot selection of Algorithm 1: per-interval maxima of the certificate
// (segmented over the sorted output frequencies), the global maximum Lambda
// and the N_* intervals with the largest maxima, each contributing its
// argmax frequency.  Deterministic: ties go to the smaller frequency inside
// an interval and to the lower interval index across intervals.
#include "device_util.h"
#include "kernels.h"

namespace mpt {

namespace {
__device__ __forceinline__ bool better(double v, int64_t i, double bv, int64_t bi) {
  // larger value wins; on equal values the smaller index (smaller omega)
  if (bi < 0) return i >= 0;
  if (i < 0) return false;
  return v > bv || (v == bv && i < bi);
}
}  // namespace

// number of k with omega[k] <= x (strict: < x) for ascending omega, by the
// whole block: a coarse pass over every stride-th entry, then the one stride
// that holds the boundary
__device__ int64_t block_count_below(const double* __restrict__ omega, int64_t n, double x,
                                     bool strict) {
  const int64_t stride = (n + blockDim.x - 1) / blockDim.x;
  const int64_t p = (int64_t)threadIdx.x * stride;
  const bool c = p < n && (strict ? omega[p] < x : omega[p] <= x);
  const int cnt = __syncthreads_count(c);
  if (cnt == 0) return 0;
  const int64_t base = (int64_t)(cnt - 1) * stride, end = min(n, base + stride);
  int64_t tot = 0;
  for (int64_t q0 = base + 1; q0 < end; q0 += blockDim.x) {
    const int64_t q = q0 + threadIdx.x;
    tot += __syncthreads_count(q < end && (strict ? omega[q] < x : omega[q] <= x));
  }
  return base + 1 + tot;
}

// one block per interval j: snap[j] < w < snap[j+1] (Algorithm 1's interval
// without its left end, which is a snapshot already); omega is ascending, so
// the interval's frequencies are one contiguous range, found first
__global__ __launch_bounds__(256) void k_interval_max(const double* __restrict__ omega, int64_t n,
                                                      const double* __restrict__ out,
                                                      const double* __restrict__ snap, int n_snap,
                                                      double* __restrict__ lambda,
                                                      int64_t* __restrict__ arg) {
  const int j = blockIdx.x;
  const double lo = snap[j], hi = snap[j + 1];
  const int64_t k0 = block_count_below(omega, n, lo, false);
  const int64_t k1 = block_count_below(omega, n, hi, true);
  double bv = -INFINITY;
  int64_t bi = -1;
  for (int64_t k = k0 + threadIdx.x; k < k1; k += blockDim.x) {
    const double w = omega[k];
    const bool in = (w > lo) && (w < hi);
    if (!in) continue;
    double d = out[18 * k + 12];
#pragma unroll
    for (int p = 13; p < 18; ++p) d = fmax(d, out[18 * k + p]);
    if (better(d, k, bv, bi)) {
      bv = d;
      bi = k;
    }
  }
  __shared__ double sv[256];
  __shared__ int64_t si[256];
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      if (better(sv[threadIdx.x + s], si[threadIdx.x + s], sv[threadIdx.x], si[threadIdx.x])) {
        sv[threadIdx.x] = sv[threadIdx.x + s];
        si[threadIdx.x] = si[threadIdx.x + s];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    lambda[j] = si[0] >= 0 ? sv[0] : -INFINITY;
    arg[j] = si[0];
  }
}

// single block: rank intervals, pick n_star, global max
__global__ __launch_bounds__(64) void k_rank(const double* __restrict__ omega,
                                             const double* __restrict__ lambda,
                                             const int64_t* __restrict__ arg, int n_int,
                                             int n_star, double* __restrict__ new_omega,
                                             double* __restrict__ Lmax) {
  if (threadIdx.x != 0) return;
  double gmax = -INFINITY;
  for (int j = 0; j < n_int; ++j)
    if (arg[j] >= 0 && lambda[j] > gmax) gmax = lambda[j];
  *Lmax = gmax;
  // selection by repeated scans (n_star <= 64 and n_int are small)
  int chosen[64];
  for (int r = 0; r < n_star; ++r) {
    int best = -1;
    for (int j = 0; j < n_int; ++j) {
      if (arg[j] < 0) continue;
      bool taken = false;
      for (int t = 0; t < r; ++t)
        if (chosen[t] == j) taken = true;
      if (taken) continue;
      if (best < 0 || lambda[j] > lambda[best]) best = j;
    }
    chosen[r] = best;
    new_omega[r] = best >= 0 ? omega[arg[best]] : NAN;
  }
}

// threshold variant: every interval j with lambda[j] >= theta * Lambda gives
// omega[arg[j]] at its rank (descending lambda, ties lower j); one thread per
// interval; new_omega has n_int entries, NaN after the last chosen
__global__ __launch_bounds__(256) void k_rank_threshold(const double* __restrict__ omega,
                                                        const double* __restrict__ lambda,
                                                        const int64_t* __restrict__ arg,
                                                        int n_int, double theta,
                                                        double* __restrict__ new_omega,
                                                        int32_t* __restrict__ n_new,
                                                        double* __restrict__ Lmax) {
  __shared__ double gmax_s;
  __shared__ int count_s;
  if (threadIdx.x == 0) {
    double gmax = -INFINITY;
    for (int j = 0; j < n_int; ++j)
      if (arg[j] >= 0 && lambda[j] > gmax) gmax = lambda[j];
    gmax_s = gmax;
    int cnt = 0;
    for (int j = 0; j < n_int; ++j)
      if (arg[j] >= 0 && lambda[j] >= theta * gmax) ++cnt;
    count_s = cnt;
    *Lmax = gmax;
    *n_new = cnt;
  }
  __syncthreads();
  const double thr = theta * gmax_s;
  for (int j = threadIdx.x; j < n_int; j += blockDim.x) {
    const bool q = arg[j] >= 0 && lambda[j] >= thr;
    if (q) {
      int rank = 0;
      for (int k = 0; k < n_int; ++k)
        if (arg[k] >= 0 && lambda[k] >= thr &&
            (lambda[k] > lambda[j] || (lambda[k] == lambda[j] && k < j)))
          ++rank;
      new_omega[rank] = omega[arg[j]];
    }
  }
  for (int r = count_s + threadIdx.x; r < n_int; r += blockDim.x) new_omega[r] = NAN;
}

hipError_t select_threshold_launch(const double* omega, int64_t n, const double* out,
                                   const double* snap, int n_snap, double theta,
                                   double* new_omega, int32_t* n_new, double* lambda,
                                   double* Lambda_max, int64_t* arg_ws, hipStream_t st) {
  const int n_int = n_snap - 1;
  hipLaunchKernelGGL(k_interval_max, dim3(n_int), dim3(256), 0, st, omega, n, out, snap, n_snap,
                     lambda, arg_ws);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rank_threshold, dim3(1), dim3(256), 0, st, omega, lambda, arg_ws, n_int,
                     theta, new_omega, n_new, Lambda_max);
  return hipGetLastError();
}

hipError_t select_launch(const double* omega, int64_t n, const double* out, const double* snap,
                         int n_snap, int n_star, double* new_omega, double* lambda,
                         double* Lambda_max, int64_t* arg_ws, hipStream_t st) {
  const int n_int = n_snap - 1;
  hipLaunchKernelGGL(k_interval_max, dim3(n_int), dim3(256), 0, st, omega, n, out, snap, n_snap,
                     lambda, arg_ws);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rank, dim3(1), dim3(64), 0, st, omega, lambda, arg_ws, n_int, n_star,
                     new_omega, Lambda_max);
  return hipGetLastError();
}

}  // namespace mpt
