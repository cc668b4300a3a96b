// Dispatch of the sweep kernels (instantiated per M bucket in sweep_m*.hip so
// the buckets compile in parallel) and the small helpers of the batched and
// adjoint paths.
#include "device_util.h"
#include "kernels.h"

namespace mpt {

template <int MAXM, bool ADJ>
hipError_t launch_plain(const mpt_rom& R, const double* omega, int64_t n, double* out,
                        double* a_out, int32_t* status, const double* dout, double* dom, int wpg,
                        const MatSens& ms, hipStream_t st);
template <int MAXM, bool ADJ>
hipError_t launch_persistent(const mpt_rom* roms, const int4* items, int n_items,
                             unsigned int* counter, const double* omega, double* out,
                             int32_t* status, const double* dout, double* dom, int wpg,
                             int groups, hipStream_t st);

__global__ void k_reset_counter(unsigned int* c, int n) {
  if (threadIdx.x < n) c[threadIdx.x] = 0u;
}

// sigma dL/dsigma = sum_k omega_k dL/domega_k per object (fixed order).
__global__ void k_sigma_reduce(const double* __restrict__ omega, const double* __restrict__ dom,
                               const int64_t* __restrict__ off, int n_obj,
                               double* __restrict__ sig) {
  const int o = blockIdx.x;
  if (o >= n_obj) return;
  __shared__ double part[256];
  double acc = 0.0;
  for (int64_t k = off[o] + threadIdx.x; k < off[o + 1]; k += blockDim.x) acc += omega[k] * dom[k];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) sig[o] = part[0];
}

// ------------------------------------------------------------ launchers
int bucket_of(int M) { return M <= 16 ? 16 : (M <= 32 ? 32 : (M <= 48 ? 48 : 64)); }

hipError_t sweep_big_launch(const mpt_rom& R, const double* omega, int64_t n, double* out,
                            double* a_out, int32_t* status, hipStream_t st);

hipError_t sweep_launch(const mpt_rom& R, const double* omega, int64_t n, double* out,
                        double* a_out, int32_t* status, const double* dout, double* dom,
                        hipStream_t st, const MatSens& ms) {
  if (n <= 0) return hipSuccess;
  const bool adj = dout != nullptr;
  if (R.M > 64) {  // LDS-resident kernel; no adjoint form at this size
    if (adj) return hipErrorInvalidValue;
    return sweep_big_launch(R, omega, n, out, a_out, status, st);
  }
  if (!adj && ms.CM1) return hipErrorInvalidValue;  // material terms need the adjoint
  switch (bucket_of(R.M)) {
    case 16: return adj ? launch_plain<16, true>(R, omega, n, out, a_out, status, dout, dom, 4, ms, st)
                        : launch_plain<16, false>(R, omega, n, out, a_out, status, dout, dom, 4, ms, st);
    case 32: return adj ? launch_plain<32, true>(R, omega, n, out, a_out, status, dout, dom, 4, ms, st)
                        : launch_plain<32, false>(R, omega, n, out, a_out, status, dout, dom, 4, ms, st);
    case 48: return adj ? launch_plain<48, true>(R, omega, n, out, a_out, status, dout, dom, 2, ms, st)
                        : launch_plain<48, false>(R, omega, n, out, a_out, status, dout, dom, 4, ms, st);
    default: return adj ? launch_plain<64, true>(R, omega, n, out, a_out, status, dout, dom, 2, ms, st)
                        : launch_plain<64, false>(R, omega, n, out, a_out, status, dout, dom, 4, ms, st);
  }
}

hipError_t persistent_launch(int bucket, bool adj, const mpt_rom* roms, const int4* items,
                             int n_items, unsigned int* counter, const double* omega, double* out,
                             int32_t* status, const double* dout, double* dom, int wpg, int groups,
                             hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
#define MPT_PL(B)                                                                                 \
  return adj ? launch_persistent<B, true>(roms, items, n_items, counter, omega, out, status,      \
                                          dout, dom, wpg, groups, st)                             \
             : launch_persistent<B, false>(roms, items, n_items, counter, omega, out, status,     \
                                           dout, dom, wpg, groups, st)
  switch (bucket) {
    case 16: MPT_PL(16);
    case 32: MPT_PL(32);
    case 48: MPT_PL(48);
    default: MPT_PL(64);
  }
#undef MPT_PL
}

hipError_t reset_counters(unsigned int* c, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, c, n);
  return hipGetLastError();
}

// sigma_1 dL/dsigma_1 = sum_k dsig[k]; the other material takes the rest of
// sum_k omega_k dL/domega_k (fixed order, one workgroup)
__global__ void k_material_reduce(const double* __restrict__ omega,
                                  const double* __restrict__ dom, const double* __restrict__ dsig,
                                  int64_t n, double* __restrict__ out) {
  __shared__ double pa[256], pb[256];
  double a = 0.0, b = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
    a += dsig[k];
    b += omega[k] * dom[k];
  }
  pa[threadIdx.x] = a;
  pb[threadIdx.x] = b;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      pa[threadIdx.x] += pa[threadIdx.x + s];
      pb[threadIdx.x] += pb[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = pa[0];
    out[1] = pb[0] - pa[0];
  }
}

hipError_t material_reduce(const double* omega, const double* dom, const double* dsig, int64_t n,
                           double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_material_reduce, dim3(1), dim3(256), 0, st, omega, dom, dsig, n, out);
  return hipGetLastError();
}

hipError_t sigma_reduce(const double* omega, const double* dom, const int64_t* off, int n_obj,
                        double* sig, hipStream_t st) {
  hipLaunchKernelGGL(k_sigma_reduce, dim3(n_obj), dim3(256), 0, st, omega, dom, off, n_obj, sig);
  return hipGetLastError();
}

// sum_k omega_k dom_k over one object (fixed order), over sigma[0] if given
__global__ void k_sigma_reduce_one(const double* __restrict__ omega,
                                   const double* __restrict__ dom, int64_t n,
                                   const double* __restrict__ sigma, double* __restrict__ sig) {
  __shared__ double part[256];
  double acc = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += blockDim.x) acc += omega[k] * dom[k];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) sig[0] = sigma ? part[0] / sigma[0] : part[0];
}

hipError_t sigma_reduce_one(const double* omega, const double* dom, int64_t n,
                            const double* sigma, double* sig, hipStream_t st) {
  hipLaunchKernelGGL(k_sigma_reduce_one, dim3(1), dim3(256), 0, st, omega, dom, n, sigma, sig);
  return hipGetLastError();
}

}  // namespace mpt
