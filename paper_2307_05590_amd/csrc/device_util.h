// Device helpers shared by the libmpt kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpt {

constexpr int kWave = 64;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
// conj(a) * b
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, a.y * b.y), fma(a.x, b.y, -a.y * b.x));
}
// acc + a * b
__device__ __forceinline__ double2 cfma(double2 acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
  return acc;
}
// acc - a * b
__device__ __forceinline__ double2 cfms(double2 acc, double2 a, double2 b) {
  acc.x = fma(-a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(-a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
  return acc;
}
// acc + conj(a) * b
__device__ __forceinline__ double2 cfmac(double2 acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
  return acc;
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// 1 / z for a non-zero complex z
__device__ __forceinline__ double2 crecip(double2 z) {
  const double d = z.x * z.x + z.y * z.y;
  const double r = 1.0 / d;
  return make_double2(z.x * r, -z.y * r);
}

// Broadcast from a wave-uniform lane (v_readlane).
__device__ __forceinline__ double bcast(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double2 bcast2(double2 v, int lane) {
  return make_double2(bcast(v.x, lane), bcast(v.y, lane));
}

__device__ __forceinline__ double shfl_xor_d(double v, int mask) {
  const int src = (__lane_id() ^ mask) << 2;
  const int lo = __builtin_amdgcn_ds_bpermute(src, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(src, __double2hiint(v));
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double shfl_d(double v, int src_lane) {
  const int src = src_lane << 2;
  const int lo = __builtin_amdgcn_ds_bpermute(src, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(src, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = fmax(v, shfl_xor_d(v, m));
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += shfl_xor_d(v, m);
  return v;
}

// Reduce-scatter of 64 per-lane partial sums: on return, lane l holds the
// wave-wide sum of slot l.  Fixed order (deterministic).
__device__ __forceinline__ double reduce_scatter64(double (&v)[64]) {
  const int lane = __lane_id();
#pragma unroll
  for (int half = 32; half >= 1; half >>= 1) {
    const bool upper = (lane & half) != 0;
#pragma unroll
    for (int t = 0; t < half; ++t) {
      const double lo = v[t], hi = v[t + half];
      const double send = upper ? lo : hi;
      const double keep = upper ? hi : lo;
      v[t] = keep + shfl_xor_d(send, half);
    }
  }
  return v[0];
}

}  // namespace mpt
