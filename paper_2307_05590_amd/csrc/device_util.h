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

// v_mfma_f64_16x16x4f64, operand layout for lane l (0..63):
//   a: A[l % 16][l / 16]   b: B[l / 16][l % 16]   d: D[(l / 16) + 4 v][l % 16]
typedef double double4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ double4_t mfma(double a, double b, double4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

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

// DPP lane moves of a double (both halves with the same control); lanes the
// control does not write keep `old`.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v, double old) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), CTRL, 0xf,
                                             0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), CTRL, 0xf,
                                             0xf, false);
  return __hiloint2double(hi, lo);
}
constexpr int kDppXor1 = 0xB1;         // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;         // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;  // lane i <-> 7-i within 8 lanes
constexpr int kDppMirror = 0x140;      // lane i <-> 15-i within 16 lanes

// sum / max over each group of 16 lanes (a DPP row), result in every lane
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_d<kDppXor1>(v, 0.0);
  v += dpp_d<kDppXor2>(v, 0.0);
  v += dpp_d<kDppHalfMirror>(v, 0.0);
  v += dpp_d<kDppMirror>(v, 0.0);
  return v;
}
__device__ __forceinline__ double row16_max(double v) {
  v = fmax(v, dpp_d<kDppXor1>(v, v));
  v = fmax(v, dpp_d<kDppXor2>(v, v));
  v = fmax(v, dpp_d<kDppHalfMirror>(v, v));
  v = fmax(v, dpp_d<kDppMirror>(v, v));
  return v;
}
// combine each lane's value with the one 16 (32) lanes away, gfx950
// v_permlane16_swap / v_permlane32_swap: the two results of the swap hold
// both values of every lane pair
__device__ __forceinline__ void swap16_d(double v, double& a, double& b) {
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(v), __double2loint(v), false,
                                                   false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(v), __double2hiint(v), false,
                                                   false);
  a = __hiloint2double(hi[0], lo[0]);
  b = __hiloint2double(hi[1], lo[1]);
}
__device__ __forceinline__ void swap32_d(double v, double& a, double& b) {
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(v), __double2loint(v), false,
                                                   false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(v), __double2hiint(v), false,
                                                   false);
  a = __hiloint2double(hi[0], lo[0]);
  b = __hiloint2double(hi[1], lo[1]);
}
// max over groups of 16 / 32 / 64 lanes, result in every lane of the group
template <int L>
__device__ __forceinline__ double group_max(double v) {
  v = row16_max(v);
  if constexpr (L >= 32) {
    double a, b;
    swap16_d(v, a, b);
    v = fmax(a, b);
  }
  if constexpr (L >= 64) {
    double a, b;
    swap32_d(v, a, b);
    v = fmax(a, b);
  }
  return v;
}

// wave-wide sum / max, result (uniform) in every lane: DPP inside each row of
// 16 lanes, then the four row results by v_readlane in a fixed order
__device__ __forceinline__ double wave_sum(double v) {
  v = row16_sum(v);
  return (bcast(v, 0) + bcast(v, 16)) + (bcast(v, 32) + bcast(v, 48));
}
__device__ __forceinline__ double wave_max(double v) {
  v = row16_max(v);
  return fmax(fmax(bcast(v, 0), bcast(v, 16)), fmax(bcast(v, 32), bcast(v, 48)));
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
