// Online reduced sweep (eq. (ReducedA)), matrix-method tensors (eqs.
// (podprealmpt), (podpimagmpt)), certificates (Lemma 4.1) and the adjoint of
// the sweep.
//
// A wave64 is split into segments of L = 16, 32 or 64 lanes (the smallest
// that holds M rows); each segment solves one frequency, so a wave sweeps
// 64/L frequencies at once.  Row r of the M x M system lives in the registers
// of lane r of its segment: the LU with partial pivoting, the three solves,
// the four reduced matrix-vector products and the quadratic forms never leave
// the register file.  Pivot rows and solution entries are broadcast inside a
// segment (v_readlane for whole waves, ds_bpermute otherwise); the quadratic
// forms are reduce-scattered inside the segment in a fixed order.
#pragma once
#include "device_util.h"
#include "kernels.h"

namespace mpt {

namespace {

// Slots of the reduce-scatter (64 per frequency).  G_s blocks (Lemma 4.1,
// unknowns [C w | X U | C U]): Gxx = G_s[XU, XU], H = G_s[CU, CU],
// F = G_s[Cw, CU], B = G_s[Cw, XU], W = G_s[Cw, Cw]; D' the defect form.
constexpr int kKQ = 0;    // Re a_i^H K_M a_j         (6 pairs)
constexpr int kCQ = 6;    // Re a_i^H C_M a_j         (6)
constexpr int kAQ = 12;   // Re a_i^H Gxx a_j         (6)
constexpr int kHQ = 18;   // Re a_i^H H a_j           (6)
constexpr int kGA = 24;   // Re g_i^H a_j             (9)
constexpr int kFA = 33;   // Re (F a_j)_i             (9)
constexpr int kBA = 42;   // Im (B a_j)_i             (9)
constexpr int kDQ = 51;   // Re a_i^H D' a_i (3); per-direction form:
                          // Re a_j^H D'_{i<-j} a_j at kDQ + 3 i + j (9)
constexpr int kSlots = 60;

// index of the reference shift of frequency om: the largest k with
// s_ref[k] <= om (s_ref ascending, s_ref[0] = 0)
__device__ __forceinline__ int ref_of(const mpt_rom& R, double om) {
  int k = 0;
  for (int j = 1; j < R.n_ref; ++j)
    if (R.s_ref[j] <= om) k = j;
  return k;
}

__device__ __constant__ int kPi[6] = {0, 0, 0, 1, 1, 2};
__device__ __constant__ int kPj[6] = {0, 1, 2, 1, 2, 2};

__device__ __forceinline__ int pair_index(int i, int j) {
  // stored order 11 12 13 22 23 33 for i <= j
  if (i > j) { const int t = i; i = j; j = t; }
  return i == 0 ? j : (i == 1 ? 2 + j : 5);
}

template <int MAXM>
struct SegOf {
  static constexpr int L = MAXM <= 16 ? 16 : (MAXM <= 32 ? 32 : 64);  // lanes per frequency
  static constexpr int S = 64 / L;                                     // frequencies per wave
};

// broadcast from lane src of this lane's segment (src is a lane id of the wave)
template <int L>
__device__ __forceinline__ double seg_bcast(double v, int src) {
  if constexpr (L == 64) return bcast(v, __builtin_amdgcn_readfirstlane(src));
  else return shfl_d(v, src);
}
template <int L>
__device__ __forceinline__ double2 seg_bcast2(double2 v, int src) {
  return make_double2(seg_bcast<L>(v.x, src), seg_bcast<L>(v.y, src));
}
// src already wave-uniform (an SGPR): no v_readfirstlane per call for L = 64
template <int L>
__device__ __forceinline__ double2 seg_bcast2u(double2 v, int src) {
  if constexpr (L == 64) return bcast2(v, src);
  else return make_double2(shfl_d(v.x, src), shfl_d(v.y, src));
}
template <int L>
__device__ __forceinline__ double seg_max(double v) {
  return group_max<L>(v);  // DPP inside rows, permlane swaps across rows
}
template <int L>
__device__ __forceinline__ double seg_sum(double v) {
#pragma unroll
  for (int m = L / 2; m >= 1; m >>= 1) v += shfl_xor_d(v, m);
  return v;
}
// first lane (as a wave lane id) of the segment whose predicate holds; -1 if none
template <int L>
__device__ __forceinline__ int seg_first(bool pred, int base) {
  const uint64_t m = __ballot(pred);
  const uint64_t mask = (L == 64) ? ~0ull : ((1ull << L) - 1ull);
  const uint64_t s = (m >> base) & mask;
  return s ? base + (__ffsll((unsigned long long)s) - 1) : -1;
}

// value of the partner lane at distance D (a lane pairing that flips bit
// log2 D of the lane id): permlane swaps across rows, DPP mirrors inside
template <int D>
__device__ __forceinline__ double xch(double x, int wl) {
  if constexpr (D == 32) {
    double a, b;
    swap32_d(x, a, b);
    return (wl & 32) ? a : b;
  } else if constexpr (D == 16) {
    double a, b;
    swap16_d(x, a, b);
    return (wl & 16) ? a : b;
  } else if constexpr (D == 8) {
    return dpp_d<kDppMirror>(x, 0.0);
  } else if constexpr (D == 4) {
    return dpp_d<kDppHalfMirror>(x, 0.0);
  } else if constexpr (D == 2) {
    return dpp_d<kDppXor2>(x, 0.0);
  } else {
    return dpp_d<kDppXor1>(x, 0.0);
  }
}

// one halving step of a reduce-scatter: partners at distance D split the
// HS-slot prefix of v (the lane with bit D set keeps the upper half)
template <int D, int HS>
__device__ __forceinline__ void rs_step(double (&v)[16], int wl) {
  const bool upper = (wl & D) != 0;
#pragma unroll
  for (int t = 0; t < HS; ++t) {
    const double lo = v[t], hi = v[t + HS];
    v[t] = (upper ? hi : lo) + xch<D>(upper ? lo : hi, wl);
  }
}

// reduce-scatter of 16 slots over a segment of L lanes (fixed order): lane
// ll ends with the segment sum of slot ll / (L / 16)
template <int L>
__device__ __forceinline__ double seg_rs16(double (&v)[16], int wl) {
  rs_step<L / 2, 8>(v, wl);
  rs_step<L / 4, 4>(v, wl);
  rs_step<L / 8, 2>(v, wl);
  rs_step<L / 16, 1>(v, wl);
  double r = v[0];
  if constexpr (L / 32 >= 2) r += xch<L / 32>(r, wl);
  if constexpr (L / 32 >= 1) r += xch<1>(r, wl);
  return r;
}

}  // namespace

// Everything for one frequency, executed by one segment of L lanes.
//   out:    18 doubles for this omega
//   status: one int
//   ADJ:    dout (18 doubles, first 12 used) -> dom (1 double);
//           lds_lu: MAXM x (MAXM+1) double2 private to the segment;
//           with ms.CM1 set, also dsig (1 double) = sigma_1 dL/dsigma_1.
//   red_lds: 64 doubles private to the segment.
//   valid:  false for a padding segment (computes, writes nothing).
//   out may be NULL (adjoint only); dscale multiplies dom (the chain rule of
//   a frequency scaling applied by the caller).
template <int MAXM, bool ADJ>
__device__ __forceinline__ void sweep_point(const mpt_rom& R, const double om, const bool valid,
                                            double* __restrict__ out, double* __restrict__ a_out,
                                            int32_t* __restrict__ status,
                                            const double* __restrict__ dout,
                                            double* __restrict__ dom, double2* lds_lu,
                                            double* red_lds, const MatSens& ms,
                                            double* __restrict__ dsig, double dscale = 1.0) {
  constexpr int L = SegOf<MAXM>::L;
  const int wl = __lane_id();
  const int ll = wl & (L - 1);   // lane within the segment
  const int base = wl - ll;      // first lane of the segment
  const int M = R.M;
  const bool act = ll < M;
  // per-direction form (one basis per direction, concatenated): block bounds
  // e1, e2 of the three directions; pd is uniform over the launch
  const bool pd = R.dirs[0] > 0;
  const int e1 = R.dirs[0], e2 = R.dirs[0] + R.dirs[1];
  const int bl = ll < e1 ? 0 : (ll < e2 ? 1 : 2);  // this lane's direction block
  const double2* A0 = reinterpret_cast<const double2*>(R.A0);
  const double2* CM = reinterpret_cast<const double2*>(R.CM);
  const double2* KM = reinterpret_cast<const double2*>(R.KM);
  const double2* gv = reinterpret_cast<const double2*>(R.g);
  const int ldG = 2 * M + 3;
  const int kref = ref_of(R, om);
  const double2* G = reinterpret_cast<const double2*>(R.G) + (size_t)kref * ldG * ldG;
  const double2* Dq = reinterpret_cast<const double2*>(R.Dp) + (size_t)kref * (pd ? 3 : 1) * M * M;

  // ---- row `ll` of A(w) = A0 - i w C_M and r_i = i w g_i ---------------
  double2 A[MAXM];
#pragma unroll
  for (int j = 0; j < MAXM; ++j) {
    double2 v = make_double2(0.0, 0.0);
    // per-direction: each direction's system lives in its own diagonal block
    const bool inblk = !pd || (j < e1 ? 0 : (j < e2 ? 1 : 2)) == bl;
    if (act && j < M && inblk) {
      // A0 and C_M are Hermitian: row ll is the conjugate of column ll, read
      // with one coalesced load per j across the lanes
      const double2 a0 = cconj(A0[j * M + ll]);
      const double2 c = cconj(CM[j * M + ll]);
      v.x = fma(om, c.y, a0.x);
      v.y = fma(-om, c.x, a0.y);
    }
    A[j] = v;
  }
  double2 gl[3], b[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    gl[i] = act ? gv[i * M + ll] : make_double2(0.0, 0.0);
    b[i] = (pd && bl != i) ? make_double2(0.0, 0.0) : make_double2(-om * gl[i].y, om * gl[i].x);
  }

  // ---- LU with partial pivoting (max |re|+|im|, lowest row on ties) -------
  bool done = !act;
  int order = -1;
  int bad = 0;
  double2 pinv = make_double2(0.0, 0.0);
#pragma unroll
  for (int k = 0; k < MAXM; ++k) {
    if (k < M) {
      const double val = done ? -1.0 : fabs(A[k].x) + fabs(A[k].y);
      const double vmax = seg_max<L>(val);
      int p = seg_first<L>((!done) && val == vmax, base);
      if (p < 0) {  // NaN pivot column: flag it and take any remaining row
        bad = 1;
        p = seg_first<L>(!done, base);
      }
      // for L = 64 the pivot lane is wave-uniform: read it into an SGPR once
      const int pu = (L == 64) ? __builtin_amdgcn_readfirstlane(p) : p;
      const double2 piv = seg_bcast2u<L>(A[k], pu);
      const double d = piv.x * piv.x + piv.y * piv.y;
      if (!(d > 0.0) || !isfinite(d)) bad = 1;
      const double2 inv = crecip(piv);
      if (wl == p) {
        done = true;
        order = k;
        pinv = inv;  // kept for the back substitution
      }
      const bool upd = !done;
      const double2 l0 = cmul(A[k], inv);
      if (upd) A[k] = l0;
      // rows already eliminated take a zero multiplier (x - 0 * y = x for
      // finite y) instead of a predicated update: no select per entry, and
      // the unrolled elimination stays small enough for short branches
      const double2 l = upd ? l0 : make_double2(0.0, 0.0);
      // columns j >= M hold exact zeros in every lane, so their update is a
      // no-op: up to M = 48 no per-column branch (one basic block per step);
      // the 64-wide bucket keeps the branch, or its registers spill
#pragma unroll
      for (int j = k + 1; j < MAXM; ++j) {
        if (MAXM <= 48 || j < M) {
          const double2 pr = seg_bcast2u<L>(A[j], pu);
          A[j] = cfms(A[j], l, pr);
        }
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double2 pb = seg_bcast2u<L>(b[i], pu);
        b[i] = cfms(b[i], l, pb);
      }
    }
  }

  // ---- back substitution; lane j of the segment receives a_i[j] -----------
  double2 x[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) x[i] = make_double2(0.0, 0.0);
#pragma unroll
  for (int k = MAXM - 1; k >= 0; --k) {
    if (k < M) {
      int q = seg_first<L>(order == k, base);
      if (q < 0) q = base;  // only after a flagged breakdown
      if (L == 64) q = __builtin_amdgcn_readfirstlane(q);
      const double2 inv = seg_bcast2u<L>(pinv, q);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double2 xk = cmul(seg_bcast2u<L>(b[i], q), inv);
        if (ll == k) x[i] = xk;
        if (order >= 0 && order < k) b[i] = cfms(b[i], A[k], xk);
      }
    }
  }

  if (ADJ) {
    // keep the factors: row k = pivot row k (L multipliers left of the
    // diagonal, U on and right of it)
    if (order >= 0) {
#pragma unroll
      for (int j = 0; j < MAXM; ++j)
        if (j < M) lds_lu[order * (MAXM + 1) + j] = A[j];
    }
  }

  // ---- reduced matrix-vector products, lane r holds row r -----------------
  double2 Ka[3], Ca[3], Aa[3], Ha[3], Da[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    Ka[i] = Ca[i] = Aa[i] = Ha[i] = Da[i] = make_double2(0.0, 0.0);
  }
  // K_M, C_M, Gxx, H and D' are Hermitian: lane ll reads column ll
  // (coalesced across lanes) and conjugates
  const double2* Xcol = G + (size_t)3 * ldG + 3 + ll;
  const double2* Hcol = G + (size_t)(3 + M) * ldG + (3 + M) + ll;
#pragma unroll 4
  for (int j = 0; j < M; ++j) {
    double2 aj[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) aj[i] = seg_bcast2u<L>(x[i], L == 64 ? j : base + j);
    if (act) {
      const double2 kk = cconj(KM[j * M + ll]);
      const double2 cc = cconj(CM[j * M + ll]);
      const double2 gx = cconj(Xcol[(size_t)j * ldG]);
      const double2 hh = cconj(Hcol[(size_t)j * ldG]);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        Ka[i] = cfma(Ka[i], kk, aj[i]);
        Ca[i] = cfma(Ca[i], cc, aj[i]);
        Aa[i] = cfma(Aa[i], gx, aj[i]);
        Ha[i] = cfma(Ha[i], hh, aj[i]);
      }
      if (!pd) {
        const double2 dd = cconj(Dq[j * M + ll]);
#pragma unroll
        for (int i = 0; i < 3; ++i) Da[i] = cfma(Da[i], dd, aj[i]);
      } else {  // D'_i applied to this lane's own direction's solution
        const double2 ab = bl == 0 ? aj[0] : (bl == 1 ? aj[1] : aj[2]);
#pragma unroll
        for (int i = 0; i < 3; ++i)
          Da[i] = cfma(Da[i], cconj(Dq[((size_t)i * M + j) * M + ll]), ab);
      }
    }
  }

  // ---- quadratic forms: per-lane partials of 54 slots, reduced in four
  // groups of 16 (segment reduce-scatter), totals to red_lds --------------
  double2 Fi[3], Bi[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    Fi[i] = act ? G[(size_t)i * ldG + 3 + M + ll] : make_double2(0.0, 0.0);
    Bi[i] = act ? G[(size_t)i * ldG + 3 + ll] : make_double2(0.0, 0.0);
  }
  auto partial = [&](int sl) -> double {
    if (sl < kGA) {
      const int q = sl % 6, kind = sl / 6;
      const int i = q < 3 ? 0 : (q < 5 ? 1 : 2);
      const int j = q == 0 ? 0 : (q == 1 ? 1 : (q == 2 ? 2 : (q == 3 ? 1 : 2)));
      const double2 y = kind == 0 ? Ka[j] : (kind == 1 ? Ca[j] : (kind == 2 ? Aa[j] : Ha[j]));
      return cmulc(x[i], y).x;
    }
    if (sl < kFA) {
      const int u = sl - kGA, i = u / 3, j = u % 3;
      return cmulc(gl[i], x[j]).x;
    }
    if (sl < kBA) {
      const int u = sl - kFA, i = u / 3, j = u % 3;
      return cmul(Fi[i], x[j]).x;
    }
    if (sl < kDQ) {
      const int u = sl - kBA, i = u / 3, j = u % 3;
      return cmul(Bi[i], x[j]).y;
    }
    if (sl < kSlots) {
      const int u = sl - kDQ;
      if (!pd) return u < 3 ? cmulc(x[u], Da[u]).x : 0.0;
      const int i = u / 3, j = u % 3;  // target basis i, source direction j
      return bl == j ? cmulc(x[j], Da[i]).x : 0.0;
    }
    return 0.0;
  };
  constexpr int kPerSlot = L / 16;  // lanes holding each slot total
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    double v[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) v[t] = act ? partial(16 * g + t) : 0.0;
    const double r = seg_rs16<L>(v, wl);
    if (ll % kPerSlot == 0) red_lds[16 * g + ll / kPerSlot] = r;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

  // ---- final formulas: outputs p = ll, ll + L, ... < 18 ------------------
  const double a3 = R.alpha * R.alpha * R.alpha;
  double iout = 0.0;  // I_p held by the lane computing output p in [6, 12)
#pragma unroll
  for (int p0 = 0; p0 < 18; p0 += L) {
    const int po = p0 + ll;
    if (po < 18) {
      const int pp = po % 6;
      const int i = kPi[pp], j = kPj[pp];
      double myout;
      if (po < 6) {
        myout = R.N0[3 * i + j] - 0.25 * a3 * red_lds[kKQ + pp];
      } else if (po < 12) {
        myout = 0.25 * a3 * om *
                (R.E[3 * i + j] + red_lds[kCQ + pp] + red_lds[kGA + 3 * i + j] +
                 red_lds[kGA + 3 * j + i]);
        iout = myout;
      } else {
        // Re c_ab = w^2 [W_ab + Re(F a_b)_a + Re(F a_a)_b + Re a_a^H H a_b]
        //           - w [Im (B a_b)_a + Im (B a_a)_b] + Re a_a^H Gxx a_b
        double cr[3];
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          const int a = t == 0 ? i : (t == 1 ? j : i);
          const int bb = t == 0 ? i : (t == 1 ? j : j);
          const int q = pair_index(a, bb);
          const double W = G[(size_t)a * ldG + bb].x;
          cr[t] = om * om * (W + red_lds[kFA + 3 * a + bb] + red_lds[kFA + 3 * bb + a] +
                             red_lds[kHQ + q]) -
                  om * (red_lds[kBA + 3 * a + bb] + red_lds[kBA + 3 * bb + a]) +
                  red_lds[kAQ + q];
        }
        const double ni = sqrt(fmax(cr[0], 0.0)), nj = sqrt(fmax(cr[1], 0.0));
        // e for (n_i, direction j) and (n_j, direction i): e_j and e_i of the
        // joint form, e_{j->i} and e_{i->j} of the per-direction form
        const double eji = sqrt(fmax(red_lds[pd ? kDQ + 3 * i + j : kDQ + j], 0.0));
        const double eij = sqrt(fmax(red_lds[pd ? kDQ + 3 * j + i : kDQ + i], 0.0));
        myout = a3 / (8.0 * R.alpha_lb) * (2.0 * cr[0] + 2.0 * cr[1] - 2.0 * cr[2]) +
                0.25 * a3 * (ni * eji + nj * eij);
      }
      if (valid && out != nullptr) out[po] = myout;
    }
  }
  if (valid && a_out != nullptr && act) {
#pragma unroll
    for (int i = 0; i < 3; ++i) reinterpret_cast<double2*>(a_out)[i * M + ll] = x[i];
  }
  if (valid && ll == 0) *status = bad ? 4 : 0;
  __builtin_amdgcn_wave_barrier();

  if (ADJ) {
    // ---- adjoint: A^H lambda_k = v_k, v_k = dL/d(conj a_k) ----------------
    // v_k = -a^3/4 sum_j rho^_kj K a_j + w a^3/4 sum_j tau^_kj (C a_j + g_j),
    // rho^_kj = dL/dR~_kj (x2 on the diagonal), tau^ likewise for I.
    double rh[3][3], th[3][3];
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      const int i = kPi[p], j = kPj[p];
      const double f = (i == j) ? 2.0 : 1.0;
      rh[i][j] = rh[j][i] = f * dout[p];
      th[i][j] = th[j][i] = f * dout[6 + p];
    }
    double2 vk[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double2 acc = make_double2(0.0, 0.0);
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double cr = -0.25 * a3 * rh[k][j];
        const double ct = 0.25 * a3 * om * th[k][j];
        acc.x += cr * Ka[j].x + ct * (Ca[j].x + gl[j].x);
        acc.y += cr * Ka[j].y + ct * (Ca[j].y + gl[j].y);
      }
      vk[k] = act ? acc : make_double2(0.0, 0.0);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // U^H z = v  (lane r holds equation r; z_j lands in lane j)
    for (int j = 0; j < M; ++j) {
      const double2 ujj = lds_lu[j * (MAXM + 1) + j];
      const double2 inv = crecip(cconj(ujj));
      const double2 urow = (ll > j && act) ? lds_lu[j * (MAXM + 1) + ll] : make_double2(0.0, 0.0);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double2 zj = cmul(seg_bcast2<L>(vk[i], base + j), inv);
        if (ll == j) vk[i] = zj;
        if (ll > j && act) vk[i] = cfms(vk[i], cconj(urow), zj);
      }
    }
    // L^H y = z  (unit diagonal)
    for (int k = M - 1; k >= 0; --k) {
      const double2 lrow = (ll < k) ? lds_lu[k * (MAXM + 1) + ll] : make_double2(0.0, 0.0);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double2 yk = seg_bcast2<L>(vk[i], base + k);
        if (ll < k) vk[i] = cfms(vk[i], cconj(lrow), yk);
      }
    }
    // lambda = P^T y: lane r (original row r) takes y[order(r)]
    const int src = base + (order >= 0 ? order : ll);
    double acc = 0.0;
    double2 lam[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      lam[i] = make_double2(shfl_d(vk[i].x, src), shfl_d(vk[i].y, src));
      if (act) {
        const double2 t = make_double2(gl[i].x + Ca[i].x, gl[i].y + Ca[i].y);
        acc -= cmulc(lam[i], t).y;  // -Im lambda^H (g + C_M a)
      }
    }
    // explicit omega-dependence of I (prefactor w): sum_p tau_p I_p / w
    if (ll >= 6 && ll < 12) acc += dout[ll] * iout / om;
    const double tot = seg_sum<L>(acc);
    if (valid && ll == 0) *dom = tot * dscale;
    __builtin_amdgcn_wave_barrier();

    // ---- sigma_1 dL/dsigma_1 for the material-1 part (C_M1, g_1, E_1) of
    // C_M, g and E: the right-hand side of the sensitivity system is
    // i w (g_1 + C_M1 a), and I depends on sigma_1 explicitly through the
    // same three parts (basis frozen, K_M independent of sigma)
    if (ms.CM1 != nullptr) {
      const double2* C1 = reinterpret_cast<const double2*>(ms.CM1);
      const double2* g1v = reinterpret_cast<const double2*>(ms.g1);
      double2 C1a[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) C1a[i] = make_double2(0.0, 0.0);
#pragma unroll 4
      for (int j = 0; j < M; ++j) {
        double2 aj[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) aj[i] = seg_bcast2<L>(x[i], base + j);
        if (act) {
          const double2 cc = cconj(C1[j * M + ll]);  // Hermitian: row ll from column ll
#pragma unroll
          for (int i = 0; i < 3; ++i) C1a[i] = cfma(C1a[i], cc, aj[i]);
        }
      }
      const double c4 = 0.25 * a3 * om;
      double accs = 0.0;
      if (act) {
        double2 g1l[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          g1l[i] = g1v[i * M + ll];
          const double2 t = make_double2(g1l[i].x + C1a[i].x, g1l[i].y + C1a[i].y);
          accs -= om * cmulc(lam[i], t).y;  // -w Im lambda^H (g_1 + C_M1 a)
        }
#pragma unroll
        for (int p = 0; p < 6; ++p) {
          const int i = kPi[p], j = kPj[p];
          accs += dout[6 + p] * c4 *
                  (cmulc(x[i], C1a[j]).x + cmulc(x[i], g1l[j]).x + cmulc(g1l[i], x[j]).x);
        }
      }
      if (ll == 0) {
#pragma unroll
        for (int p = 0; p < 6; ++p) accs += dout[6 + p] * c4 * ms.E1[3 * kPi[p] + kPj[p]];
      }
      const double tots = seg_sum<L>(accs);
      if (valid && ll == 0) *dsig = tots;
      __builtin_amdgcn_wave_barrier();
    }
  }
}

// ---------------------------------------------------------------- kernels
template <int MAXM, bool ADJ>
__global__ __launch_bounds__(256) void k_sweep(const mpt_rom R, const double* __restrict__ omega,
                                               int64_t n, double* __restrict__ out,
                                               double* __restrict__ a_out,
                                               int32_t* __restrict__ status,
                                               const double* __restrict__ dout,
                                               double* __restrict__ dom, const MatSens ms) {
  constexpr int L = SegOf<MAXM>::L, S = SegOf<MAXM>::S;
  extern __shared__ double2 lds[];
  __shared__ double red[4 * 64 * S];
  const int wave = threadIdx.x >> 6;
  const int wpg = blockDim.x >> 6;
  const int seg = __lane_id() / L;
  double2* my_lds = ADJ ? lds + ((size_t)wave * S + seg) * MAXM * (MAXM + 1) : nullptr;
  double* my_red = red + (wave * S + seg) * 64;
  // evaluation at w sigma / sigma0 when a conductivity is given
  const double sc = ms.sigma ? ms.sigma[0] * ms.inv_sigma0 : 1.0;
  for (int64_t k0 = ((int64_t)blockIdx.x * wpg + wave) * S; k0 < n;
       k0 += (int64_t)gridDim.x * wpg * S) {
    const int64_t k = k0 + seg;
    const bool valid = k < n;
    const int64_t kc = valid ? k : n - 1;
    sweep_point<MAXM, ADJ>(R, omega[kc] * sc, valid, out ? out + 18 * kc : nullptr,
                           a_out ? a_out + (size_t)kc * 6 * R.M : nullptr, status + kc,
                           ADJ ? dout + 18 * kc : nullptr, ADJ ? dom + kc : nullptr, my_lds,
                           my_red, ms, ms.dsig ? ms.dsig + kc : nullptr, sc);
  }
}

// Persistent batched kernel: waves pull work items (object, omega range)
// from a queue ordered by decreasing cost; one instantiation per M bucket.
template <int MAXM, bool ADJ>
__global__ __launch_bounds__(256) void k_sweep_persistent(
    const mpt_rom* __restrict__ roms, const int4* __restrict__ items, int n_items,
    unsigned int* __restrict__ counter, const double* __restrict__ omega,
    double* __restrict__ out, int32_t* __restrict__ status, const double* __restrict__ dout,
    double* __restrict__ dom) {
  constexpr int L = SegOf<MAXM>::L, S = SegOf<MAXM>::S;
  extern __shared__ double2 lds[];
  __shared__ double red[4 * 64 * S];
  const int wave = threadIdx.x >> 6;
  const int seg = __lane_id() / L;
  double2* my_lds = ADJ ? lds + ((size_t)wave * S + seg) * MAXM * (MAXM + 1) : nullptr;
  double* my_red = red + (wave * S + seg) * 64;
  while (true) {
    int it = 0;
    if (__lane_id() == 0) it = (int)atomicAdd(counter, 1u);
    it = __builtin_amdgcn_readfirstlane(it);
    if (it >= n_items) break;
    const int4 w = items[it];  // x: object, y: first row, z: count
    const mpt_rom R = roms[w.x];
    for (int r = 0; r < w.z; r += S) {
      const bool valid = r + seg < w.z;
      const int64_t k = (int64_t)w.y + (valid ? r + seg : w.z - 1);
      sweep_point<MAXM, ADJ>(R, omega[k], valid, out ? out + 18 * k : nullptr, nullptr, status + k,
                             ADJ ? dout + 18 * k : nullptr, ADJ ? dom + k : nullptr, my_lds,
                             my_red, MatSens{}, nullptr);
    }
  }
}

template <int MAXM, bool ADJ>
hipError_t launch_plain(const mpt_rom& R, const double* omega, int64_t n, double* out,
                        double* a_out, int32_t* status, const double* dout, double* dom, int wpg,
                        const MatSens& ms, hipStream_t st) {
  constexpr int S = SegOf<MAXM>::S;
  const int64_t waves = (n + S - 1) / S;
  int64_t groups = (waves + wpg - 1) / wpg;
  if (groups > 65535 * 8) groups = 65535 * 8;
  const size_t lds = ADJ ? (size_t)wpg * S * MAXM * (MAXM + 1) * sizeof(double2) : 0;
  hipLaunchKernelGGL((k_sweep<MAXM, ADJ>), dim3((unsigned)groups), dim3(64 * wpg), lds, st, R,
                     omega, n, out, a_out, status, dout, dom, ms);
  return hipGetLastError();
}

template <int MAXM, bool ADJ>
hipError_t launch_persistent(const mpt_rom* roms, const int4* items, int n_items,
                             unsigned int* counter, const double* omega, double* out,
                             int32_t* status, const double* dout, double* dom, int wpg,
                             int groups, hipStream_t st) {
  constexpr int S = SegOf<MAXM>::S;
  const size_t lds = ADJ ? (size_t)wpg * S * MAXM * (MAXM + 1) * sizeof(double2) : 0;
  hipLaunchKernelGGL((k_sweep_persistent<MAXM, ADJ>), dim3(groups), dim3(64 * wpg), lds, st, roms,
                     items, n_items, counter, omega, out, status, dout, dom);
  return hipGetLastError();
}

}  // namespace mpt
