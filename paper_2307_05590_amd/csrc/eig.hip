// Hermitian eigen-decomposition of a small matrix (n <= 192) by cyclic
// two-sided Jacobi with the parallel round-robin ordering.
//
// Each round rotates n/2 disjoint index pairs at once.  With the rotations of
// a round fixed, every 2x2 block A[{p1,q1},{p2,q2}] transforms independently
// (Q1^H B Q2), so one pass over the blocks of the upper triangle applies the
// whole round.  Only the upper triangle is stored (packed, in LDS when it
// fits), so a round reads and writes each stored entry once.  The rotations
// of every round are recorded and a second kernel, one wave per row of V,
// accumulates the eigenvector matrix V = prod Q (rows of V are independent),
// keeping the sequential kernel's work to A.
//
// Rotation test: |a_pq| > tol sqrt(|a_pp a_qq|) (keeps the relative accuracy
// of the small eigenvalues of graded Gram matrices) and |a_pq| > floor * max
// |a_ii| (entries under the rounding level of the data need no rotation).
#include "device_util.h"
#include "kernels.h"

namespace mpt {

constexpr int kJacobiMaxN = 192;
constexpr int kJacobiThreads = 1024;
constexpr int kJacobiMaxBlk = ((kJacobiMaxN / 2) * (kJacobiMaxN / 2 + 1) / 2 + kJacobiThreads - 1) /
                              kJacobiThreads;
constexpr size_t kJacobiLdsBudget = 150 * 1024;

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

// packed upper triangle: entry (i, j), i <= j
__device__ __forceinline__ int upos(int i, int j, int n) { return i * (2 * n - i + 1) / 2 + (j - i); }

__device__ __forceinline__ double2 uget(const double2* A, int i, int j, int n) {
  return i <= j ? A[upos(i, j, n)] : cconj(A[upos(j, i, n)]);
}
__device__ __forceinline__ void uset(double2* A, int i, int j, int n, double2 v) {
  if (i <= j) A[upos(i, j, n)] = v;
  else A[upos(j, i, n)] = cconj(v);
}

// Q = [[c, s], [-s ph, c ph]]: right product B Q2 on columns (0, 1) of a 2x2
__device__ __forceinline__ void rot_right(double2& b00, double2& b01, double2& b10, double2& b11,
                                          const Rot& R) {
  const double c = R.c, s = R.s;
  const double2 t0 = cmul(b01, R.ph), t1 = cmul(b11, R.ph);
  const double2 n00 = make_double2(c * b00.x - s * t0.x, c * b00.y - s * t0.y);
  const double2 n01 = make_double2(s * b00.x + c * t0.x, s * b00.y + c * t0.y);
  const double2 n10 = make_double2(c * b10.x - s * t1.x, c * b10.y - s * t1.y);
  const double2 n11 = make_double2(s * b10.x + c * t1.x, s * b10.y + c * t1.y);
  b00 = n00; b01 = n01; b10 = n10; b11 = n11;
}
// left product Q1^H B on rows (0, 1)
__device__ __forceinline__ void rot_left(double2& b00, double2& b01, double2& b10, double2& b11,
                                         const Rot& R) {
  const double c = R.c, s = R.s;
  const double2 phc = cconj(R.ph);
  const double2 t0 = cmul(b10, phc), t1 = cmul(b11, phc);
  const double2 n00 = make_double2(c * b00.x - s * t0.x, c * b00.y - s * t0.y);
  const double2 n01 = make_double2(c * b01.x - s * t1.x, c * b01.y - s * t1.y);
  const double2 n10 = make_double2(s * b00.x + c * t0.x, s * b00.y + c * t0.y);
  const double2 n11 = make_double2(s * b01.x + c * t1.x, s * b01.y + c * t1.y);
  b00 = n00; b01 = n01; b10 = n10; b11 = n11;
}

// A: packed upper triangle (LDS copy when SHARED_A, else the global scratch Ap)
template <bool SHARED_A, int KB>
__global__ __launch_bounds__(kJacobiThreads) void k_jacobi(const double2* __restrict__ Ag, int n,
                                                           double2* __restrict__ Ap,
                                                           double* __restrict__ lam,
                                                           Rot* __restrict__ rec,
                                                           int* __restrict__ info, int max_sweeps,
                                                           double tol, double floor_rel) {
  extern __shared__ double2 smem[];
  __shared__ Rot rot[kJacobiMaxN / 2];
  __shared__ int pq[kJacobiMaxN / 2];
  __shared__ int nrot;
  __shared__ double dmax;
  double2* A = SHARED_A ? smem : Ap;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < n * n; i += nt) {
    const int r = i / n, c = i % n;
    if (r <= c) A[upos(r, c, n)] = Ag[i];
  }
  const int ne = n + (n & 1);
  const int np = ne / 2;
  const int nblk = np * (np + 1) / 2;
  // this thread's blocks e = tid + k nt of the slot triangle: (ta <= tb)
  int blk[KB];
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const int e = tid + k * nt;
    blk[k] = -1;
    if (e < nblk) {
      int t1 = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
      while ((t1 + 1) * (t1 + 2) / 2 <= e) ++t1;
      while (t1 * (t1 + 1) / 2 > e) --t1;
      blk[k] = (e - t1 * (t1 + 1) / 2) | (t1 << 16);
    }
  }
  int sweep = 0;
  bool converged = false;
  __syncthreads();
  for (; sweep < max_sweeps; ++sweep) {
    if (tid < 64) {
      double m = 0.0;
      for (int i = tid; i < n; i += 64) m = fmax(m, fabs(A[upos(i, i, n)].x));
      m = wave_max(m);
      if (tid == 0) {
        dmax = m;
        nrot = 0;
      }
    }
    __syncthreads();
    const double floor_abs = floor_rel * dmax;
    // would this sweep rotate at all?  A sweep that rotates nothing leaves A
    // unchanged, so testing every pair once on A as it stands is the same
    // test; the converged case then costs one barrier instead of a sweep of
    // rounds (and records no identity rotations)
    for (int idx = tid; idx < n * n; idx += nt) {
      const int p = idx / n, q = idx % n;
      if (q > p) {
        const double a = A[upos(p, p, n)].x, d = A[upos(q, q, n)].x;
        const double2 b = A[upos(p, q, n)];
        const double ab = sqrt(b.x * b.x + b.y * b.y);
        if (ab > floor_abs && ab > 1e-300 && ab > tol * sqrt(fabs(a * d))) nrot = 1;
      }
    }
    __syncthreads();
    if (nrot == 0) {  // every thread reads the same value after the barrier
      converged = true;
      break;
    }
    __syncthreads();  // all have read nrot
    if (tid == 0) nrot = 0;  // counts the rotations of this sweep again
    __syncthreads();
    for (int r = 0; r < ne - 1; ++r) {
      if (tid < np) {
        const int t = tid;
        int p, q;
        rr_pair(t, r, ne, p, q);
        Rot R = {1.0, 0.0, make_double2(1.0, 0.0)};
        if (q < n) {
          const double a = A[upos(p, p, n)].x, d = A[upos(q, q, n)].x;
          const double2 b = A[upos(p, q, n)];
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
        pq[t] = p | (q << 16);
        rec[((size_t)sweep * (ne - 1) + r) * np + t] = R;
      }
      __syncthreads();
      // gather every entry of this thread's blocks first (blocks are disjoint,
      // so no read below depends on a write of this round), then rotate/store
      double2 bv[KB][4];
      int bpos[KB][4];
      unsigned bconj[KB];
      bool act[KB];
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        act[k] = false;
        bconj[k] = 0u;
        if (blk[k] < 0) continue;
        const int ta = blk[k] & 0xffff, tb = blk[k] >> 16;
        if (rot[ta].s == 0.0 && rot[tb].s == 0.0) continue;
        act[k] = true;
        const int pq1 = pq[ta], pq2 = pq[tb];
        const int r0 = pq1 & 0xffff, r1 = pq1 >> 16, c0 = pq2 & 0xffff, c1 = pq2 >> 16;
        const int rr[4] = {r0, r0, r1, r1}, cc[4] = {c0, c1, c0, c1};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = rr[u], j = cc[u];
          const bool ok = i < n && j < n && !(ta == tb && u == 2);
          const bool cj = i > j;
          bpos[k][u] = ok ? (cj ? upos(j, i, n) : upos(i, j, n)) : -1;
          if (cj) bconj[k] |= 1u << u;
          bv[k][u] = ok ? A[bpos[k][u]] : make_double2(0.0, 0.0);
        }
      }
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        if (!act[k]) continue;
        const int ta = blk[k] & 0xffff, tb = blk[k] >> 16;
        const Rot R1 = rot[ta], R2 = rot[tb];
        double2 b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) b[u] = (bconj[k] >> u) & 1u ? cconj(bv[k][u]) : bv[k][u];
        if (ta == tb) b[2] = cconj(b[1]);  // (q, p) of a diagonal block
        if (R2.s != 0.0) rot_right(b[0], b[1], b[2], b[3], R2);
        if (R1.s != 0.0) rot_left(b[0], b[1], b[2], b[3], R1);
        if (ta == tb) {  // exactly diagonal after the rotation
          b[0].y = 0.0;
          b[3].y = 0.0;
          b[1] = make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (bpos[k][u] >= 0) A[bpos[k][u]] = (bconj[k] >> u) & 1u ? cconj(b[u]) : b[u];
      }
      __syncthreads();
    }
    const bool done = nrot == 0;
    __syncthreads();
    if (done) {
      converged = true;
      break;
    }
  }
  for (int i = tid; i < n; i += nt) lam[i] = A[upos(i, i, n)].x;
  if (tid == 0) {
    info[0] = converged ? sweep : -1;              // sweeps that rotated
    info[2] = converged ? sweep : max_sweeps;      // recorded sweeps
  }
}

// V = prod of the recorded rotations; one wave per row of V (rows are
// independent), the row in LDS, the disjoint pairs of a round applied by the
// lanes.  The waves of a workgroup share the rotation record: chunks of
// kVecChunk rounds are staged in LDS once per workgroup, the next chunk
// loaded while the current one is applied.
constexpr int kVecWaves = 16;
constexpr int kVecChunk = 8;
constexpr int kVecMaxNp = kJacobiMaxN / 2;

__global__ __launch_bounds__(64 * kVecWaves) void k_jacobi_vectors(int n,
                                                                   const Rot* __restrict__ rec,
                                                                   const int* __restrict__ info,
                                                                   double2* __restrict__ V) {
  __shared__ double2 rows[kVecWaves][kJacobiMaxN];
  __shared__ Rot stage[2][kVecChunk * kVecMaxNp];
  const int wave = threadIdx.x >> 6;
  const int lane = __lane_id();
  const int k = blockIdx.x * kVecWaves + wave;
  const bool live = k < n;  // idle waves still take part in the staging
  double2* row = rows[wave];
  if (live)
    for (int j = lane; j < n; j += 64) row[j] = make_double2(j == k ? 1.0 : 0.0, 0.0);
  const int ne = n + (n & 1);
  const int np = ne / 2;
  const int total = info[2] * (ne - 1);
  const int nchunk = (total + kVecChunk - 1) / kVecChunk;
  // one staged rotation per thread and chunk (kVecChunk * np <= block size):
  // fetched into registers before a chunk is applied, stored to LDS after it
  static_assert(kVecChunk * kVecMaxNp <= 64 * kVecWaves, "one rotation per thread");
  const int i = threadIdx.x;
  auto fetch = [&](int c, Rot& R) {
    const int g0 = c * kVecChunk;
    const int cnt = min(kVecChunk, total - g0) * np;
    if (i < cnt) R = rec[(size_t)g0 * np + i];
  };
  Rot pre = {1.0, 0.0, make_double2(1.0, 0.0)};
  if (nchunk > 0) {
    fetch(0, pre);
    if (i < kVecChunk * kVecMaxNp) stage[0][i] = pre;
  }
  __syncthreads();
  for (int c = 0; c < nchunk; ++c) {
    if (c + 1 < nchunk) fetch(c + 1, pre);
    const int g0 = c * kVecChunk;
    const int cnt = min(kVecChunk, total - g0);
    const Rot* sr = stage[c & 1];
    if (live) {
      for (int u = 0; u < cnt; ++u) {
        const int r = (g0 + u) % (ne - 1);
        for (int t = lane; t < np; t += 64) {
          const Rot R = sr[u * np + t];
          if (R.s == 0.0) continue;
          int p, q;
          rr_pair(t, r, ne, p, q);
          if (q >= n) continue;
          const double2 vp = row[p], vq = row[q];
          const double2 t2 = cmul(vq, R.ph);
          row[p] = make_double2(R.c * vp.x - R.s * t2.x, R.c * vp.y - R.s * t2.y);
          row[q] = make_double2(R.s * vp.x + R.c * t2.x, R.s * vp.y + R.c * t2.y);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    if (c + 1 < nchunk && i < kVecChunk * kVecMaxNp) stage[(c + 1) & 1][i] = pre;
    __syncthreads();
  }
  if (live)
    for (int j = lane; j < n; j += 64) V[(size_t)k * n + j] = row[j];
}

static size_t jacobi_packed_bytes(int n) { return (size_t)n * (n + 1) / 2 * sizeof(double2); }

size_t jacobi_ws_size(int n, int max_sweeps) {
  const int ne = n + (n & 1);
  const size_t recb = (size_t)max_sweeps * (ne - 1) * (ne / 2) * sizeof(Rot);
  return (recb + 255) / 256 * 256 + jacobi_packed_bytes(n);
}

hipError_t jacobi_launch(double* A, int n, double* V, double* lam, int* info, void* ws,
                         int max_sweeps, double tol, double floor_rel, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (n > kJacobiMaxN) return hipErrorInvalidValue;
  Rot* rec = reinterpret_cast<Rot*>(ws);
  const int ne = n + (n & 1);
  const size_t recb = (size_t)max_sweeps * (ne - 1) * (ne / 2) * sizeof(Rot);
  double2* Ap = reinterpret_cast<double2*>(reinterpret_cast<char*>(ws) + (recb + 255) / 256 * 256);
  const size_t lds = jacobi_packed_bytes(n);
  const double2* Ag = reinterpret_cast<const double2*>(A);
  const int np = ne / 2;
  const int kb = (np * (np + 1) / 2 + kJacobiThreads - 1) / kJacobiThreads;  // blocks per thread
#define MPT_JAC(SH, KB_)                                                                    \
  hipLaunchKernelGGL((k_jacobi<SH, KB_>), dim3(1), dim3(kJacobiThreads), SH ? lds : 0, st, Ag, \
                     n, Ap, lam, rec, info, max_sweeps, tol, floor_rel)
  if (lds <= kJacobiLdsBudget) {
    if (kb <= 1) MPT_JAC(true, 1);
    else if (kb <= 2) MPT_JAC(true, 2);
    else MPT_JAC(true, 3);
  } else {
    if (kb <= 3) MPT_JAC(false, 3);
    else MPT_JAC(false, kJacobiMaxBlk);
  }
#undef MPT_JAC
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_jacobi_vectors, dim3((n + kVecWaves - 1) / kVecWaves), dim3(64 * kVecWaves),
                     0, st, n, rec, info, reinterpret_cast<double2*>(V));
  return hipGetLastError();
}

}  // namespace mpt
