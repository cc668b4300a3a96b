// C ABI of libmpt: handles, argument validation, and the orchestration of the
// POD basis (a1), Galerkin projection (a2), sweep (a3+a4), selection (a5),
// batched persistent sweep in a HIP graph (a6) and adjoint sweep (a7).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "device_util.h"
#include "kernels.h"

// Scratch of mpt_select_snapshots_static (per-interval argmax): a static
// device array, so that call allocates nothing.  Each GPU holds its own copy
// until the process ends; host code uses only the per-device address that
// hipGetSymbolAddress returns (select_scratch_ptr), never the array's name.
static __device__ __align__(256) int64_t scratch[MPT_SELECT_STATIC_MAX_SNAP];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

struct mpt_handle_s {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  int n_cu = 256;
  int* host_M = nullptr;  // pinned
  // cached graph of the last batched launch
  hipGraphExec_t gexec = nullptr;
  std::vector<int64_t> gkey;
  hipStream_t cap = nullptr;  // private stream used only to record graphs
  // private stream and events of mpt_project_pencil (the reduction runs beside
  // the certificate data)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // key of the plan (jobs, per-object arguments, work items) that the last
  // batched pencil call uploaded into its caller's buffer
  std::vector<int64_t> pkey;
  int pn[4] = {0, 0, 0, 0};
  int pmaxM = 0;
  int pmaxRef = 0;
};

namespace {

mpt_status fail(mpt_handle h, mpt_status s, const std::string& m) {
  if (h) h->err = m;
  return s;
}

#define HIP_OK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(h, MPT_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
  } while (0)

#define ARG(cond, msg)                                  \
  do {                                                  \
    if (!(cond)) return fail(h, MPT_E_ARG, (msg));      \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// allow_dirs: the entry point takes the per-direction form (mpt_sweep only)
mpt_status check_rom(mpt_handle h, const mpt_rom* R, bool allow_dirs = false) {
  ARG(R != nullptr, "rom is NULL");
  ARG(R->M >= 1 && R->M <= 96, "rom M must be in [1, 96]");
  ARG(R->KM && R->A0 && R->CM && R->g && R->G && R->Dp && R->s_ref && R->E && R->N0,
      "rom has a NULL matrix");
  ARG(R->n_ref >= 1 && R->n_ref <= 64, "rom n_ref must be in [1, 64]");
  ARG(R->alpha > 0.0 && R->alpha_lb > 0.0, "rom alpha and alpha_lb must be positive");
  if (R->dirs[0] != 0 || R->dirs[1] != 0 || R->dirs[2] != 0) {
    if (!allow_dirs) return fail(h, MPT_E_UNSUPPORTED, "a per-direction rom needs mpt_sweep");
    ARG(R->dirs[0] >= 1 && R->dirs[1] >= 1 && R->dirs[2] >= 1 &&
            R->dirs[0] + R->dirs[1] + R->dirs[2] == R->M,
        "rom dirs must hold three widths >= 1 that sum to M");
    ARG(R->M <= 64, "the per-direction form takes M <= 64");
  }
  return MPT_OK;
}

}  // namespace

// ------------------------------------------------------------- small kernels
namespace mpt {

// sort eigenvalues (descending), singular values, truncation rank and the
// scaled rotation W (m x Mcap): W[:, j] = V[:, idx_j] / sigma_j for j < M
// Number of pass-1 eigenvalues (ascending) under h times the largest: the
// tail whose eigenvectors pass 1 leaves mixed (absolute accuracy eps lam_max).
__global__ void k_pod_tail(const double* __restrict__ lam, int m, double h, int* __restrict__ nt) {
  if (threadIdx.x == 0) {
    int n = 0;
    while (n < m && lam[n] < h * lam[m - 1]) ++n;
    nt[0] = n;
  }
}

// V' = [V0_T VT | V0_H]: the tail columns of the pass-1 eigenvectors turned
// by the eigenvectors VT (nt x nt) of the tail's own Gram
__global__ void k_pod_tail_mix(const double2* __restrict__ V0, int m, int nt,
                               const double2* __restrict__ VT, double2* __restrict__ Vout) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < m * m; e += gridDim.x * blockDim.x) {
    const int r = e / m, j = e % m;
    double2 acc = make_double2(0.0, 0.0);
    if (j < nt) {
      for (int k = 0; k < nt; ++k) acc = cfma(acc, V0[(size_t)r * m + k], VT[(size_t)k * nt + j]);
    } else {
      acc = V0[(size_t)r * m + j];
    }
    Vout[e] = acc;
  }
}

// Columns of the rotated snapshots that enter the Jacobi: squared norm >=
// floor * the largest (the others lie under the numerical rank floor and
// no truncation keeps them).  Compacts their Gram into Gc (n' x n', in
// index order) and lists them in live.
__global__ void k_pod_live(const double2* __restrict__ G, int m, double floor,
                           double2* __restrict__ Gc, int* __restrict__ live,
                           int* __restrict__ nlive) {
  __shared__ int idx[192];
  __shared__ int cnt;
  const int t = threadIdx.x;
  if (t == 0) {
    double dmax = 0.0;
    for (int j = 0; j < m; ++j) dmax = fmax(dmax, G[(size_t)j * m + j].x);
    int n = 0;
    for (int j = 0; j < m; ++j)
      if (dmax > 0.0 && G[(size_t)j * m + j].x >= floor * dmax) idx[n++] = j;
    cnt = n;
    nlive[0] = n;
  }
  __syncthreads();
  const int n = cnt;
  for (int e = t; e < n * n; e += blockDim.x) {
    const int r = e / n, c = e % n;
    Gc[e] = G[(size_t)idx[r] * m + idx[c]];
  }
  for (int j = t; j < n; j += blockDim.x) live[j] = idx[j];
}

// Number of tail eigenvalues (ascending, nt of them) under rel times the
// largest: directions the tail's own eigen-decomposition cannot resolve
__global__ void k_pod_dead(const double* __restrict__ lam, int nt, double rel, int* __restrict__ nd) {
  if (threadIdx.x == 0) {
    int n = 0;
    while (n < nt && lam[n] < rel * lam[nt - 1]) ++n;
    nd[0] = n;
  }
}

// Singular values of all nq + nd directions - the Jacobi's n eigenvalues, the
// squared norms of the nq - n columns it left out, and the nd unresolved tail
// eigenvalues lamd - sorted descending; M by the truncation rule; W (nq x
// Mcap) = the kept eigenvectors scattered back to the nq columns of the
// rotated snapshots and divided by their singular values.
__global__ void k_pod_finalize(const double* __restrict__ lam, const double2* __restrict__ V,
                               int n, const int* __restrict__ live,
                               const double2* __restrict__ G, int nq,
                               const double* __restrict__ lamd, int nd, double tol, int Mcap,
                               double* __restrict__ sigma, double2* __restrict__ W,
                               int* __restrict__ Mout) {
  __shared__ int src[192];   // sorted entry -> eigenpair (>= 0) or < 0 for the others
  __shared__ double sv[192];
  __shared__ double val[192];
  __shared__ int code[192];
  __shared__ int pos[192];   // column -> its row of V, or -1 when left out
  __shared__ int Msh;
  const int t = threadIdx.x;
  const int m = nq + nd;
  if (t < nq) pos[t] = -1;
  __syncthreads();
  if (t < n) pos[live[t]] = t;
  __syncthreads();
  if (t == 0) {  // entries: the n eigenvalues, the left-out columns, the tail remainder
    int k = n;
    for (int j = 0; j < nq; ++j)
      if (pos[j] < 0) {
        val[k] = G[(size_t)j * nq + j].x;
        code[k++] = -1;
      }
    for (int j = 0; j < nd; ++j) {
      val[k] = lamd[j];
      code[k++] = -1;
    }
  }
  if (t < n) {
    val[t] = lam[t];
    code[t] = t;
  }
  __syncthreads();
  if (t < m) {
    const double li = val[t];
    int rank = 0;
    for (int j = 0; j < m; ++j) {
      const double lj = val[j];
      if (lj > li || (lj == li && j < t)) ++rank;
    }
    src[rank] = code[t];
    sv[rank] = sqrt(fmax(li, 0.0));
  }
  __syncthreads();
  if (t == 0) {
    int M = 0;
    const double s1 = sv[0];
    if (s1 > 0.0)
      for (int j = 0; j < m; ++j)
        if (sv[j] / s1 >= tol) ++M;
    M = min(M, min(Mcap, m));
    while (M > 0 && M < m && sv[M] / sv[M - 1] > 1.0 - 1e-8) --M;
    for (int j = 0; j < M; ++j)  // only resolved directions are kept
      if (src[j] < 0) {
        M = j;
        break;
      }
    Msh = M;
    *Mout = M;
  }
  __syncthreads();
  if (t < m) sigma[t] = sv[t];
  for (int e = t; e < nq * Mcap; e += blockDim.x) {
    const int r = e / Mcap, j = e % Mcap;
    double2 v = make_double2(0.0, 0.0);
    if (j < Msh && pos[r] >= 0) {
      const double2 x = V[(size_t)pos[r] * n + src[j]];
      const double inv = 1.0 / sv[j];
      v = make_double2(x.x * inv, x.y * inv);
    }
    W[(size_t)r * Mcap + j] = v;
  }
}

// Zc = sqrt(c) [w (3) | U (M)] on the n_c conductor rows
__global__ void k_gather_cond(const int32_t* __restrict__ cond, int64_t nc,
                              const double* __restrict__ c, const double* __restrict__ w,
                              const double2* __restrict__ U, int64_t ldU, int M,
                              double2* __restrict__ Zc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = nc * (M + 3);
  if (e >= tot) return;
  const int64_t r = e / (M + 3);
  const int j = (int)(e % (M + 3));
  const int64_t row = cond[r];
  const double sc = sqrt(c[row]);
  if (j < 3) {
    Zc[e] = make_double2(sc * w[row * 3 + j], 0.0);
  } else {
    const double2 u = U[row * ldU + (j - 3)];
    Zc[e] = make_double2(sc * u.x, sc * u.y);
  }
}

// o^T K o (3 x 3, real; o is N x 3 row-major) for the static tensor N0: one
// row per thread, (K o)_r in registers, the nine products summed per
// workgroup (wave sums, then the waves in order) into part[block][9]
constexpr int kOkoThreads = 256;
__global__ __launch_bounds__(kOkoThreads) void k_oko_partial(int64_t N,
                                                             const int32_t* __restrict__ rowptr,
                                                             const int32_t* __restrict__ colind,
                                                             const double* __restrict__ val,
                                                             const double* __restrict__ o,
                                                             double* __restrict__ part) {
  __shared__ double sh[kOkoThreads / 64][9];
  const int64_t r = (int64_t)blockIdx.x * kOkoThreads + threadIdx.x;
  double y[3] = {0.0, 0.0, 0.0}, orow[3] = {0.0, 0.0, 0.0};
  if (r < N) {
    const int b = rowptr[r], e = rowptr[r + 1];
#pragma unroll 4
    for (int k = b; k < e; ++k) {
      const double v = val[k];
      const int64_t c = colind[k];
#pragma unroll
      for (int j = 0; j < 3; ++j) y[j] = fma(v, o[3 * c + j], y[j]);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) orow[i] = o[3 * r + i];
  }
  const int lane = __lane_id(), wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double s = wave_sum(orow[i] * y[j]);
      if (lane == 0) sh[wave][3 * i + j] = s;
    }
  __syncthreads();
  if (threadIdx.x < 9) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kOkoThreads / 64; ++w) s += sh[w][threadIdx.x];
    part[(size_t)blockIdx.x * 9 + threadIdx.x] = s;
  }
}

// No[e] = sum of the partials of entry e (wave e, fixed order), imaginary part 0
__global__ __launch_bounds__(576) void k_oko_sum(const double* __restrict__ part, int nb,
                                                 double2* __restrict__ No) {
  const int lane = __lane_id(), e = threadIdx.x >> 6;
  double s = 0.0;
  for (int p = lane; p < nb; p += 64) s += part[(size_t)p * 9 + e];
  s = wave_sum(s);
  if (lane == 0) No[e] = make_double2(s, 0.0);
}

// assemble K_M, A0, C_M, g, E, N0 from the small contractions
//   KMt (M x M = U^H K U), UhU (M x M), P ((M+3)^2 = Zc^H Zc: C_M, g and E),
//   No (3 x 3, = o^T K o in the real parts, or NULL)
__global__ void k_assemble(int M, double eps_h, const double2* __restrict__ KMt,
                           const double2* __restrict__ UhU, const double2* __restrict__ P,
                           const double2* __restrict__ No, const double* __restrict__ vol,
                           double alpha, double2* __restrict__ KMo, double2* __restrict__ A0,
                           double2* __restrict__ CM, double2* __restrict__ g,
                           double* __restrict__ E, double* __restrict__ N0) {
  const int L = M + 3;
  // K_M, U^H U and C_M are Hermitian by definition; the two computed
  // triangles are averaged (the sweep reads them column-wise)
  auto herm = [&](const double2* X, int ld, int off, int i, int j) {
    const double2 u = X[(off + i) * ld + off + j], t = X[(off + j) * ld + off + i];
    return make_double2(0.5 * (u.x + t.x), 0.5 * (u.y - t.y));
  };
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int nthreads = gridDim.x * blockDim.x;
  for (int e = tid; e < M * M; e += nthreads) {
    const int i = e / M, j = e % M;
    const double2 k = herm(KMt, M, 0, i, j), u = herm(UhU, M, 0, i, j);
    KMo[e] = k;
    A0[e] = make_double2(fma(eps_h, u.x, k.x), fma(eps_h, u.y, k.y));
    CM[e] = herm(P, L, 3, i, j);
  }
  for (int e = tid; e < 3 * M; e += nthreads) {
    const int i = e / M, m = e % M;
    g[e] = P[(3 + m) * L + i];  // g_i[m] = (U_c^H c w_i)[m]
  }
  if (tid < 9) {
    const int i = tid / 3, j = tid % 3;
    E[tid] = 0.5 * (P[i * L + j].x + P[j * L + i].x);
    const double a3 = alpha * alpha * alpha;
    double n0 = (i == j) ? a3 * vol[i] : 0.0;
    if (No) n0 += 0.25 * a3 * No[tid].x;
    N0[tid] = n0;
  }
}

}  // namespace mpt

using namespace mpt;

// ------------------------------------------------------------------- handle
extern "C" mpt_status mpt_create(int device, void* hip_stream, mpt_handle* out) {
  mpt_handle h = nullptr;
  if (!out) return MPT_E_ARG;
  h = new mpt_handle_s();
  h->device = device;
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) {
    delete h;
    return MPT_E_HIP;
  }
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
      ncu > 0)
    h->n_cu = ncu;
  if (hipHostMalloc(reinterpret_cast<void**>(&h->host_M), 4 * sizeof(int), 0) != hipSuccess) {
    delete h;
    return MPT_E_HIP;
  }
  // address of this device's copy of the static selection scratch, looked up
  // once per device with the device current
  if (device >= 0 && device < kMaxDevices) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
      void* p = nullptr;
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        hipHostFree(h->host_M);
        delete h;
        return MPT_E_HIP;
      }
      g_scratch_ptr[device] = p;
    }
  }
  *out = h;
  return MPT_OK;
}

extern "C" mpt_status mpt_destroy(mpt_handle h) {
  if (!h) return MPT_E_ARG;
  hipSetDevice(h->device);
  if (h->stream) hipStreamSynchronize(h->stream);
  else hipDeviceSynchronize();
  if (h->gexec) hipGraphExecDestroy(h->gexec);
  if (h->cap) hipStreamDestroy(h->cap);
  if (h->side) hipStreamDestroy(h->side);
  if (h->ev_fork) hipEventDestroy(h->ev_fork);
  if (h->ev_join) hipEventDestroy(h->ev_join);
  if (h->host_M) hipHostFree(h->host_M);
  delete h;
  return MPT_OK;
}

extern "C" mpt_status mpt_set_stream(mpt_handle h, void* hip_stream) {
  if (!h) return MPT_E_ARG;
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return MPT_OK;
}

extern "C" const char* mpt_last_error(mpt_handle h) { return h ? h->err.c_str() : "null handle"; }

extern "C" int mpt_max_reduced_dim(void) { return 96; }

// ------------------------------------------------------------------ a1 POD
constexpr int kJacobiSweeps = 40;
// absolute rotation floor of the pass-2 Jacobi (times max |g_ii|)
constexpr double kJacobiFloor = 1e-30;
// relative singular values below this are rounding noise of FP64 data: the
// truncation never keeps them, even for a fixed-rank request (tol_sigma = 0)
constexpr double kRankFloor = 1e-12;

// pass-1 eigenvalues under this times the largest form the tail that gets a
// Gram and an eigen-decomposition of its own before pass 2
constexpr double kTailRel = 1e-10;
// tail eigenvalues under this times the tail's largest are beyond what its
// eigen-decomposition resolves (absolute accuracy ~eps of the largest):
// their directions stay out of pass 2 (singular values under
// sqrt(64 eps kTailRel) s_1 ~ 1.2e-12 s_1, at the rank floor)
constexpr double kDeadRel = 64.0 * 2.220446049250313e-16;
// pass-2 columns with squared norms under this times the largest stay out of
// the Jacobi: their singular values lie under 1e-13 s_1, below kRankFloor
constexpr double kLiveFloor = 1e-26;

static void pod_layout(int64_t N, int m, size_t* off) {
  // 0 G0, 1 V0, 2 lam, 3 Q1, 4 gram ws, 5 W, 6 info, 7 Mdev, 8 eigen ws,
  // 9 compact Gram, 10 live columns, 11 unresolved tail eigenvalues, 12 end
  size_t o = 0;
  off[0] = o; o = align256(o + (size_t)m * m * 16);
  off[1] = o; o = align256(o + (size_t)m * m * 16);
  off[2] = o; o = align256(o + (size_t)m * 8);
  off[3] = o; o = align256(o + (size_t)N * m * 16);
  off[4] = o; o = align256(o + gram_ws_size(N, m, m));
  off[5] = o; o = align256(o + (size_t)m * 192 * 16);
  off[6] = o; o = align256(o + 64);
  off[7] = o; o = align256(o + 64);
  off[8] = o; o = align256(o + std::max(jacobi_ws_size(m, kJacobiSweeps), tridiag_ws_size(m)));
  off[9] = o; o = align256(o + (size_t)m * m * 16);
  off[10] = o; o = align256(o + (size_t)m * 4);
  off[11] = o; o = align256(o + (size_t)m * 8);
  off[12] = o;
}

extern "C" size_t mpt_pod_basis_ws_size(int64_t N, int ncol) {
  if (N <= 0 || ncol <= 0) return 0;
  size_t off[13];
  pod_layout(N, ncol, off);
  return off[12];
}

extern "C" mpt_status mpt_pod_basis(mpt_handle h, const double* D, int64_t ldD, int64_t N,
                                    int ncol, double tol_sigma, int M_cap, double* U, int64_t ldU,
                                    double* sigma, int* M_out, void* ws, size_t ws_bytes) {
  if (!h) return MPT_E_ARG;
  ARG(D && U && sigma && M_out && ws, "NULL pointer");
  ARG(N > 0 && ncol >= 1 && ncol <= 192, "need N > 0 and 1 <= ncol <= 192");
  ARG(ldD >= ncol && ldU >= M_cap && M_cap >= 1, "bad leading dimension or M_cap");
  ARG(tol_sigma >= 0.0 && tol_sigma < 1.0, "tol_sigma must be in [0, 1)");
  ARG(ws_bytes >= mpt_pod_basis_ws_size(N, ncol), "workspace too small");
  HIP_OK(hipSetDevice(h->device));
  const int m = ncol;
  const int Mc = std::min(M_cap, m);
  size_t off[13];
  pod_layout(N, m, off);
  char* w = reinterpret_cast<char*>(ws);
  double* G0 = reinterpret_cast<double*>(w + off[0]);
  double* V0 = reinterpret_cast<double*>(w + off[1]);
  double* lam = reinterpret_cast<double*>(w + off[2]);
  double* Q1 = reinterpret_cast<double*>(w + off[3]);
  void* gws = w + off[4];
  double* W = reinterpret_cast<double*>(w + off[5]);
  int* info = reinterpret_cast<int*>(w + off[6]);
  int* Mdev = reinterpret_cast<int*>(w + off[7]);
  void* jws = w + off[8];
  double* Gc = reinterpret_cast<double*>(w + off[9]);
  int* live = reinterpret_cast<int*>(w + off[10]);
  double* lamd = reinterpret_cast<double*>(w + off[11]);
  hipStream_t st = h->stream;
  // pass 1: G0 = D^H D, eigenvectors V0 (absolute accuracy eps lam_max)
  HIP_OK(gram_launch(D, ldD, D, ldD, N, m, m, G0, m, gws, st));
  HIP_OK(hipMemsetAsync(info, 0, 4 * sizeof(int), st));
  HIP_OK(tridiag_eig_launch(G0, m, V0, lam, jws, st));
  // the tail (pass-1 eigenvalues under kTailRel lam_max) is an arbitrary
  // mixture of the small singular directions: its columns D V0_T get a Gram
  // and an eigen-decomposition of their own, which resolves them on their
  // scale, so that the pass-2 Gram is close to diagonal and the Jacobi
  // converges in a few sweeps
  hipLaunchKernelGGL(k_pod_tail, dim3(1), dim3(64), 0, st, lam, m, kTailRel, Mdev + 1);
  HIP_OK(hipGetLastError());
  HIP_OK(hipMemcpyAsync(h->host_M + 1, Mdev + 1, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  const int nt = h->host_M[1];
  const double* Vr = V0;
  int nd = 0;  // unresolved tail directions, left out from here on
  if (nt >= 2) {
    HIP_OK(rotate_launch(D, ldD, N, m, V0, m, nt, Q1, nt, st));            // D V0_T
    HIP_OK(gram_launch(Q1, nt, Q1, nt, N, nt, nt, Gc, nt, gws, st));        // its Gram
    HIP_OK(tridiag_eig_launch(Gc, nt, W, lam, jws, st));                    // VT, ascending
    hipLaunchKernelGGL(k_pod_tail_mix, dim3((m * m + 255) / 256), dim3(256), 0, st,
                       reinterpret_cast<const double2*>(V0), m, nt,
                       reinterpret_cast<const double2*>(W), reinterpret_cast<double2*>(G0));
    HIP_OK(hipGetLastError());
    hipLaunchKernelGGL(k_pod_dead, dim3(1), dim3(64), 0, st, lam, nt, kDeadRel, Mdev + 2);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(h->host_M + 2, Mdev + 2, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    nd = h->host_M[2];
    if (nd > 0)
      HIP_OK(hipMemcpyAsync(lamd, lam, (size_t)nd * sizeof(double), hipMemcpyDeviceToDevice, st));
    Vr = G0;
  }
  // Q1 = D V' over the resolved directions (columns nd.. of V')
  const int nq = m - nd;
  HIP_OK(rotate_launch(D, ldD, N, m, Vr + 2 * nd, m, nq, Q1, nq, st));
  // pass 2 on the rotated snapshots (graded Gram): Jacobi on the columns
  // above the floor (relative accuracy of the small singular values)
  HIP_OK(gram_launch(Q1, nq, Q1, nq, N, nq, nq, G0, nq, gws, st));
  hipLaunchKernelGGL(k_pod_live, dim3(1), dim3(256), 0, st,
                     reinterpret_cast<const double2*>(G0), nq, kLiveFloor,
                     reinterpret_cast<double2*>(Gc), live, Mdev + 1);
  HIP_OK(hipGetLastError());
  HIP_OK(hipMemcpyAsync(h->host_M + 1, Mdev + 1, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  const int nl = h->host_M[1];
  if (nl > 0)
    HIP_OK(jacobi_launch(Gc, nl, V0, lam, info + 1, jws, kJacobiSweeps,
                         4.0 * nl * 2.220446049250313e-16, kJacobiFloor, st));
  hipLaunchKernelGGL(k_pod_finalize, dim3(1), dim3(256), 0, st, lam,
                     reinterpret_cast<const double2*>(V0), nl, live,
                     reinterpret_cast<const double2*>(G0), nq, lamd, nd,
                     std::max(tol_sigma, kRankFloor), Mc, sigma,
                     reinterpret_cast<double2*>(W), Mdev);
  HIP_OK(hipGetLastError());
  // M to the host, then U = Q1 W on the M kept columns, columns M..M_cap-1
  // cleared in the same pass
  HIP_OK(hipMemcpyAsync(h->host_M, Mdev, sizeof(int), hipMemcpyDeviceToHost, st));
  int hinfo[4] = {0, 0, 0, 0};
  HIP_OK(hipMemcpyAsync(hinfo, info, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  const int M = *h->host_M;
  if (hinfo[0] < 0 || hinfo[1] < 0) return fail(h, MPT_E_NOTPD, "Jacobi did not converge");
  HIP_OK(rotate_launch(Q1, nq, N, nq, W, Mc, M, U, ldU, st, M_cap));
  *M_out = M;
  return MPT_OK;
}

// ---------------------------------------------------------- a2 projection
static void proj_layout(int64_t N, int M, int64_t nc, int n_ref, size_t* off) {
  const int L = M + 3;
  const int64_t gN = std::max<int64_t>(N, nc);
  size_t o = 0;
  off[0] = o; o = align256(o + (size_t)N * M * 16);         // Y (when not given)
  off[1] = o; o = align256(o + (size_t)M * M * 16);         // UhU
  off[2] = o; o = align256(o + (size_t)nc * L * 16);        // Zc
  off[3] = o; o = align256(o + (size_t)L * L * 16);         // P = Zc^H Zc
  off[4] = o; o = align256(o + (size_t)((N + 255) / 256) * 9 * 8);  // o^T K o partials
  off[5] = o;
  off[6] = o; o = align256(o + 9 * 16);                     // No
  off[7] = o; o = align256(o + (size_t)M * M * 16);         // U^H K U before symmetrising
  off[8] = o; o = align256(o + std::max(gram2c_ws_size(gN, L, L), gram2c_ws_size(gN, M, M)));
  off[9] = o; o = align256(o + cert_ws_size(M, nc, n_ref));
  off[10] = o; o = align256(o + (size_t)M * M * 16);        // U^H conj(K U)
  off[11] = o; o = align256(o + (size_t)M * M * 16);        // U^H conj(U)
  off[12] = o; o = align256(o + (size_t)L * L * 16);        // Zc^H conj(Zc)
  off[13] = o;
}

extern "C" size_t mpt_project_ws_size(int64_t N, int M, int64_t n_c, int n_ref) {
  if (N <= 0 || M <= 0 || n_ref <= 0) return 0;
  size_t off[14];
  proj_layout(N, M, n_c, n_ref, off);
  return off[13];
}

static bool row_blocks_ok(const mpt_csr& K) {
  return K.row_blocks >= 0 && (K.row_blocks <= 1 || K.n % K.row_blocks == 0);
}

extern "C" mpt_status mpt_spmm(mpt_handle h, const mpt_csr* K, const double* U, int64_t ldU,
                               int M, double* Y, int64_t ldY) {
  if (!h) return MPT_E_ARG;
  ARG(K && K->rowptr && K->colind && K->val && U && Y, "NULL pointer");
  ARG(K->n > 0 && K->nnz >= 0 && K->nnz < (int64_t)1 << 31, "bad CSR sizes");
  ARG(row_blocks_ok(*K), "row_blocks must be >= 0 and divide n");
  ARG(M >= 1 && ldU >= M && ldY >= M, "bad M or leading dimensions");
  HIP_OK(hipSetDevice(h->device));
  HIP_OK(spmm_launch(*K, U, ldU, M, Y, ldY, h->stream));
  return MPT_OK;
}

// dirs: NULL (joint basis) or the three per-direction widths (host)
static mpt_status project_impl(mpt_handle h, const mpt_csr* K, const double* c, double eps_h,
                               const double* w, const double* o, const double* vol, double alpha,
                               const double* U, int64_t ldU, int M, const int32_t* dirs,
                               const int32_t* cond, int64_t n_c, const double* Vt,
                               const double* lam, int n_ref, const double* s_ref, double* KM,
                               double* A0, double* CM, double* g, double* G, double* Dp, double* E,
                               double* N0, double* Y, void* ws, size_t ws_bytes,
                               char* pbuf = nullptr) {
  if (!h) return MPT_E_ARG;
  ARG(K && K->rowptr && K->colind && K->val && c && w && vol && U && cond && Vt && lam && s_ref,
      "NULL input");
  ARG(KM && A0 && CM && g && G && Dp && E && N0 && ws, "NULL output");
  ARG(K->n > 0 && M >= 1 && M <= mpt_max_reduced_dim() && ldU >= M && n_c >= 1 && n_c <= K->n,
      "bad sizes");
  ARG(n_ref >= 1 && n_ref <= 64, "n_ref must be in [1, 64]");
  ARG(row_blocks_ok(*K), "row_blocks must be >= 0 and divide n");
  ARG(eps_h >= 0.0 && alpha > 0.0, "bad eps_h or alpha");
  ARG(ws_bytes >= mpt_project_ws_size(K->n, M, n_c, n_ref), "workspace too small");
  HIP_OK(hipSetDevice(h->device));
  hipStream_t st = h->stream;
  const int64_t N = K->n;
  const int L = M + 3;
  size_t off[14];
  proj_layout(N, M, n_c, n_ref, off);
  char* wsb = reinterpret_cast<char*>(ws);
  double* Yb = Y ? Y : reinterpret_cast<double*>(wsb + off[0]);
  const int64_t ldY = M;
  double* UhU = reinterpret_cast<double*>(wsb + off[1]);
  double* Zc = reinterpret_cast<double*>(wsb + off[2]);
  double* P = reinterpret_cast<double*>(wsb + off[3]);
  double* OkoPart = reinterpret_cast<double*>(wsb + off[4]);
  double* No = reinterpret_cast<double*>(wsb + off[6]);
  double* KMt = reinterpret_cast<double*>(wsb + off[7]);
  void* gws = wsb + off[8];
  void* cws = wsb + off[9];
  double* TXk = reinterpret_cast<double*>(wsb + off[10]);
  double* TXu = reinterpret_cast<double*>(wsb + off[11]);
  double* TCz = reinterpret_cast<double*>(wsb + off[12]);

  // Y = K U; K_M = U^H Y (Hermitian: K is real symmetric), U^H U and, from
  // the same products, U^H conj(Y), U^H conj(U) (the conjugation defect's T_X)
  HIP_OK(spmm_launch(*K, U, ldU, M, Yb, ldY, st));
  HIP_OK(gram2c_launch(U, ldU, Yb, ldY, N, M, M, KMt, M, UhU, M, TXk, M, TXu, M, true, gws, st));
  // conductor rows: Zc = sqrt(c) [w | U], P = Zc^H Zc (C_M, g, E) and Zc^H conj(Zc)
  {
    const int64_t tot = n_c * L;
    hipLaunchKernelGGL(k_gather_cond, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, cond,
                       n_c, c, w, reinterpret_cast<const double2*>(U), ldU, M,
                       reinterpret_cast<double2*>(Zc));
    HIP_OK(hipGetLastError());
  }
  HIP_OK(gram2c_launch(Zc, L, Zc, L, n_c, L, L, P, L, nullptr, 0, TCz, L, nullptr, 0, false, gws,
                       st));
  // static tensor: o^T K o (o real)
  const double2* Nop = nullptr;
  if (o) {
    const int64_t nb = (N + kOkoThreads - 1) / kOkoThreads;
    hipLaunchKernelGGL(k_oko_partial, dim3((unsigned)nb), dim3(kOkoThreads), 0, st, N, K->rowptr,
                       K->colind, K->val, o, OkoPart);
    HIP_OK(hipGetLastError());
    hipLaunchKernelGGL(k_oko_sum, dim3(1), dim3(576), 0, st, OkoPart, (int)nb,
                       reinterpret_cast<double2*>(No));
    HIP_OK(hipGetLastError());
    Nop = reinterpret_cast<const double2*>(No);
  }
  hipLaunchKernelGGL(k_assemble, dim3(64), dim3(256), 0, st, M, eps_h,
                     reinterpret_cast<const double2*>(KMt), reinterpret_cast<const double2*>(UhU),
                     reinterpret_cast<const double2*>(P), Nop, vol, alpha,
                     reinterpret_cast<double2*>(KM), reinterpret_cast<double2*>(A0),
                     reinterpret_cast<double2*>(CM), reinterpret_cast<double2*>(g), E, N0);
  HIP_OK(hipGetLastError());
  // pencil form requested: its reduction needs A0, C_M and g only, so it runs
  // on the private stream while this stream computes the certificate data
  const mpt::PencilJob job{M,  n_ref, A0, CM, KM, G, Dp, s_ref, g, E, N0, pbuf};
  if (pbuf) {
    HIP_OK(hipEventRecord(h->ev_fork, st));
    HIP_OK(hipStreamWaitEvent(h->side, h->ev_fork, 0));
    HIP_OK(mpt::pencil_core_launch(job, nullptr, 1, M, h->side));
    HIP_OK(hipEventRecord(h->ev_join, h->side));
  }
  // certificate data per reference shift: G_s and D'_s (Lemma 4.1)
  HIP_OK(cert_launch(M, Zc, n_c, Vt, lam, n_ref, s_ref, A0, CM, UhU, TXk, TXu, TCz, eps_h, dirs,
                     G, Dp, cws, st));
  if (pbuf) {
    HIP_OK(hipStreamWaitEvent(st, h->ev_join, 0));
    HIP_OK(mpt::pencil_layout_launch(job, nullptr, 1, n_ref, st));
  }
  return MPT_OK;
}

extern "C" mpt_status mpt_project(mpt_handle h, const mpt_csr* K, const double* c, double eps_h,
                                  const double* w, const double* o, const double* vol,
                                  double alpha, const double* U, int64_t ldU, int M,
                                  const int32_t* cond, int64_t n_c, const double* Vt,
                                  const double* lam, int n_ref, const double* s_ref, double* KM,
                                  double* A0, double* CM, double* g, double* G, double* Dp,
                                  double* E, double* N0, double* Y, void* ws, size_t ws_bytes) {
  return project_impl(h, K, c, eps_h, w, o, vol, alpha, U, ldU, M, nullptr, cond, n_c, Vt, lam,
                      n_ref, s_ref, KM, A0, CM, g, G, Dp, E, N0, Y, ws, ws_bytes);
}

extern "C" mpt_status mpt_project_pencil(
    mpt_handle h, const mpt_csr* K, const double* c, double eps_h, const double* w,
    const double* o, const double* vol, double alpha, const double* U, int64_t ldU, int M,
    const int32_t* cond, int64_t n_c, const double* Vt, const double* lam, int n_ref,
    const double* s_ref, double* KM, double* A0, double* CM, double* g, double* G, double* Dp,
    double* E, double* N0, double* Y, void* ws, size_t ws_bytes, void* pbuf, size_t pbytes,
    double alpha_lb, mpt_pencil* pen) {
  if (!h) return MPT_E_ARG;
  ARG(pbuf != nullptr && pen != nullptr, "NULL pencil buffer/out");
  ARG(alpha_lb > 0.0, "alpha_lb must be positive");
  ARG(M >= 1 && M <= 96, "the pencil form takes 1 <= M <= 96");
  ARG(n_ref >= 1 && n_ref <= mpt::kPenMaxRef, "the pencil form takes 1 <= n_ref <= 64");
  if (pbytes < mpt::pencil_total_bytes(M, n_ref))
    return fail(h, MPT_E_NOMEM, "pencil buffer smaller than mpt_pencil_bytes");
  HIP_OK(hipSetDevice(h->device));
  if (!h->side) HIP_OK(hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
  if (!h->ev_fork) HIP_OK(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
  if (!h->ev_join) HIP_OK(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
  mpt_status s = project_impl(h, K, c, eps_h, w, o, vol, alpha, U, ldU, M, nullptr, cond, n_c,
                              Vt, lam, n_ref, s_ref, KM, A0, CM, g, G, Dp, E, N0, Y, ws,
                              ws_bytes, static_cast<char*>(pbuf));
  if (s != MPT_OK) return s;
  const mpt::PencilLayout L = mpt::pencil_layout(M);
  char* b = static_cast<char*>(pbuf);
  pen->M = M;
  pen->n_ref = n_ref;
  pen->H = reinterpret_cast<const double*>(b + L.H);
  pen->T = reinterpret_cast<const double*>(b + L.T);
  pen->f = reinterpret_cast<const double*>(b + L.f);
  pen->Z = reinterpret_cast<const double*>(b + L.Z);
  pen->W = reinterpret_cast<const double*>(b + L.W);
  pen->S = reinterpret_cast<const double*>(b + L.S);
  pen->alpha = alpha;
  pen->alpha_lb = alpha_lb;
  return MPT_OK;
}

extern "C" mpt_status mpt_project_dirs(mpt_handle h, const mpt_csr* K, const double* c,
                                       double eps_h, const double* w, const double* o,
                                       const double* vol, double alpha, const double* U,
                                       int64_t ldU, int M, const int32_t* dirs,
                                       const int32_t* cond, int64_t n_c, const double* Vt,
                                       const double* lam, int n_ref, const double* s_ref,
                                       double* KM, double* A0, double* CM, double* g, double* G,
                                       double* Dp, double* E, double* N0, double* Y, void* ws,
                                       size_t ws_bytes) {
  if (!h) return MPT_E_ARG;
  ARG(dirs && dirs[0] >= 1 && dirs[1] >= 1 && dirs[2] >= 1 && dirs[0] + dirs[1] + dirs[2] == M,
      "dirs must hold three widths >= 1 that sum to M");
  ARG(M <= 64, "the per-direction form takes M <= 64");
  return project_impl(h, K, c, eps_h, w, o, vol, alpha, U, ldU, M, dirs, cond, n_c, Vt, lam,
                      n_ref, s_ref, KM, A0, CM, g, G, Dp, E, N0, Y, ws, ws_bytes);
}

// ----------------------------------------- residual Gram from X^{-1} Z
// G = (P + P^H) / 2 for the L x L contraction P = Z^H (X^{-1} Z)
__global__ void k_herm_mean(const double2* __restrict__ P, int L, double2* __restrict__ G) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= L * L) return;
  const int i = e / L, j = e % L;
  const double2 u = P[i * L + j], t = P[j * L + i];
  G[e] = make_double2(0.5 * (u.x + t.x), 0.5 * (u.y - t.y));
}

extern "C" size_t mpt_residual_gram_ws_size(int64_t N, int M) {
  if (N < 1 || M < 1 || M > mpt_max_reduced_dim()) return 0;
  const int L = 2 * M + 3;
  return align256((size_t)L * L * sizeof(double2)) + mpt::gram_ws_size(N, L, L);
}

extern "C" mpt_status mpt_residual_gram(mpt_handle h, const double* Z, int64_t ldZ,
                                        const double* XinvZ, int64_t ldY, int64_t N, int M,
                                        double* G, void* ws, size_t ws_bytes) {
  if (!h) return MPT_E_ARG;
  ARG(Z && XinvZ && G && ws, "NULL pointer");
  ARG(N >= 1 && M >= 1 && M <= mpt_max_reduced_dim(), "bad N or M");
  const int L = 2 * M + 3;
  ARG(ldZ >= L && ldY >= L, "leading dimensions below 2M+3");
  ARG(ws_bytes >= mpt_residual_gram_ws_size(N, M), "workspace too small");
  HIP_OK(hipSetDevice(h->device));
  hipStream_t st = h->stream;
  char* wsb = reinterpret_cast<char*>(ws);
  double* P = reinterpret_cast<double*>(wsb);
  void* gws = wsb + align256((size_t)L * L * sizeof(double2));
  HIP_OK(gram_launch(Z, ldZ, XinvZ, ldY, N, L, L, P, L, gws, st));
  hipLaunchKernelGGL(k_herm_mean, dim3((L * L + 255) / 256), dim3(256), 0, st,
                     reinterpret_cast<const double2*>(P), L, reinterpret_cast<double2*>(G));
  HIP_OK(hipGetLastError());
  return MPT_OK;
}

// ------------------------------------------------------------ a3+a4 sweep
extern "C" mpt_status mpt_sweep(mpt_handle h, const mpt_rom* rom, const double* omega,
                                int64_t n_omega, double* out, double* a_out, int32_t* status) {
  if (!h) return MPT_E_ARG;
  mpt_status s = check_rom(h, rom, true);
  if (s != MPT_OK) return s;
  ARG(n_omega >= 0, "n_omega < 0");
  ARG(n_omega == 0 || (omega && out && status), "NULL omega/out/status");
  HIP_OK(hipSetDevice(h->device));
  HIP_OK(sweep_launch(*rom, omega, n_omega, out, a_out, status, nullptr, nullptr, h->stream));
  return MPT_OK;
}

extern "C" mpt_status mpt_sweep_adjoint(mpt_handle h, const mpt_rom* rom, const double* omega,
                                        int64_t n, const double* dout, double* dL_domega,
                                        double* sig_dsig, int32_t* status) {
  if (!h) return MPT_E_ARG;
  mpt_status s = check_rom(h, rom);
  if (s != MPT_OK) return s;
  if (rom->M > 64) return fail(h, MPT_E_UNSUPPORTED, "the adjoint sweep takes M <= 64");
  ARG(n >= 1, "n must be >= 1");
  ARG(omega && dout && dL_domega && sig_dsig && status, "NULL pointer");
  HIP_OK(hipSetDevice(h->device));
  // the forward outputs are not kept (out = NULL)
  HIP_OK(sweep_launch(*rom, omega, n, nullptr, nullptr, status, dout, dL_domega, h->stream));
  HIP_OK(sigma_reduce_one(omega, dL_domega, n, nullptr, sig_dsig, h->stream));
  return MPT_OK;
}

extern "C" mpt_status mpt_signature(mpt_handle h, const mpt_rom* rom, const double* omega,
                                    int64_t n, const double* sigma, double sigma0, double* out,
                                    int32_t* status) {
  if (!h) return MPT_E_ARG;
  mpt_status s = check_rom(h, rom);
  if (s != MPT_OK) return s;
  if (rom->M > 64) return fail(h, MPT_E_UNSUPPORTED, "the signature form takes M <= 64");
  ARG(n >= 0, "n < 0");
  ARG(sigma && sigma0 > 0.0, "need a conductivity pointer and sigma0 > 0");
  ARG(n == 0 || (omega && out && status), "NULL omega/out/status");
  HIP_OK(hipSetDevice(h->device));
  mpt::MatSens ms;
  ms.sigma = sigma;
  ms.inv_sigma0 = 1.0 / sigma0;
  HIP_OK(sweep_launch(*rom, omega, n, out, nullptr, status, nullptr, nullptr, h->stream, ms));
  return MPT_OK;
}

extern "C" mpt_status mpt_signature_adjoint(mpt_handle h, const mpt_rom* rom,
                                            const double* omega, int64_t n, const double* sigma,
                                            double sigma0, const double* dout,
                                            double* dL_domega, double* dL_dsigma,
                                            int32_t* status) {
  if (!h) return MPT_E_ARG;
  mpt_status s = check_rom(h, rom);
  if (s != MPT_OK) return s;
  if (rom->M > 64) return fail(h, MPT_E_UNSUPPORTED, "the signature form takes M <= 64");
  ARG(n >= 1, "n must be >= 1");
  ARG(sigma && sigma0 > 0.0, "need a conductivity pointer and sigma0 > 0");
  ARG(omega && dout && dL_domega && dL_dsigma && status, "NULL pointer");
  HIP_OK(hipSetDevice(h->device));
  mpt::MatSens ms;
  ms.sigma = sigma;
  ms.inv_sigma0 = 1.0 / sigma0;
  HIP_OK(sweep_launch(*rom, omega, n, nullptr, nullptr, status, dout, dL_domega, h->stream, ms));
  // the model depends on w sigma only: dL/dsigma = sum_k w_k dL/dw_k / sigma
  HIP_OK(sigma_reduce_one(omega, dL_domega, n, sigma, dL_dsigma, h->stream));
  return MPT_OK;
}

extern "C" size_t mpt_sweep_adjoint_materials_ws_size(int64_t n) {
  return n < 1 ? 0 : align256((size_t)n * 8);
}

extern "C" mpt_status mpt_sweep_adjoint_materials(mpt_handle h, const mpt_rom* rom,
                                                  const double* CM1, const double* g1,
                                                  const double* E1, const double* omega,
                                                  int64_t n, const double* dout,
                                                  double* dL_domega, double* sig_dsig,
                                                  int32_t* status, void* ws, size_t ws_bytes) {
  if (!h) return MPT_E_ARG;
  mpt_status s = check_rom(h, rom);
  if (s != MPT_OK) return s;
  if (rom->M > 64) return fail(h, MPT_E_UNSUPPORTED, "the adjoint sweep takes M <= 64");
  ARG(n >= 1, "n must be >= 1");
  ARG(CM1 && g1 && E1, "NULL material part");
  ARG(omega && dout && dL_domega && sig_dsig && status && ws, "NULL pointer");
  ARG(ws_bytes >= mpt_sweep_adjoint_materials_ws_size(n), "workspace too small");
  HIP_OK(hipSetDevice(h->device));
  // ws: the per-frequency sigma_1 terms
  double* dsig = reinterpret_cast<double*>(ws);
  mpt::MatSens ms;
  ms.CM1 = CM1;
  ms.g1 = g1;
  ms.E1 = E1;
  ms.dsig = dsig;
  HIP_OK(sweep_launch(*rom, omega, n, nullptr, nullptr, status, dout, dL_domega, h->stream, ms));
  HIP_OK(mpt::material_reduce(omega, dL_domega, dsig, n, sig_dsig, h->stream));
  return MPT_OK;
}

// ------------------------------------------------------ pencil form sweep
extern "C" size_t mpt_pencil_bytes(int M, int n_ref) {
  if (M < 1 || M > 96 || n_ref < 1 || n_ref > mpt::kPenMaxRef) return 0;
  return mpt::pencil_total_bytes(M, n_ref);
}

extern "C" mpt_status mpt_pencil_reduce(mpt_handle h, const mpt_rom* rom, void* buf,
                                        size_t bytes, mpt_pencil* out) {
  if (!h) return MPT_E_ARG;
  mpt_status s = check_rom(h, rom);
  if (s != MPT_OK) return s;
  ARG(buf != nullptr && out != nullptr, "NULL buf/out");
  const mpt::PencilLayout L = mpt::pencil_layout(rom->M);
  if (bytes < mpt::pencil_total_bytes(rom->M, rom->n_ref))
    return fail(h, MPT_E_NOMEM, "pencil buffer smaller than mpt_pencil_bytes");
  HIP_OK(hipSetDevice(h->device));
  mpt::PencilJob job{rom->M,     rom->n_ref, rom->A0, rom->CM, rom->KM, rom->G,
                     rom->Dp,    rom->s_ref, rom->g,  rom->E,  rom->N0, static_cast<char*>(buf)};
  HIP_OK(mpt::pencil_reduce_launch(job, nullptr, 1, rom->M, rom->n_ref, h->stream));
  char* b = static_cast<char*>(buf);
  out->M = rom->M;
  out->n_ref = rom->n_ref;
  out->H = reinterpret_cast<const double*>(b + L.H);
  out->T = reinterpret_cast<const double*>(b + L.T);
  out->f = reinterpret_cast<const double*>(b + L.f);
  out->Z = reinterpret_cast<const double*>(b + L.Z);
  out->W = reinterpret_cast<const double*>(b + L.W);
  out->S = reinterpret_cast<const double*>(b + L.S);
  out->alpha = rom->alpha;
  out->alpha_lb = rom->alpha_lb;
  return MPT_OK;
}

extern "C" mpt_status mpt_sweep_pencil(mpt_handle h, const mpt_pencil* pen, const double* omega,
                                       int64_t n_omega, double* out, double* a_out,
                                       int32_t* status) {
  if (!h) return MPT_E_ARG;
  ARG(pen != nullptr, "pencil is NULL");
  ARG(pen->M >= 1 && pen->M <= 96, "pencil M must be in [1, 96]");
  ARG(pen->n_ref >= 1 && pen->n_ref <= mpt::kPenMaxRef, "pencil n_ref must be in [1, 64]");
  ARG(pen->H && pen->T && pen->f && pen->Z && pen->W && pen->S, "pencil has a NULL part");
  ARG(pen->alpha > 0.0 && pen->alpha_lb > 0.0, "pencil alpha and alpha_lb must be positive");
  ARG(n_omega >= 0, "n_omega < 0");
  ARG(n_omega == 0 || (omega && out && status), "NULL omega/out/status");
  HIP_OK(hipSetDevice(h->device));
  HIP_OK(mpt::pencil_sweep_launch(mpt::pencil_args(*pen), omega, n_omega, out, a_out, status,
                                  h->stream));
  return MPT_OK;
}

// ------------------------------------------ pencil form for a dictionary
// the objects' pencils, packed in order, then the plan: jobs, per-object
// sweep arguments, work items of at most 16 frequencies (plan_items of them)
static size_t pencil_plan_bytes(int n_obj, size_t plan_items) {
  return align256(n_obj * sizeof(mpt::PencilJob)) + align256(n_obj * sizeof(mpt::PencilArgs)) +
         align256(plan_items * sizeof(int4));
}

extern "C" size_t mpt_pencil_batched_bytes(const mpt_rom* roms_host, int n_obj,
                                           const int64_t* omega_off) {
  if (!roms_host || !omega_off || n_obj < 1) return 0;
  size_t tot = 0, items = 0;
  for (int o = 0; o < n_obj; ++o) {
    const int M = roms_host[o].M;
    if (M < 1 || M > 96) return 0;
    const int nr = roms_host[o].n_ref;
    if (nr < 1 || nr > mpt::kPenMaxRef) return 0;
    tot += mpt::pencil_total_bytes(M, nr);
    const int64_t cnt = omega_off[o + 1] - omega_off[o];
    if (cnt < 0) return 0;
    items += (size_t)((cnt + 15) / 16);
  }
  return align256(tot) + pencil_plan_bytes(n_obj, items);
}

extern "C" mpt_status mpt_sweep_pencil_batched(mpt_handle h, const mpt_rom* roms_host, int n_obj,
                                               const int64_t* omega_off, const double* omega,
                                               void* buf, size_t bytes, double* out,
                                               int32_t* status) {
  if (!h) return MPT_E_ARG;
  ARG(roms_host && omega_off && omega && buf && out && status && n_obj >= 1, "NULL or empty");
  for (int o = 0; o < n_obj; ++o) {
    mpt_status s = check_rom(h, &roms_host[o]);
    if (s != MPT_OK) return s;
    ARG(omega_off[o + 1] >= omega_off[o], "omega_off must be non-decreasing");
  }
  ARG(omega_off[0] == 0, "omega_off[0] must be 0");
  if (bytes < mpt_pencil_batched_bytes(roms_host, n_obj, omega_off))
    return fail(h, MPT_E_NOMEM, "buffer smaller than mpt_pencil_batched_bytes");
  size_t pen_bytes = 0;
  for (int o = 0; o < n_obj; ++o)
    pen_bytes += mpt::pencil_total_bytes(roms_host[o].M, roms_host[o].n_ref);
  char* pb = static_cast<char*>(buf) + align256(pen_bytes);  // the plan region
  HIP_OK(hipSetDevice(h->device));
  std::vector<int64_t> key = {(int64_t)buf, (int64_t)omega, (int64_t)out, (int64_t)status, n_obj};
  for (int o = 0; o <= n_obj; ++o) key.push_back(omega_off[o]);
  for (int o = 0; o < n_obj; ++o) {
    const mpt_rom& r = roms_host[o];
    int64_t a, b;
    std::memcpy(&a, &r.alpha, 8);
    std::memcpy(&b, &r.alpha_lb, 8);
    for (int64_t v : {(int64_t)r.M, (int64_t)r.n_ref, (int64_t)r.KM, (int64_t)r.A0,
                      (int64_t)r.CM, (int64_t)r.g, (int64_t)r.G, (int64_t)r.Dp, (int64_t)r.s_ref,
                      (int64_t)r.E, (int64_t)r.N0, a, b})
      key.push_back(v);
  }
  if (key != h->pkey) {
    std::vector<mpt::PencilJob> jobs(n_obj);
    std::vector<mpt::PencilArgs> args(n_obj);
    std::vector<int4> items[4];
    char* base = static_cast<char*>(buf);
    int maxM = 1, maxRef = 1;
    for (int o = 0; o < n_obj; ++o) {
      const mpt_rom& r = roms_host[o];
      jobs[o] = mpt::PencilJob{r.M, r.n_ref, r.A0,   r.CM, r.KM, r.G,
                               r.Dp, r.s_ref, r.g, r.E, r.N0, base};
      mpt_pencil pen{};
      pen.M = r.M;
      pen.n_ref = r.n_ref;
      pen.H = reinterpret_cast<const double*>(base);
      pen.alpha = r.alpha;
      pen.alpha_lb = r.alpha_lb;
      args[o] = mpt::pencil_args(pen);
      base += mpt::pencil_total_bytes(r.M, r.n_ref);
      maxM = std::max(maxM, r.M);
      maxRef = std::max(maxRef, r.n_ref);
      const int bi = r.M <= 16 ? 0 : (r.M <= 32 ? 1 : (r.M <= 64 ? 2 : 3));
      for (int64_t k = omega_off[o]; k < omega_off[o + 1]; k += 16) {
        const int cnt = (int)std::min<int64_t>(16, omega_off[o + 1] - k);
        items[bi].push_back(make_int4(o, (int)k, cnt, 0));
      }
    }
    const size_t jb = align256(n_obj * sizeof(mpt::PencilJob));
    const size_t ab = align256(n_obj * sizeof(mpt::PencilArgs));
    const size_t ni = items[0].size() + items[1].size() + items[2].size() + items[3].size();
    std::vector<int4> all;
    all.reserve(ni);
    for (auto& v : items) all.insert(all.end(), v.begin(), v.end());
    HIP_OK(hipMemcpyAsync(pb, jobs.data(), n_obj * sizeof(mpt::PencilJob), hipMemcpyHostToDevice,
                          h->stream));
    HIP_OK(hipMemcpyAsync(pb + jb, args.data(), n_obj * sizeof(mpt::PencilArgs),
                          hipMemcpyHostToDevice, h->stream));
    if (ni)
      HIP_OK(hipMemcpyAsync(pb + jb + ab, all.data(), ni * sizeof(int4), hipMemcpyHostToDevice,
                            h->stream));
    HIP_OK(hipStreamSynchronize(h->stream));  // host vectors go out of scope
    for (int b = 0; b < 4; ++b) h->pn[b] = (int)items[b].size();
    h->pmaxM = maxM;
    h->pmaxRef = maxRef;
    h->pkey = key;
  }
  const size_t jb = align256(n_obj * sizeof(mpt::PencilJob));
  const size_t ab = align256(n_obj * sizeof(mpt::PencilArgs));
  const auto* jobs = reinterpret_cast<const mpt::PencilJob*>(pb);
  const auto* args = reinterpret_cast<const mpt::PencilArgs*>(pb + jb);
  const int4* items = reinterpret_cast<const int4*>(pb + jb + ab);
  mpt::PencilJob none{};
  HIP_OK(mpt::pencil_reduce_launch(none, jobs, n_obj, h->pmaxM, h->pmaxRef, h->stream));
  const int Ls[4] = {16, 32, 64, 96};
  int at = 0;
  for (int b = 0; b < 4; ++b) {
    HIP_OK(mpt::pencil_sweep_items_launch(Ls[b], args, items + at, h->pn[b], omega, out, status,
                                          h->stream));
    at += h->pn[b];
  }
  return MPT_OK;
}

// --------------------------------------------------- full matrix method
extern "C" size_t mpt_tensors_fmm_ws_size(int64_t N, int M) {
  if (N < 1 || M < 1) return 0;
  return mpt::fmm_ws_size(N, N, M);
}

extern "C" size_t mpt_tensors_im_ws_size(int64_t N, int64_t n_faces, int M) {
  if (N < 1 || n_faces < 1 || M < 1) return 0;
  return mpt::fmm_ws_size(N, n_faces, M);
}

extern "C" mpt_status mpt_tensors_im(mpt_handle h, const mpt_csr* curl, const double* face_w,
                                     const double* c, const double* w, const double* U,
                                     int64_t N, int64_t ldU, int M, const int32_t* cond,
                                     int64_t n_c, const double* a, const double* omega, int64_t n,
                                     const double* N0, double alpha, double* out, void* ws,
                                     size_t ws_bytes) {
  if (!h) return MPT_E_ARG;
  ARG(curl && curl->rowptr && curl->colind && curl->val && curl->n >= 1, "bad curl");
  ARG(row_blocks_ok(*curl), "row_blocks must be >= 0 and divide the row count");
  ARG(face_w && c && w && U && N0 && out && a && omega, "NULL pointer");
  ARG(N >= 1 && M >= 1 && ldU >= M, "bad N / M / ldU");
  ARG(n_c >= 0 && (n_c == 0 || cond), "bad conductor list");
  ARG(n >= 0 && alpha > 0.0, "bad n / alpha");
  if (n == 0) return MPT_OK;
  if (!ws || ws_bytes < mpt::fmm_ws_size(N, curl->n, M))
    return fail(h, MPT_E_NOMEM, "workspace smaller than mpt_tensors_im_ws_size");
  HIP_OK(hipSetDevice(h->device));
  HIP_OK(mpt::fmm_launch(*curl, face_w, c, w, U, N, ldU, M, cond, n_c, a, omega, n, N0, alpha,
                         out, ws, h->stream));
  return MPT_OK;
}

extern "C" mpt_status mpt_tensors_fmm(mpt_handle h, const mpt_csr* K, const double* c,
                                      const double* w, const double* U, int64_t ldU, int M,
                                      const int32_t* cond, int64_t n_c, const double* a,
                                      const double* omega, int64_t n, const double* N0,
                                      double alpha, double* out, void* ws, size_t ws_bytes) {
  if (!h) return MPT_E_ARG;
  ARG(K && K->rowptr && K->colind && K->val && K->n >= 1, "bad K");
  ARG(row_blocks_ok(*K), "row_blocks must be >= 0 and divide n");
  ARG(c && w && U && N0 && out && a && omega, "NULL pointer");
  ARG(M >= 1 && ldU >= M, "bad M / ldU");
  ARG(n_c >= 0 && (n_c == 0 || cond), "bad conductor list");
  ARG(n >= 0 && alpha > 0.0, "bad n / alpha");
  if (n == 0) return MPT_OK;
  if (!ws || ws_bytes < mpt::fmm_ws_size(K->n, K->n, M))
    return fail(h, MPT_E_NOMEM, "workspace smaller than mpt_tensors_fmm_ws_size");
  HIP_OK(hipSetDevice(h->device));
  HIP_OK(mpt::fmm_launch(*K, nullptr, c, w, U, K->n, ldU, M, cond, n_c, a, omega, n, N0, alpha,
                         out, ws, h->stream));
  return MPT_OK;
}

// -------------------------------------------------------------- a5 select
extern "C" size_t mpt_select_snapshots_ws_size(int n_snap) {
  return n_snap < 2 ? 0 : align256((size_t)n_snap * 8);
}

extern "C" mpt_status mpt_select_snapshots(mpt_handle h, const double* omega, int64_t n,
                                           const double* out, const double* snap, int n_snap,
                                           int n_star, double* new_omega, double* lambda,
                                           double* Lambda_max, void* ws, size_t ws_bytes) {
  if (!h) return MPT_E_ARG;
  ARG(omega && out && snap && new_omega && lambda && Lambda_max && ws, "NULL pointer");
  ARG(n >= 1 && n_snap >= 2 && n_star >= 1 && n_star <= 64, "bad sizes");
  ARG(ws_bytes >= mpt_select_snapshots_ws_size(n_snap), "workspace too small");
  HIP_OK(hipSetDevice(h->device));
  HIP_OK(select_launch(omega, n, out, snap, n_snap, n_star, new_omega, lambda, Lambda_max,
                       reinterpret_cast<int64_t*>(ws), h->stream));
  return MPT_OK;
}

extern "C" mpt_status mpt_select_snapshots_threshold(mpt_handle h, const double* omega, int64_t n,
                                                     const double* out, const double* snap,
                                                     int n_snap, double theta, double* new_omega,
                                                     int32_t* n_new, double* lambda,
                                                     double* Lambda_max, void* ws,
                                                     size_t ws_bytes) {
  if (!h) return MPT_E_ARG;
  ARG(omega && out && snap && new_omega && n_new && lambda && Lambda_max && ws, "NULL pointer");
  ARG(n >= 1 && n_snap >= 2, "bad sizes");
  ARG(theta > 0.0 && theta <= 1.0, "theta must be in (0, 1]");
  ARG(ws_bytes >= mpt_select_snapshots_ws_size(n_snap), "workspace too small");
  HIP_OK(hipSetDevice(h->device));
  HIP_OK(select_threshold_launch(omega, n, out, snap, n_snap, theta, new_omega, n_new, lambda,
                                 Lambda_max, reinterpret_cast<int64_t*>(ws), h->stream));
  return MPT_OK;
}

extern "C" mpt_status mpt_select_snapshots_static(mpt_handle h, const double* omega, int64_t n,
                                                  const double* out, const double* snap,
                                                  int n_snap, int n_star, double* new_omega,
                                                  double* lambda, double* Lambda_max) {
  if (!h) return MPT_E_ARG;
  ARG(omega && out && snap && new_omega && lambda && Lambda_max, "NULL pointer");
  ARG(n >= 1 && n_snap >= 2 && n_star >= 1 && n_star <= 64, "bad sizes");
  ARG(n_snap <= MPT_SELECT_STATIC_MAX_SNAP,
      "n_snap above MPT_SELECT_STATIC_MAX_SNAP (the static scratch's size)");
  ARG(h->device >= 0 && h->device < kMaxDevices, "device index out of range");
  void* scr = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    scr = g_scratch_ptr[h->device];
  }
  if (!scr) return fail(h, MPT_E_HIP, "static scratch address unknown for this device");
  HIP_OK(hipSetDevice(h->device));
  // every interval's slot is written before it is read: nothing to clear
  HIP_OK(select_launch(omega, n, out, snap, n_snap, n_star, new_omega, lambda, Lambda_max,
                       reinterpret_cast<int64_t*>(scr), h->stream));
  return MPT_OK;
}

// -------------------------------------------------- a6/a7 batched launches
namespace {

double sweep_cost(int M) { return 2.67 * M * M * M + 172.0 * M * M; }

struct Plan {
  std::vector<int4> items[4];
};

mpt_status build_plan(mpt_handle h, const mpt_rom* roms_host, int n_obj, const int64_t* off,
                      int per_item, Plan& plan) {
  for (int o = 0; o < n_obj; ++o) {
    mpt_status s = check_rom(h, &roms_host[o]);
    if (s != MPT_OK) return s;
    if (roms_host[o].M > 64)
      return fail(h, MPT_E_UNSUPPORTED, "batched sweeps take M <= 64");
    ARG(off[o + 1] >= off[o], "omega_off must be non-decreasing");
    const int b = bucket_of(roms_host[o].M);
    const int bi = b == 16 ? 0 : (b == 32 ? 1 : (b == 48 ? 2 : 3));
    for (int64_t k = off[o]; k < off[o + 1]; k += per_item) {
      const int cnt = (int)std::min<int64_t>(per_item, off[o + 1] - k);
      plan.items[bi].push_back(make_int4(o, (int)k, cnt, roms_host[o].M));
    }
  }
  for (auto& v : plan.items)
    std::stable_sort(v.begin(), v.end(), [](const int4& a, const int4& b) {
      return sweep_cost(a.w) * a.z > sweep_cost(b.w) * b.z;
    });
  return MPT_OK;
}

// bytes of the batched workspace: work items, counters, object offsets
size_t batched_ws_bytes(size_t nitems, int n_obj) {
  return align256(nitems * sizeof(int4)) + 256 + align256((size_t)(n_obj + 1) * 8);
}

mpt_status batched_common(mpt_handle h, const mpt_rom* roms_host, const mpt_rom* roms_dev,
                          int n_obj, const int64_t* omega_off, const double* omega, double* out,
                          int32_t* status, const mpt_tuning* tune, int use_graph,
                          const double* dout, double* dom, double* sig, void* ws,
                          size_t ws_bytes) {
  ARG(roms_host && roms_dev && omega_off && omega && status && ws && n_obj >= 1, "NULL or empty");
  ARG(out || dout, "NULL out");
  HIP_OK(hipSetDevice(h->device));
  mpt_tuning t = {8, 4, 2, 0};
  if (tune) t = *tune;
  ARG(t.omegas_per_item >= 1 && (t.waves_per_group == 1 || t.waves_per_group == 2 ||
                                 t.waves_per_group == 4) && t.groups_per_cu >= 1,
      "bad tuning");
  const bool adj = dout != nullptr;
  Plan plan;
  mpt_status s = build_plan(h, roms_host, n_obj, omega_off, t.omegas_per_item, plan);
  if (s != MPT_OK) return s;
  size_t nitems = 0;
  for (auto& v : plan.items) nitems += v.size();
  const size_t items_bytes = align256(nitems * sizeof(int4));
  const size_t cnt_off = items_bytes;
  const size_t off_off = cnt_off + 256;
  ARG(ws_bytes >= batched_ws_bytes(nitems, n_obj), "workspace smaller than mpt_sweep_batched_ws_size");
  // graph cache key: every argument the recorded launches depend on
  std::vector<int64_t> key = {(int64_t)roms_dev, (int64_t)omega, (int64_t)out, (int64_t)status,
                              (int64_t)dout, (int64_t)dom, (int64_t)sig, (int64_t)ws, n_obj,
                              t.omegas_per_item, t.waves_per_group, t.groups_per_cu, adj};
  for (auto& v : plan.items) key.push_back((int64_t)v.size());
  for (int o = 0; o <= n_obj; ++o) key.push_back(omega_off[o]);
  for (int o = 0; o < n_obj; ++o) key.push_back(roms_host[o].M);
  const bool cached = use_graph && h->gexec && key == h->gkey;
  if (!cached) {
    // the plan is rewritten into ws: a recorded graph reading that region
    // would now see another plan, so it is dropped
    if (h->gexec) {
      HIP_OK(hipGraphExecDestroy(h->gexec));
      h->gexec = nullptr;
      h->gkey.clear();
    }
    std::vector<int4> all;
    all.reserve(nitems);
    for (auto& v : plan.items) all.insert(all.end(), v.begin(), v.end());
    char* b = reinterpret_cast<char*>(ws);
    HIP_OK(hipMemcpyAsync(b, all.data(), nitems * sizeof(int4), hipMemcpyHostToDevice, h->stream));
    HIP_OK(hipMemcpyAsync(b + off_off, omega_off, (size_t)(n_obj + 1) * 8, hipMemcpyHostToDevice,
                          h->stream));
    HIP_OK(hipStreamSynchronize(h->stream));  // host vectors go out of scope
  }
  char* b = reinterpret_cast<char*>(ws);
  const int4* items = reinterpret_cast<const int4*>(b);
  unsigned int* counters = reinterpret_cast<unsigned int*>(b + cnt_off);
  const int64_t* offd = reinterpret_cast<const int64_t*>(b + off_off);
  auto enqueue = [&](hipStream_t st) -> hipError_t {
    hipError_t e = reset_counters(counters, 4, st);
    if (e != hipSuccess) return e;
    size_t base = 0;
    const int buckets[4] = {16, 32, 48, 64};
    for (int bi = 0; bi < 4; ++bi) {
      const int ni = (int)plan.items[bi].size();
      if (ni) {
        const int wpg = (adj && buckets[bi] >= 48) ? std::min(2, t.waves_per_group) : t.waves_per_group;
        int groups = h->n_cu * t.groups_per_cu;
        groups = std::max(1, std::min(groups, (ni + wpg - 1) / wpg));
        e = persistent_launch(buckets[bi], adj, roms_dev, items + base, ni, counters + bi, omega,
                              adj ? nullptr : out, status, dout, dom, wpg, groups, st);
        if (e != hipSuccess) return e;
      }
      base += ni;
    }
    if (adj) e = sigma_reduce(omega, dom, offd, n_obj, sig, st);
    return e;
  };
  if (!use_graph) {
    HIP_OK(enqueue(h->stream));
    return MPT_OK;
  }
  if (!cached) {
    // record on a private stream (the caller's may be the null stream, which
    // cannot be captured); the instantiated graph is launched on the caller's
    if (!h->cap) HIP_OK(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    HIP_OK(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue(h->cap);
    hipError_t e2 = hipStreamEndCapture(h->cap, &g);
    if (e != hipSuccess) {
      if (g) hipGraphDestroy(g);
      return fail(h, MPT_E_HIP, std::string("capture: ") + hipGetErrorString(e));
    }
    if (e2 != hipSuccess) return fail(h, MPT_E_HIP, std::string("end capture: ") + hipGetErrorString(e2));
    HIP_OK(hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0));
    HIP_OK(hipGraphDestroy(g));
    h->gkey = key;
  }
  HIP_OK(hipGraphLaunch(h->gexec, h->stream));
  return MPT_OK;
}

}  // namespace

extern "C" size_t mpt_sweep_batched_ws_size(const mpt_rom* roms_host, int n_obj,
                                            const int64_t* omega_off, const mpt_tuning* tune) {
  if (!roms_host || !omega_off || n_obj < 1) return 0;
  const int per = tune ? tune->omegas_per_item : 8;
  if (per < 1) return 0;
  size_t nitems = 0;
  for (int o = 0; o < n_obj; ++o) {
    const int64_t cnt = omega_off[o + 1] - omega_off[o];
    if (cnt < 0) return 0;
    nitems += (size_t)((cnt + per - 1) / per);
  }
  return batched_ws_bytes(nitems, n_obj);
}

extern "C" mpt_status mpt_sweep_batched(mpt_handle h, const mpt_rom* roms_host,
                                        const mpt_rom* roms_dev, int n_obj,
                                        const int64_t* omega_off, const double* omega, double* out,
                                        int32_t* status, const mpt_tuning* tune, int use_graph,
                                        void* ws, size_t ws_bytes) {
  if (!h) return MPT_E_ARG;
  ARG(out != nullptr, "NULL out");
  return batched_common(h, roms_host, roms_dev, n_obj, omega_off, omega, out, status, tune,
                        use_graph, nullptr, nullptr, nullptr, ws, ws_bytes);
}

extern "C" mpt_status mpt_sweep_adjoint_batched(mpt_handle h, const mpt_rom* roms_host,
                                                const mpt_rom* roms_dev, int n_obj,
                                                const int64_t* omega_off, const double* omega,
                                                const double* dout, double* dL_domega,
                                                double* sig_dsig, int32_t* status, void* ws,
                                                size_t ws_bytes) {
  if (!h) return MPT_E_ARG;
  ARG(dout && dL_domega && sig_dsig, "NULL adjoint pointer");
  return batched_common(h, roms_host, roms_dev, n_obj, omega_off, omega, nullptr, status, nullptr,
                        1, dout, dL_domega, sig_dsig, ws, ws_bytes);
}
