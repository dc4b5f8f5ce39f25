// Persistent Krylov solver for V sigma = b, b = |T| (Section 2.5; CG applies
// because V is symmetric positive definite, Remark (ii)), and the capacity
// reduction Cap = (1/4pi) sum sigma_i |T_i| (eq. "cap:ell").
//
// One cooperative launch holds one or many systems; each system owns a fixed
// number of workgroups (a function of N only), each workgroup a contiguous
// band of rows.  Per system the workgroups run the same state machine:
//
//   RESID  r = b - A x in FP64 (A = V, plus the FP64 sparse correction of
//          touching/near entries in mixed precision); stop if
//          ||r|| <= rtol ||b||; else start an inner CG on A d = r / ||r||.
//   CG     preconditioned CG in the Chronopoulos-Gear arrangement: the two
//          inner products of an iteration are reduced together, so an
//          iteration costs one product with V and two cross-workgroup
//          barriers.  Vectors and the matrix product are in the matrix
//          precision (FP32 products accumulate in FP32); the scalar
//          reductions are summed in FP64.
//   UPDATE x += ||r|| d in FP64, back to RESID.
//   DONE   sigma = x, Cap, result.
//
// The dense product streams V once from HBM (bandwidth-bound: 4 or 8 bytes
// per entry, 2 flops): all 256 threads of a workgroup sweep 8 rows at a time
// with 16-byte non-temporal loads, the vector comes from L2.  Every
// reduction has a fixed order, so results are bitwise reproducible and do
// not depend on which other systems share the launch.
#include <climits>

#include "bc_internal.h"

namespace bc {

enum Phase : int32_t { PH_INIT = 0, PH_RESID = 1, PH_CG = 2, PH_UPDATE = 3, PH_DONE = 4 };

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

__host__ __device__ inline void solve_offsets(int64_t N, int32_t precision, size_t &ctl, size_t &partial,
                                              size_t &x64, size_t &r64, size_t &vec, int64_t &ld) {
  ld = (N + 63) / 64 * 64;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = (o + bytes + 255) & ~size_t(255);
    return r;
  };
  ctl = take(1024);
  partial = take(sizeof(double) * 2 * 4 * kGMax);
  x64 = take(sizeof(double) * ld);
  r64 = take(sizeof(double) * ld);
  vec = take((precision == BC_FP64 ? 8 : 4) * ld * 7);
}

// ------------------------------------------------------------ barrier
struct SysBarrier {
  SolveCtl *ctl;
  int G;
  unsigned gen;
  uint32_t spin_limit;

  // All workgroups of the system; returns false if the system was aborted
  // (a barrier exceeded its spin limit somewhere).
  __device__ bool sync(int *s_flag) {
    if (G == 1) {
      __syncthreads();
      return true;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
      const unsigned target = gen + 1u;
      int ok = 1;
      unsigned prev = __hip_atomic_fetch_add(&ctl->bar_count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      if (prev == (unsigned)G - 1u) {
        __hip_atomic_store(&ctl->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctl->bar_gen, target, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        uint32_t spins = 0;
        while (__hip_atomic_load(&ctl->bar_gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != target) {
          __builtin_amdgcn_s_sleep(2);
          if (++spins > spin_limit ||
              __hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            ok = 0;
            break;
          }
        }
      }
      if (!ok) __hip_atomic_store(&ctl->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      *s_flag = ok;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    gen += 1u;
    return *s_flag != 0;
  }
};

// Workgroup sum of K values; every thread receives the totals.
template <int K>
__device__ __forceinline__ void wg_sum(double (&v)[K], double *lds) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) lds[w * K + k] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = ((lds[k] + lds[K + k]) + lds[2 * K + k]) + lds[3 * K + k];
  __syncthreads();
}

// Sum of slot values of the G workgroup partials of one set (fixed order).
template <int K>
__device__ __forceinline__ void sum_partials(const double *set, int G, const int (&slot)[K], double (&out)[K],
                                             double *lds) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double a = 0.0;
    for (int g = threadIdx.x; g < G; g += kWG) a += set[4 * g + slot[k]];
    out[k] = a;
  }
  wg_sum<K>(out, lds);
}

template <typename MT, typename XT>
struct Load16;
template <>
struct Load16<float, float> {  // 4 matrix entries, 4 vector entries
  static constexpr int VEC = 4;
  __device__ static void mat(const float *p, float (&v)[4]) {
    f4 t = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(p));
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
  }
  __device__ static void vec(const float *p, float (&v)[4]) {
    f4 t = *reinterpret_cast<const f4 *>(p);
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
  }
};
template <>
struct Load16<float, double> {
  static constexpr int VEC = 4;
  __device__ static void mat(const float *p, float (&v)[4]) { Load16<float, float>::mat(p, v); }
  __device__ static void vec(const double *p, double (&v)[4]) {
    d2 a = reinterpret_cast<const d2 *>(p)[0], b = reinterpret_cast<const d2 *>(p)[1];
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
  }
};
template <>
struct Load16<double, double> {
  static constexpr int VEC = 2;
  __device__ static void mat(const double *p, double (&v)[2]) {
    d2 t = __builtin_nontemporal_load(reinterpret_cast<const d2 *>(p));
    v[0] = t.x; v[1] = t.y;
  }
  __device__ static void vec(const double *p, double (&v)[2]) {
    d2 t = *reinterpret_cast<const d2 *>(p);
    v[0] = t.x; v[1] = t.y;
  }
};

constexpr int kR = 8;  // rows per sweep of a workgroup

// out(i) = sum_j V[i][j] x[j] for rows [r0, r1), accumulated in AT; the
// epilogue is called by thread r for row g0 + r.
template <typename MT, typename XT, typename AT, typename Epi>
__device__ __forceinline__ void band_matvec(const MT *__restrict__ V, int64_t ld, const XT *__restrict__ x, int r0,
                                            int r1, AT *lds, Epi epi) {
  using L = Load16<MT, XT>;
  constexpr int VEC = L::VEC;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  for (int g0 = r0; g0 < r1; g0 += kR) {
    AT acc[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) acc[r] = AT(0);
    const int nr = min(kR, r1 - g0);
    const MT *row0 = V + (size_t)g0 * ld;
#pragma unroll 1
    for (int64_t c = (int64_t)t * VEC; c < ld; c += (int64_t)kWG * VEC) {
      XT xv[VEC];
      L::vec(x + c, xv);
#pragma unroll
      for (int r = 0; r < kR; ++r) {
        if (r < nr) {
          MT vv[VEC];
          L::mat(row0 + (size_t)r * ld + c, vv);
#pragma unroll
          for (int q = 0; q < VEC; ++q) acc[r] = __builtin_fma((AT)vv[q], (AT)xv[q], acc[r]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < kR; ++r) acc[r] = wave_sum(acc[r]);
    if (lane == 0)
#pragma unroll
      for (int r = 0; r < kR; ++r) lds[w * kR + r] = acc[r];
    __syncthreads();
    if (t < nr) {
      AT v = ((lds[t] + lds[kR + t]) + lds[2 * kR + t]) + lds[3 * kR + t];
      epi(g0 + t, v);
    }
    __syncthreads();
  }
}

// At most 128 VGPRs, so that four workgroups fit on every CU (kGMax = 1024
// co-resident workgroups on 256 CUs).
template <typename MT>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(4))) void k_solve(
    const SysDesc *__restrict__ descs, SolveParams P) {
  using VT = MT;
  constexpr bool MIXED = sizeof(MT) == 4;
  __shared__ double s_red[4 * 4];
  __shared__ double s_mvd[4 * kR];
  __shared__ VT s_mv[4 * kR];
  __shared__ int s_flag;

  // system of this workgroup: last descriptor with wg_begin <= blockIdx.x
  int lo = 0, hi = P.n_sys - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (descs[mid].wg_begin <= (int)blockIdx.x) lo = mid; else hi = mid - 1;
  }
  const SysDesc S = descs[lo];
  const int rank = (int)blockIdx.x - S.wg_begin;
  if (rank < 0 || rank >= S.wg_count) return;
  const int G = S.wg_count;
  const int N = (int)S.N;
  const int r0 = (int)((int64_t)N * rank / G), r1 = (int)((int64_t)N * (rank + 1) / G);
  size_t o_ctl, o_part, o_x, o_r, o_vec;
  int64_t ld;
  solve_offsets(S.N, MIXED ? BC_MIXED : BC_FP64, o_ctl, o_part, o_x, o_r, o_vec, ld);
  SolveCtl *ctl = reinterpret_cast<SolveCtl *>(S.ws + o_ctl);
  double *part = reinterpret_cast<double *>(S.ws + o_part);
  double *x64 = reinterpret_cast<double *>(S.ws + o_x);
  double *r64 = reinterpret_cast<double *>(S.ws + o_r);
  VT *vr = reinterpret_cast<VT *>(S.ws + o_vec);
  VT *vu = vr + ld, *vw = vu + ld, *vp = vw + ld, *vs = vp + ld, *vd = vs + ld, *idg = vd + ld;
  const MT *V = static_cast<const MT *>(S.V);
  const double *b = S.area;
  const int t = threadIdx.x;

  SysBarrier bar{ctl, G, __hip_atomic_load(&ctl->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                 P.spin_limit};

  int32_t phase, iters, outer, inner;
  uint32_t epoch;
  double bnorm, rnorm, scale, gamma, eta, alpha, beta;
  if (S.start) {
    phase = PH_INIT; iters = 0; outer = 0; inner = 0; epoch = 0;
    bnorm = rnorm = scale = gamma = eta = alpha = beta = 0.0;
  } else {
    phase = ctl->phase; iters = ctl->iters; outer = ctl->outer; inner = ctl->inner; epoch = ctl->epoch;
    bnorm = ctl->bnorm; rnorm = ctl->rnorm; scale = ctl->scale; gamma = ctl->gamma; eta = ctl->eta;
    alpha = ctl->alpha; beta = ctl->beta;
  }
  if (phase == PH_DONE) return;
  int32_t status = BC_OK;
  int budget = P.iter_budget > 0 ? P.iter_budget : INT_MAX;
  bool aborted = false;

  auto my_part = [&](int k) -> double * { return part + ((size_t)(epoch & 1u) * kGMax + rank) * 4 + k; };
  auto prev_set = [&]() -> const double * { return part + (size_t)((epoch - 1u) & 1u) * kGMax * 4; };
  // every partial set written in epoch e is read only in epoch e + 1
  auto sync = [&]() -> bool {
    bool ok = bar.sync(&s_flag);
    epoch += 1u;
    return ok;
  };

  while (true) {
    if (phase == PH_INIT) {
      for (int i = r0 + t; i < r1; i += kWG) {
        x64[i] = P.x0_given ? S.sigma[i] : 0.0;
        idg[i] = P.jacobi ? VT(1) / V[(size_t)i * ld + i] : VT(1);
      }
      if (rank == G - 1)
        for (int i = N + t; i < ld; i += kWG) {
          x64[i] = 0.0; r64[i] = 0.0;
          vr[i] = vu[i] = vw[i] = vp[i] = vs[i] = vd[i] = VT(0);
          idg[i] = VT(0);
        }
      if (!sync()) { aborted = true; break; }
      phase = PH_RESID;
      continue;
    }
    if (phase == PH_RESID) {
      if (budget <= 0) break;
      budget -= 2;
      // r = b - A x in FP64
      double pr = 0.0, pb = 0.0;
      band_matvec<MT, double, double>(V, ld, x64, r0, r1, s_mvd, [&](int i, double acc) {
        if (MIXED && S.pcorr != nullptr) {
          for (int e = S.prowptr[i]; e < S.prowptr[i + 1]; ++e) acc = __builtin_fma(S.pcorr[e], x64[S.pcol[e]], acc);
        }
        const double ri = b[i] - acc;
        r64[i] = ri;
        pr = __builtin_fma(ri, ri, pr);
        pb = __builtin_fma(b[i], b[i], pb);
      });
      {
        double v[2] = {pr, pb};
        wg_sum<2>(v, s_red);
        if (t == 0) { *my_part(0) = v[0]; *my_part(1) = v[1]; }
      }
      if (!sync()) { aborted = true; break; }
      {
        double tot[2];
        const int sl[2] = {0, 1};
        sum_partials<2>(prev_set(), G, sl, tot, s_red);
        if (outer == 0) bnorm = sqrt(tot[1]);
        rnorm = sqrt(tot[0]);
      }
      outer += 1;
      if (!(rnorm > P.rtol * bnorm)) { status = BC_OK; phase = PH_DONE; continue; }
      if (outer > P.max_outer || iters >= P.max_iter) { status = BC_ENOCONV; phase = PH_DONE; continue; }
      scale = 1.0 / rnorm;
      // inner start: r = r64 / ||r64||, u = M^-1 r, d = p = s = 0
      double pru = 0.0;
      for (int i = r0 + t; i < r1; i += kWG) {
        const VT ri = (VT)(r64[i] * scale);
        const VT ui = idg[i] * ri;
        vr[i] = ri; vu[i] = ui; vd[i] = VT(0); vp[i] = VT(0); vs[i] = VT(0);
        pru += (double)ri * (double)ui;
      }
      {
        double v[1] = {pru};
        wg_sum<1>(v, s_red);
        if (t == 0) *my_part(0) = v[0];
      }
      if (!sync()) { aborted = true; break; }
      {
        double tot[1];
        const int sl[1] = {0};
        sum_partials<1>(prev_set(), G, sl, tot, s_red);
        gamma = tot[0];
      }
      double pwu = 0.0;
      band_matvec<MT, VT, VT>(V, ld, vu, r0, r1, s_mv, [&](int i, VT acc) {
        vw[i] = acc;
        pwu += (double)acc * (double)vu[i];
      });
      {
        double v[1] = {pwu};
        wg_sum<1>(v, s_red);
        if (t == 0) *my_part(0) = v[0];
      }
      if (!sync()) { aborted = true; break; }
      {
        double tot[1];
        const int sl[1] = {0};
        sum_partials<1>(prev_set(), G, sl, tot, s_red);
        eta = tot[0];
      }
      iters += 1;
      inner = 0;
      if (!(eta > 0.0)) { status = BC_EBREAKDOWN; phase = PH_DONE; continue; }
      alpha = gamma / eta;
      beta = 0.0;
      phase = PH_CG;
      continue;
    }
    if (phase == PH_CG) {
      if (budget <= 0) break;
      budget -= 1;
      const VT a = (VT)alpha, bt = (VT)beta;
      double pru = 0.0, prr = 0.0;
      for (int i = r0 + t; i < r1; i += kWG) {
        const VT pi = vu[i] + bt * vp[i];
        const VT si = vw[i] + bt * vs[i];
        vp[i] = pi;
        vs[i] = si;
        vd[i] = vd[i] + a * pi;
        const VT ri = vr[i] - a * si;
        vr[i] = ri;
        const VT ui = idg[i] * ri;
        vu[i] = ui;
        pru += (double)ri * (double)ui;
        prr += (double)ri * (double)ri;
      }
      {
        double v[2] = {pru, prr};
        wg_sum<2>(v, s_red);
        if (t == 0) { *my_part(0) = v[0]; *my_part(1) = v[1]; }
      }
      if (!sync()) { aborted = true; break; }
      double gnew, rr;
      {
        double tot[2];
        const int sl[2] = {0, 1};
        sum_partials<2>(prev_set(), G, sl, tot, s_red);
        gnew = tot[0];
        rr = tot[1];
      }
      inner += 1;
      if (!(sqrt(rr) > P.inner_rtol) || iters >= P.max_iter) { phase = PH_UPDATE; continue; }
      double pwu = 0.0;
      band_matvec<MT, VT, VT>(V, ld, vu, r0, r1, s_mv, [&](int i, VT acc) {
        vw[i] = acc;
        pwu += (double)acc * (double)vu[i];
      });
      {
        double v[1] = {pwu};
        wg_sum<1>(v, s_red);
        if (t == 0) *my_part(0) = v[0];
      }
      if (!sync()) { aborted = true; break; }
      double delta;
      {
        double tot[1];
        const int sl[1] = {0};
        sum_partials<1>(prev_set(), G, sl, tot, s_red);
        delta = tot[0];
      }
      iters += 1;
      beta = gnew / gamma;
      eta = delta - beta * gnew / alpha;
      if (!(eta > 0.0)) { status = BC_EBREAKDOWN; phase = PH_DONE; continue; }
      alpha = gnew / eta;
      gamma = gnew;
      continue;
    }
    if (phase == PH_UPDATE) {
      for (int i = r0 + t; i < r1; i += kWG) x64[i] = __builtin_fma((double)vd[i], rnorm, x64[i]);
      if (!sync()) { aborted = true; break; }
      phase = PH_RESID;
      continue;
    }
    // PH_DONE: sigma = x, Cap = (1/4pi) sum x_i |T_i|
    double pc = 0.0;
    for (int i = r0 + t; i < r1; i += kWG) {
      S.sigma[i] = x64[i];
      pc = __builtin_fma(x64[i], b[i], pc);
    }
    {
      double v[1] = {pc};
      wg_sum<1>(v, s_red);
      if (t == 0) *my_part(0) = v[0];
    }
    if (!sync()) { aborted = true; break; }
    double cap;
    {
      double tot[1];
      const int sl[1] = {0};
      sum_partials<1>(prev_set(), G, sl, tot, s_red);
      cap = tot[0] * kInv4Pi;
    }
    if (rank == 0 && t == 0) {
      S.result->cap = cap;
      S.result->rel_residual = bnorm > 0.0 ? rnorm / bnorm : 0.0;
      S.result->iters = iters;
      S.result->outer = outer;
      S.result->status = status;
      S.result->precision = MIXED ? BC_MIXED : BC_FP64;
      ctl->phase = PH_DONE;
    }
    return;
  }
  if (rank == 0 && t == 0) {
    if (aborted) {
      S.result->iters = iters;
      S.result->outer = outer;
      S.result->status = BC_ETIMEOUT;
      S.result->precision = MIXED ? BC_MIXED : BC_FP64;
      ctl->phase = PH_DONE;
    } else {
      ctl->phase = phase; ctl->iters = iters; ctl->outer = outer; ctl->inner = inner; ctl->epoch = epoch;
      ctl->bnorm = bnorm; ctl->rnorm = rnorm; ctl->scale = scale; ctl->gamma = gamma; ctl->eta = eta;
      ctl->alpha = alpha; ctl->beta = beta;
      S.result->iters = iters;
      S.result->outer = outer;
      S.result->status = BC_RUNNING;
      S.result->precision = MIXED ? BC_MIXED : BC_FP64;
    }
  }
}

// Reset the control block of systems that (re)start.
__global__ void k_solve_init(const SysDesc *__restrict__ descs, int n_sys) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_sys) return;
  const SysDesc &S = descs[s];
  if (!S.start) return;
  size_t o_ctl, o_part, o_x, o_r, o_vec;
  int64_t ld;
  solve_offsets(S.N, BC_FP64, o_ctl, o_part, o_x, o_r, o_vec, ld);
  SolveCtl *ctl = reinterpret_cast<SolveCtl *>(S.ws + o_ctl);
  ctl->bar_count = 0u;
  ctl->bar_gen = 0u;
  ctl->abort = 0;
  ctl->phase = PH_INIT;
  ctl->epoch = 0u;
  S.result->status = BC_RUNNING;
}

struct DescBatch {
  SysDesc d[16];
  int n;
  int offset;
};

__global__ void k_set_desc(DescBatch batch, SysDesc *dst) {
  const int t = threadIdx.x;
  if (t < batch.n) dst[batch.offset + t] = batch.d[t];
}

int launch_set_desc(const SysDesc *h, int n, SysDesc *d, hipStream_t s) {
  for (int o = 0; o < n; o += 16) {
    DescBatch b{};
    b.n = n - o < 16 ? n - o : 16;
    b.offset = o;
    for (int k = 0; k < b.n; ++k) b.d[k] = h[o + k];
    hipLaunchKernelGGL(k_set_desc, dim3(1), dim3(64), 0, s, b, d);
    if (hipGetLastError() != hipSuccess) return BC_EDEVICE;
  }
  return BC_OK;
}

int solve_workgroups(int64_t N) {
  int64_t g = (N + 31) / 32;
  if (g < 1) g = 1;
  if (g > kGMax) g = kGMax;
  return (int)g;
}

int solve_capacity(int32_t precision) {
  int dev = 0, cus = 0, nb = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1;
  hipError_t e = precision == BC_FP64
                     ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_solve<double>, kWG, 0)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_solve<float>, kWG, 0);
  if (e != hipSuccess) return -1;
  return nb * cus;
}

int launch_solve(int32_t precision, const SysDesc *d_desc, int n_sys, int total_wg, const SolveParams &p,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_solve_init, dim3((n_sys + 63) / 64), dim3(64), 0, s, d_desc, n_sys);
  if (hipGetLastError() != hipSuccess) return BC_EDEVICE;
  SolveParams pp = p;
  void *args[] = {(void *)&d_desc, (void *)&pp};
  hipError_t e = precision == BC_FP64
                     ? hipLaunchCooperativeKernel((const void *)k_solve<double>, dim3(total_wg), dim3(kWG), args, 0, s)
                     : hipLaunchCooperativeKernel((const void *)k_solve<float>, dim3(total_wg), dim3(kWG), args, 0, s);
  return e == hipSuccess ? BC_OK : BC_EDEVICE;
}

// Fixed-order FP64 capacity reduction in one workgroup.
__global__ __launch_bounds__(kWG) void k_capacity(const double *__restrict__ sigma, const double *__restrict__ area,
                                                  int N, double *cap) {
  __shared__ double lds[4];
  double v[1] = {0.0};
  for (int i = threadIdx.x; i < N; i += kWG) v[0] = __builtin_fma(sigma[i], area[i], v[0]);
  wg_sum<1>(v, lds);
  if (threadIdx.x == 0) *cap = v[0] * kInv4Pi;
}

int launch_capacity(const double *sigma, const double *area, int64_t N, double *cap, hipStream_t s) {
  hipLaunchKernelGGL(k_capacity, dim3(1), dim3(kWG), 0, s, sigma, area, (int)N, cap);
  return hipGetLastError() == hipSuccess ? BC_OK : BC_EDEVICE;
}

}  // namespace bc
