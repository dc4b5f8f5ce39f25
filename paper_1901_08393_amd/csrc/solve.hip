// Persistent Krylov solver for V sigma = b, b = |T| (Section 2.5; CG applies
// because V is symmetric positive definite, Remark (ii)), and the capacity
// reduction Cap = (1/4pi) sum sigma_i |T_i| (eq. "cap:ell").
//
// One cooperative launch holds one or many systems; each system owns a fixed
// number of 1024-thread workgroups (a function of N only), each workgroup a
// contiguous band of rows and each wavefront a contiguous part of that band.
// Per system the workgroups run the same state machine:
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
// per entry, 2 flops): the 64 lanes of a wavefront sweep up to 8 of its rows
// at a time with 16-byte non-temporal loads; the vector comes from L2.
// Every reduction has a fixed order, so results are bitwise reproducible and
// do not depend on which other systems share the launch.
#include <climits>

#include "bc_internal.h"

namespace bc {

enum Phase : int32_t { PH_INIT = 0, PH_RESID = 1, PH_CG = 2, PH_UPDATE = 3, PH_DONE = 4 };

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

constexpr int kWaves = kSolveWG / 64;

// ------------------------------------------------------------ barrier
// Cross-workgroup barrier of one system fused with a fixed-order reduction.
// Every workgroup writes its partial sums and the barrier epoch into its own
// 64-byte slot (no contended atomics); workgroup 0 of the system gathers the
// slots in rank order, sums them and publishes the totals with the epoch in
// kNRep copies of a release record; each workgroup waits on one copy.  Only
// one thread per workgroup issues the agent-scope release and acquire fences
// (an L2 write-back and an L2 invalidate), after every wavefront has waited
// for its own stores, so a barrier costs one fence pair per workgroup.
// Spins are bounded: on time-out the system is marked aborted and every
// workgroup leaves its loop.
struct SysBar {
  gptr<BarSlot> slots;
  gptr<BarRel> rel;
  int G, rank;
  unsigned epoch;
  uint32_t spin_limit;
};

template <int K>
__device__ __noinline__ bool sys_sync(SysBar &B, const double (&v)[K], double (&tot)[K], double *lds, int *flag) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double s = wave_sum(v[k]);
    if (lane == 0) lds[w * 4 + k] = s;
  }
  __builtin_amdgcn_s_waitcnt(0);  // this wavefront's global stores have reached L2
  __syncthreads();
  B.epoch += 1u;
  const unsigned ep = B.epoch;
  if (B.G == 1) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
      for (int q = 0; q < kWaves; ++q) s += lds[q * 4 + k];
      tot[k] = s;
    }
    __syncthreads();
    return true;
  }
  if (t == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
      for (int q = 0; q < kWaves; ++q) s += lds[q * 4 + k];
      B.slots[B.rank].v[k] = s;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(&B.slots[B.rank].tag, ep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  int ok = 1;
  if (B.rank == 0) {
    double a[K];
#pragma unroll
    for (int k = 0; k < K; ++k) a[k] = 0.0;
    if (t < B.G) {
      uint32_t spins = 0;
      while (__hip_atomic_load(&B.slots[t].tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != ep) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > B.spin_limit) {
          ok = 0;
          break;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (t < B.G) {
#pragma unroll
      for (int k = 0; k < K; ++k) a[k] = B.slots[t].v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double s = wave_sum(a[k]);
      if (lane == 0) lds[w * 4 + k] = s;
    }
    const int bad = __syncthreads_or(!ok);
    if (t < kNRep) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int q = 0; q < kWaves; ++q) s += lds[q * 4 + k];
        B.rel[t].v[k] = s;
      }
      B.rel[t].abort = bad;
    }
    if (t < 64) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (t < kNRep) __hip_atomic_store(&B.rel[t].gen, ep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (t == 0) {
    gptr<BarRel> my = B.rel + (B.rank % kNRep);
    uint32_t spins = 0;
    while (__hip_atomic_load(&my->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != ep) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > B.spin_limit) {
        ok = 0;
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (ok && my->abort) ok = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) lds[64 + k] = my->v[k];
    *flag = ok;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) tot[k] = lds[64 + k];
  const int r = *flag;
  __syncthreads();
  return r != 0;
}

// ------------------------------------------------------- matrix product
template <typename MT, typename XT>
struct Load16;
template <>
struct Load16<float, float> {  // 4 matrix entries, 4 vector entries
  static constexpr int VEC = 4;
  __device__ static void mat(gptr<const float> p, float (&v)[4]) {
    f4 t = __builtin_nontemporal_load(reinterpret_cast<gptr<const f4>>(p));
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
  }
  __device__ static void vec(gptr<const float> p, float (&v)[4]) {
    f4 t = *reinterpret_cast<gptr<const f4>>(p);
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
  }
};
template <>
struct Load16<float, double> {
  static constexpr int VEC = 4;
  __device__ static void mat(gptr<const float> p, float (&v)[4]) { Load16<float, float>::mat(p, v); }
  __device__ static void vec(gptr<const double> p, double (&v)[4]) {
    d2 a = reinterpret_cast<gptr<const d2>>(p)[0], b = reinterpret_cast<gptr<const d2>>(p)[1];
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
  }
};
template <>
struct Load16<double, double> {
  static constexpr int VEC = 2;
  __device__ static void mat(gptr<const double> p, double (&v)[2]) {
    d2 t = __builtin_nontemporal_load(reinterpret_cast<gptr<const d2>>(p));
    v[0] = t.x; v[1] = t.y;
  }
  __device__ static void vec(gptr<const double> p, double (&v)[2]) {
    d2 t = *reinterpret_cast<gptr<const d2>>(p);
    v[0] = t.x; v[1] = t.y;
  }
};

// out(i) = sum_j V[i][j] x[j] for the R rows g0..g0+R-1: the 64 lanes of the
// wavefront sweep the columns with 16-byte loads, R independent rows per
// step (no branch inside the sweep, so all loads of a step are in flight
// together); lane 0 calls epi(row, sum) after a fixed-order reduction.
template <typename MT, typename XT, typename AT, int R, typename Epi>
__device__ __forceinline__ void sweep_rows(gptr<const MT> V, int64_t ld, gptr<const XT> x, int g0, Epi &epi) {
  using L = Load16<MT, XT>;
  constexpr int VEC = L::VEC;
  const int lane = threadIdx.x & 63;
  AT acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = AT(0);
  gptr<const MT> row0 = V + (size_t)g0 * ld;
#pragma unroll 2
  for (int64_t c = (int64_t)lane * VEC; c < ld; c += 64 * VEC) {
    XT xv[VEC];
    L::vec(x + c, xv);
    MT vv[R][VEC];
#pragma unroll
    for (int r = 0; r < R; ++r) L::mat(row0 + (size_t)r * ld + c, vv[r]);
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int q = 0; q < VEC; ++q) acc[r] = __builtin_fma((AT)vv[r][q], (AT)xv[q], acc[r]);
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const AT sum = wave_sum(acc[r]);
    if (lane == 0) epi(g0 + r, sum);
  }
}

// The rows [wr0, wr1) of this wavefront, at most 8 per sweep.
template <typename MT, typename XT, typename AT, typename Epi>
__device__ __forceinline__ void wave_matvec(gptr<const MT> V, int64_t ld, gptr<const XT> x, int wr0, int wr1,
                                            Epi epi) {
  int g0 = wr0;
  while (g0 < wr1) {
    const int n = min(8, wr1 - g0);
    switch (n) {
      case 8: sweep_rows<MT, XT, AT, 8>(V, ld, x, g0, epi); break;
      case 7: sweep_rows<MT, XT, AT, 7>(V, ld, x, g0, epi); break;
      case 6: sweep_rows<MT, XT, AT, 6>(V, ld, x, g0, epi); break;
      case 5: sweep_rows<MT, XT, AT, 5>(V, ld, x, g0, epi); break;
      case 4: sweep_rows<MT, XT, AT, 4>(V, ld, x, g0, epi); break;
      case 3: sweep_rows<MT, XT, AT, 3>(V, ld, x, g0, epi); break;
      case 2: sweep_rows<MT, XT, AT, 2>(V, ld, x, g0, epi); break;
      default: sweep_rows<MT, XT, AT, 1>(V, ld, x, g0, epi); break;
    }
    g0 += n;
  }
}

// At most 128 VGPRs, so that one 1024-thread workgroup fits on every CU.
template <typename MT>
__global__ __launch_bounds__(kSolveWG) __attribute__((amdgpu_waves_per_eu(4))) void k_solve(
    const SysDesc *__restrict__ descs, SolveParams P) {
  using VT = MT;
  constexpr bool MIXED = sizeof(MT) == 4;
  __shared__ double s_red[80];
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
  const int t = threadIdx.x, w = t >> 6;
  const int r0 = (int)((int64_t)N * rank / G), r1 = (int)((int64_t)N * (rank + 1) / G);
  const int nb = r1 - r0;
  const int wr0 = r0 + nb * w / kWaves, wr1 = r0 + nb * (w + 1) / kWaves;  // this wavefront's rows
  size_t o_ctl, o_slots, o_rel, o_x, o_r, o_vec, o_total;
  int64_t ld;
  solve_offsets(S.N, MIXED ? BC_MIXED : BC_FP64, o_ctl, o_slots, o_rel, o_x, o_r, o_vec, o_total, ld);
  gptr<char> ws = as_global(S.ws);
  gptr<SolveCtl> ctl = reinterpret_cast<gptr<SolveCtl>>(ws + o_ctl);
  gptr<double> x64 = reinterpret_cast<gptr<double>>(ws + o_x);
  gptr<double> r64 = reinterpret_cast<gptr<double>>(ws + o_r);
  gptr<VT> vr = reinterpret_cast<gptr<VT>>(ws + o_vec);
  gptr<VT> vu = vr + ld, vw = vu + ld, vp = vw + ld, vs = vp + ld, vd = vs + ld, idg = vd + ld;
  gptr<const MT> V = as_global(static_cast<const MT *>(S.V));
  gptr<const double> b = as_global(S.area);
  gptr<double> sigma = as_global(S.sigma);
  gptr<bc_result> result = as_global(S.result);
  gptr<const double> pcorr = as_global(S.pcorr);
  gptr<const int32_t> prowptr = as_global(S.prowptr), pcol = as_global(S.pcol);

  SysBar bar{reinterpret_cast<gptr<BarSlot>>(ws + o_slots), reinterpret_cast<gptr<BarRel>>(ws + o_rel), G, rank, 0u,
             P.spin_limit};

  int32_t phase, iters, outer, inner;
  double bnorm, rnorm, scale, gamma, eta, alpha, beta, itol;
  if (S.start) {
    phase = PH_INIT; iters = 0; outer = 0; inner = 0;
    bnorm = rnorm = scale = gamma = eta = alpha = beta = itol = 0.0;
  } else {
    phase = ctl->phase; iters = ctl->iters; outer = ctl->outer; inner = ctl->inner; bar.epoch = ctl->epoch;
    bnorm = ctl->bnorm; rnorm = ctl->rnorm; scale = ctl->scale; gamma = ctl->gamma; eta = ctl->eta;
    alpha = ctl->alpha; beta = ctl->beta; itol = ctl->itol;
  }
  if (phase == PH_DONE) return;
  int32_t status = BC_OK;
  int budget = S.budget > 0 ? S.budget : (P.iter_budget > 0 ? P.iter_budget : INT_MAX);
  bool aborted = false;
  const double none[1] = {0.0};

  while (true) {
    if (phase == PH_INIT) {
      for (int i = r0 + t; i < r1; i += kSolveWG) {
        x64[i] = P.x0_given ? sigma[i] : 0.0;
        idg[i] = P.jacobi ? VT(1) / V[(size_t)i * ld + i] : VT(1);
      }
      if (rank == G - 1)
        for (int i = N + t; i < ld; i += kSolveWG) {
          x64[i] = 0.0; r64[i] = 0.0;
          vr[i] = vu[i] = vw[i] = vp[i] = vs[i] = vd[i] = VT(0);
          idg[i] = VT(0);
        }
      double dummy[1];
      if (!sys_sync<1>(bar, none, dummy, s_red, &s_flag)) { aborted = true; break; }
      phase = PH_RESID;
      continue;
    }
    if (phase == PH_RESID) {
      if (budget <= 0) break;
      budget -= 2;
      // r = b - A x in FP64
      double pr = 0.0, pb = 0.0;
      wave_matvec<MT, double, double>(V, ld, x64, wr0, wr1, [&](int i, double acc) {
        if (MIXED && S.pcorr != nullptr) {
          for (int e = prowptr[i]; e < prowptr[i + 1]; ++e) acc = __builtin_fma(pcorr[e], x64[pcol[e]], acc);
        }
        const double ri = b[i] - acc;
        r64[i] = ri;
        pr = __builtin_fma(ri, ri, pr);
        pb = __builtin_fma(b[i], b[i], pb);
      });
      {
        const double v[2] = {pr, pb};
        double tot[2];
        if (!sys_sync<2>(bar, v, tot, s_red, &s_flag)) { aborted = true; break; }
        if (outer == 0) bnorm = sqrt(tot[1]);
        rnorm = sqrt(tot[0]);
      }
      outer += 1;
      if (!(rnorm > P.rtol * bnorm)) { status = BC_OK; phase = PH_DONE; continue; }
      if (outer > P.max_outer || iters >= P.max_iter) { status = BC_ENOCONV; phase = PH_DONE; continue; }
      scale = 1.0 / rnorm;
      // the inner solve need not go further than the outer tolerance asks
      itol = fmax(P.inner_rtol, 0.3 * P.rtol * bnorm / rnorm);
      // inner start: r = r64 / ||r64||, u = M^-1 r, d = p = s = 0
      double pru = 0.0;
      for (int i = r0 + t; i < r1; i += kSolveWG) {
        const VT ri = (VT)(r64[i] * scale);
        const VT ui = idg[i] * ri;
        vr[i] = ri; vu[i] = ui; vd[i] = VT(0); vp[i] = VT(0); vs[i] = VT(0);
        pru += (double)ri * (double)ui;
      }
      {
        const double v[1] = {pru};
        double tot[1];
        if (!sys_sync<1>(bar, v, tot, s_red, &s_flag)) { aborted = true; break; }
        gamma = tot[0];
      }
      double pwu = 0.0;
      wave_matvec<MT, VT, VT>(V, ld, vu, wr0, wr1, [&](int i, VT acc) {
        vw[i] = acc;
        pwu += (double)acc * (double)vu[i];
      });
      {
        const double v[1] = {pwu};
        double tot[1];
        if (!sys_sync<1>(bar, v, tot, s_red, &s_flag)) { aborted = true; break; }
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
      for (int i = r0 + t; i < r1; i += kSolveWG) {
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
      double gnew, rr;
      {
        const double v[2] = {pru, prr};
        double tot[2];
        if (!sys_sync<2>(bar, v, tot, s_red, &s_flag)) { aborted = true; break; }
        gnew = tot[0];
        rr = tot[1];
      }
      inner += 1;
      if (!(sqrt(rr) > itol) || iters >= P.max_iter) { phase = PH_UPDATE; continue; }
      double pwu = 0.0;
      wave_matvec<MT, VT, VT>(V, ld, vu, wr0, wr1, [&](int i, VT acc) {
        vw[i] = acc;
        pwu += (double)acc * (double)vu[i];
      });
      double delta;
      {
        const double v[1] = {pwu};
        double tot[1];
        if (!sys_sync<1>(bar, v, tot, s_red, &s_flag)) { aborted = true; break; }
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
      for (int i = r0 + t; i < r1; i += kSolveWG) x64[i] = __builtin_fma((double)vd[i], rnorm, x64[i]);
      double dummy[1];
      if (!sys_sync<1>(bar, none, dummy, s_red, &s_flag)) { aborted = true; break; }
      phase = PH_RESID;
      continue;
    }
    // PH_DONE: sigma = x, Cap = (1/4pi) sum x_i |T_i|
    double pc = 0.0;
    for (int i = r0 + t; i < r1; i += kSolveWG) {
      sigma[i] = x64[i];
      pc = __builtin_fma(x64[i], b[i], pc);
    }
    double cap;
    {
      const double v[1] = {pc};
      double tot[1];
      if (!sys_sync<1>(bar, v, tot, s_red, &s_flag)) { aborted = true; break; }
      cap = tot[0] * kInv4Pi;
    }
    if (rank == 0 && t == 0) {
      result->cap = cap;
      result->rel_residual = bnorm > 0.0 ? rnorm / bnorm : 0.0;
      result->iters = iters;
      result->outer = outer;
      result->status = status;
      result->precision = MIXED ? BC_MIXED : BC_FP64;
      ctl->phase = PH_DONE;
    }
    return;
  }
  if (rank == 0 && t == 0) {
    if (aborted) {
      result->iters = iters;
      result->outer = outer;
      result->status = BC_ETIMEOUT;
      result->precision = MIXED ? BC_MIXED : BC_FP64;
      ctl->phase = PH_DONE;
    } else {
      ctl->phase = phase; ctl->iters = iters; ctl->outer = outer; ctl->inner = inner; ctl->epoch = bar.epoch;
      ctl->bnorm = bnorm; ctl->rnorm = rnorm; ctl->scale = scale; ctl->gamma = gamma; ctl->eta = eta;
      ctl->alpha = alpha; ctl->beta = beta; ctl->itol = itol;
      result->iters = iters;
      result->outer = outer;
      result->status = BC_RUNNING;
      result->precision = MIXED ? BC_MIXED : BC_FP64;
    }
  }
}

// Reset the control block, barrier slots and release records of systems
// that (re)start: one workgroup per system.
__global__ __launch_bounds__(256) void k_solve_init(const SysDesc *__restrict__ descs, int n_sys) {
  const int s = blockIdx.x;
  if (s >= n_sys) return;
  const SysDesc &S = descs[s];
  if (!S.start) return;
  size_t o_ctl, o_slots, o_rel, o_x, o_r, o_vec, o_total;
  int64_t ld;
  solve_offsets(S.N, BC_FP64, o_ctl, o_slots, o_rel, o_x, o_r, o_vec, o_total, ld);
  const int t = threadIdx.x;
  BarSlot *slots = reinterpret_cast<BarSlot *>(S.ws + o_slots);
  BarRel *rel = reinterpret_cast<BarRel *>(S.ws + o_rel);
  if (t < kGMax) slots[t].tag = 0u;
  if (t < kNRep) {
    rel[t].gen = 0u;
    rel[t].abort = 0;
  }
  if (t == 0) {
    SolveCtl *ctl = reinterpret_cast<SolveCtl *>(S.ws + o_ctl);
    ctl->phase = PH_INIT;
    ctl->epoch = 0u;
    S.result->status = BC_RUNNING;
  }
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

// About 80 rows (5 per wavefront) per workgroup, at most kGMax workgroups.
int solve_workgroups(int64_t N) {
  int64_t g = (N + 79) / 80;
  if (g < 1) g = 1;
  if (g > kGMax) g = kGMax;
  return (int)g;
}

int solve_capacity(int32_t precision) {
  int dev = 0, cus = 0, nb = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1;
  hipError_t e = precision == BC_FP64
                     ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_solve<double>, kSolveWG, 0)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_solve<float>, kSolveWG, 0);
  if (e != hipSuccess) return -1;
  return nb * cus;
}

int launch_solve(int32_t precision, const SysDesc *d_desc, int n_sys, int total_wg, const SolveParams &p,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_solve_init, dim3(n_sys), dim3(256), 0, s, d_desc, n_sys);
  if (hipGetLastError() != hipSuccess) return BC_EDEVICE;
  SolveParams pp = p;
  void *args[] = {(void *)&d_desc, (void *)&pp};
  hipError_t e = precision == BC_FP64
                     ? hipLaunchCooperativeKernel((const void *)k_solve<double>, dim3(total_wg), dim3(kSolveWG), args,
                                                  0, s)
                     : hipLaunchCooperativeKernel((const void *)k_solve<float>, dim3(total_wg), dim3(kSolveWG), args,
                                                  0, s);
  return e == hipSuccess ? BC_OK : BC_EDEVICE;
}

// Fixed-order FP64 capacity reduction in one workgroup.
__global__ __launch_bounds__(kWG) void k_capacity(const double *__restrict__ sigma, const double *__restrict__ area,
                                                  int N, double *cap) {
  __shared__ double lds[4];
  double v = 0.0;
  for (int i = threadIdx.x; i < N; i += kWG) v = __builtin_fma(sigma[i], area[i], v);
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) *cap = (((lds[0] + lds[1]) + lds[2]) + lds[3]) * kInv4Pi;
}

int launch_capacity(const double *sigma, const double *area, int64_t N, double *cap, hipStream_t s) {
  hipLaunchKernelGGL(k_capacity, dim3(1), dim3(kWG), 0, s, sigma, area, (int)N, cap);
  return hipGetLastError() == hipSuccess ? BC_OK : BC_EDEVICE;
}

}  // namespace bc
