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
//          ||r|| <= rtol ||b||, or, with a capacity tolerance, once the
//          capacity's algebraic error is estimated below it.  The capacity
//          is reported as (1/4pi) J(x), J(x) = 2 b^T x - x^T A x =
//          b^T x + x^T r, which for symmetric positive definite A
//          falls short of J(x*) = b^T x* by exactly ||x* - x||_A^2 (the
//          algebraic form of Section 2.7's Proposition: the capacity error is
//          the squared energy error).  The estimate of that error comes from
//          the last inner CG (QUAD in cg_loop); ||x|| ||r|| <= cap_rtol
//          |b^T x|, which bounds 4pi (Cap* - b^T x / 4pi) = x*^T r to first
//          order, also stops.  Else start an inner CG on A d = r / ||r||.
//   CG     preconditioned CG in the Chronopoulos-Gear arrangement: the two
//          inner products of an iteration are reduced together, so an
//          iteration costs one product with V and two cross-workgroup
//          barriers.  Vectors and the matrix product are in the matrix
//          precision (FP32 products accumulate in FP32); the scalar
//          reductions are summed in FP64.
//   UPDATE x += ||r|| d in FP64, back to RESID.
//   DONE   sigma = x, Cap, result.
//
// The product streams the diagonal blocks of V and the blocks above them once
// from HBM (bandwidth-bound: 4 or 8 bytes per entry read, 4 flops) and uses
// each off-diagonal block for both of its triangles (strip_product,
// strip_gather).  At the first step without an initial guess x = 0 and r = b
// needs no product.  Every reduction has a fixed order, so results are
// bitwise reproducible and do not depend on which other systems share the
// launch.
#include <climits>

#include "bc_internal.h"

namespace bc {

enum Phase : int32_t { PH_INIT = 0, PH_RESID = 1, PH_CG = 2, PH_UPDATE = 3, PH_DONE = 4 };

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f2 __attribute__((ext_vector_type(2)));

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
__device__ __forceinline__ bool sys_sync_body(SysBar &B, const double (&v)[K], double (&tot)[K], lptr<double> lds,
                                              lptr<int> flag) {
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

// The barrier as a call of its own, for the phases of the state machine
// other than the CG iteration (which inlines it).
template <int K>
__device__ __noinline__ bool sys_sync(SysBar &B, const double (&v)[K], double (&tot)[K], lptr<double> lds,
                                      lptr<int> flag) {
  return sys_sync_body<K>(B, v, tot, lds, flag);
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

// one FP64 column per lane: the product with several vectors, whose row and
// column sums take the registers that wider loads would need
struct LoadD1 {
  static constexpr int VEC = 1;
  __device__ static void mat(gptr<const double> p, double (&v)[1]) { v[0] = __builtin_nontemporal_load(p); }
  __device__ static void vec(gptr<const double> p, double (&v)[1]) { v[0] = *p; }
};

// one FP32 column per lane with FP64 vectors
struct LoadF1D {
  static constexpr int VEC = 1;
  __device__ static void mat(gptr<const float> p, float (&v)[1]) { v[0] = __builtin_nontemporal_load(p); }
  __device__ static void vec(gptr<const double> p, double (&v)[1]) { v[0] = *p; }
};

// ------------------------------------------------ symmetric half product
// Y = V X for several vectors (the dual mesh's products; one vector takes the
// strip product below), reading V only on its diagonal blocks and above
// them.  A unit
// (block B, chunk c) covers the rows [kRB B, kRB B + kRB) and CW = 64 VEC
// columns; wavefront w of the workgroup owns 8 of the block's rows and lane l
// VEC consecutive columns of the chunk.  For its rows a unit adds
// V[i][j] x[j] to the row sums (kept in registers across the chunks of a
// segment: the units of one block that one workgroup holds), and for the
// columns right of the diagonal block it forms the column sums
// sum_i V[i][j] x[i], which stand for the lower triangle by symmetry.  The
// sixteen wavefronts' column sums are added in LDS in wavefront order and
// stored per row block (cpart); the row sums are stored per segment (rpart).
// half_gather then forms y_i = (row sums of i's segments) + (column sums of
// the row blocks above i), each in a fixed order, so the result depends on
// N and the workgroup count only.  With DELTA the kernel also returns this
// workgroup's share of x^T V x, summed from the same column sums (weight 1 on
// the diagonal block, 2 right of it), so that an inner product of the CG
// iteration needs no pass over y.
struct HalfPlan {
  int64_t ld, m64, T;
  int N, nB, k, G;
  int64_t u0, u1;  // this workgroup's units
};

template <typename MT, typename XT, typename AT, bool DELTA, bool LDS2, int NR = 1, typename L = Load16<MT, XT>>
__device__ __forceinline__ void half_product(gptr<const MT> V, gptr<const XT> x, const HalfPlan &H, gptr<AT> rpart,
                                             gptr<AT> cpart, lptr<AT> lbuf, double &delta) {
  constexpr int VEC = L::VEC;
  constexpr int CW = 64 * VEC;
  int64_t u = H.u0;
  if (u >= H.u1) return;
  // lane from mbcnt and the wavefront index as a scalar: both can be
  // recomputed where needed instead of being kept in registers
  const int lane = (int)__lane_id();
  const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int N = H.N;
  const int ld = (int)H.ld;
  // with NR right-hand sides, vector m and its partial sums sit at these
  // strides from the first ones
  const size_t xs = (size_t)H.ld, rs = (size_t)kRB * (size_t)H.T, cps = (size_t)H.nB * (size_t)H.ld;
  // block of the first unit
  int B;
  {
    int lo = 0, hi = H.nB - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (half_units_before(mid, H.m64, H.k) <= u) lo = mid; else hi = mid - 1;
    }
    B = lo;
  }
  int64_t SE = half_units_before(B + 1, H.m64, H.k);  // first unit of the next block
  int c = (int)(u - half_units_before(B, H.m64, H.k));
  int64_t useg = u;  // first unit of the current segment (its row sums are stored there)

  // x values of the wavefront's 8 rows (the same for all its lanes): in
  // registers for one vector; for several in LDS behind the column-sum
  // buffers, loaded by lanes 0 .. 8 NR - 1 of the wavefront at each block
  // start and read back as broadcasts by the same wavefront (the LDS
  // operations of a wavefront complete in order)
  constexpr bool XR_LDS = NR > 1;
  static_assert(XR_LDS || NR == 1, "several vectors keep their row values in LDS");
  static_assert(XR_LDS || kRB <= 64 * VEC, "chunk 0 must hold the block's row values");
  AT xr[8], acc[NR][8];
  lptr<AT> xl = lbuf + (LDS2 ? 2 : 1) * NR * 16 * CW + w * NR * 8;
  auto load_xr_lds = [&](int Bl) {
    if (lane < 8 * NR) {
      const int row = kRB * Bl + 8 * w + (lane & 7);
      xl[lane] = row < N ? (AT)x[(lane >> 3) * xs + row] : AT(0);
    }
  };
  auto get_xr = [&](int m, int r) -> AT { return XR_LDS ? xl[m * 8 + r] : xr[r]; };
  if (XR_LDS) load_xr_lds(B);
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int row = kRB * B + 8 * w + r;
    xr[r] = (!XR_LDS && c > 0 && row < N) ? (AT)x[row] : AT(0);  // chunk 0 brings them itself
  }
#pragma unroll
  for (int m = 0; m < NR; ++m)
#pragma unroll
    for (int r = 0; r < 8; ++r) acc[m][r] = AT(0);
  MT va[8][VEC];
  XT xa[NR][VEC];
  // loads of unit (Bl, cl): the wavefront's 8 rows of block Bl (their bases
  // are the same for the whole wavefront) and the lane's VEC columns
  auto load = [&](int Bl, int cl) {
    const int c0 = kRB * Bl + CW * cl + lane * VEC;
    const int cc = c0 < ld ? c0 : ld - VEC;  // lanes past the end read the last columns, weighted 0
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int row = min(kRB * Bl + 8 * w + r, N - 1);
      L::mat(V + (size_t)row * (size_t)ld + cc, va[r]);
    }
#pragma unroll
    for (int m = 0; m < NR; ++m) L::vec(x + m * xs + cc, xa[m]);
  };
  load(B, c);
  // Units are swept as one stream: the loads of the next unit (of this block
  // or the next) are issued as soon as this unit's registers are free, so
  // they are in flight across the workgroup barrier and across block ends.
  while (true) {
    const int col = kRB * B + CW * c + lane * VEC;
    const bool act = col < ld;
    if (!XR_LDS && c == 0) {
      // chunk 0 starts at column kRB B: lane l holds x[kRB B + VEC l + q],
      // among them the x values of this wavefront's rows
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const XT v = lane_f(xa[0][r % VEC], (8 * w + r) / VEC);  // the source lane is the same for the wavefront
        xr[r] = kRB * B + 8 * w + r < N ? (AT)v : AT(0);
      }
    }
    AT xq[NR][VEC], cs[NR][VEC];
#pragma unroll
    for (int m = 0; m < NR; ++m)
#pragma unroll
      for (int q = 0; q < VEC; ++q) {
        xq[m][q] = act ? (AT)xa[m][q] : AT(0);
        cs[m][q] = AT(0);
      }
#pragma unroll
    for (int m = 0; m < NR; ++m)
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
          acc[m][r] = fma_t((AT)va[r][q], xq[m][q], acc[m][r]);
          cs[m][q] = fma_t((AT)va[r][q], get_xr(m, r), cs[m][q]);
        }
    const int diag_end = kRB * B + kRB;
    if (DELTA) {
      double d = 0.0;
#pragma unroll
      for (int q = 0; q < VEC; ++q) d = __builtin_fma((double)xq[0][q], (double)cs[0][q], d);
      delta = __builtin_fma(col < diag_end ? 1.0 : 2.0, d, delta);
    }
    lptr<AT> lb = lbuf + (LDS2 ? (int)(u & 1) * (NR * 16 * CW) : 0);
#pragma unroll
    for (int m = 0; m < NR; ++m)
#pragma unroll
      for (int q = 0; q < VEC; ++q) lb[(m * 16 + w) * CW + lane * VEC + q] = cs[m][q];
    const bool more = u + 1 < H.u1;
    const bool same = u + 1 < SE;
    if (more) load(same ? B : B + 1, same ? c + 1 : 0);
    __syncthreads();
    // the NR CW column sums of the unit: with one vector shared out evenly
    // over the sixteen wavefronts (a few lanes each), so that no wavefront
    // lags behind the others at the next barrier; with three, by the first
    // NR CW threads (measured faster there)
    constexpr int kPer = NR * CW / 16;
    if (NR == 1 ? lane < kPer : 64 * w + lane < NR * CW) {
      const int item = NR == 1 ? w * kPer + lane : 64 * w + lane;
      const int m = NR == 1 ? 0 : item / CW, t = item - m * CW;
      const int ct = kRB * B + CW * c + t;
      if (ct >= diag_end && ct < ld) {
        AT sum = AT(0);
#pragma unroll
        for (int q = 0; q < 16; ++q) sum += lb[(m * 16 + q) * CW + t];
        cpart[m * cps + (size_t)B * (size_t)ld + ct] = sum;
      }
    }
    // with two buffers the next unit writes the other one; the barrier of
    // that unit orders these reads before the writes of the unit after
    if (!LDS2) __syncthreads();
    if (!more || !same) {
      // end of a segment: the row sums of this block's units
#pragma unroll
      for (int m = 0; m < NR; ++m)
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const AT sum = wave_sum_full(acc[m][r]);
          if (lane == r && kRB * B + 8 * w + r < N) rpart[m * rs + (size_t)useg * kRB + 8 * w + r] = sum;
          acc[m][r] = AT(0);
        }
      useg = u + 1;
    }
    if (!more) break;
    ++u;
    if (same) {
      ++c;
    } else {
      ++B;
      c = 0;
      SE = half_units_before(B + 1, H.m64, H.k);
      if (XR_LDS) load_xr_lds(B);
    }
  }
  if (LDS2) __syncthreads();  // the last column sums are read before lbuf is reused
}

// y_i for the rows [r0, r1) of this workgroup into band[i - r0]: the row
// sums of the segments of i's block (one per workgroup that holds units of
// it, in workgroup order) and then the column sums of the row blocks
// 0 .. B(i)-1.  The band is cut into groups of 64 rows (a lane per row);
// the sixteen wavefronts are shared out over up to sixteen groups at a time,
// S per group, and the S wavefronts of a group take every S-th term.  A
// wavefront issues the loads of sixteen of its terms before adding any, so
// that a band's column sums arrive in one or two memory round trips; it
// keeps one partial sum per load slot and adds them in a fixed tree, and the
// S wavefront sums of a row are added in wavefront order.  The order depends
// on N and the workgroup count only.
template <typename AT>
__device__ __forceinline__ void half_gather_body(const HalfPlan &H, int r0, int r1, gptr<const AT> rpart,
                                                 gptr<const AT> cpart, lptr<AT> lpart, lptr<AT> band) {
  constexpr int NB = 16;  // loads in flight per wavefront
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int ngr = (r1 - r0 + 63) >> 6;  // groups of 64 rows
  const int gpp = ngr < 16 ? ngr : 16;  // groups per pass
  const int S = 16 / (gpp > 0 ? gpp : 1);  // wavefronts per group
  for (int p0 = 0; p0 < ngr; p0 += gpp) {
    const int g = p0 + w / S, sl = w % S;
    const int i = r0 + 64 * g + lane;
    AT s[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) s[k] = AT(0);
    if (w < S * gpp && g < ngr && i < r1) {
      const int B = i / kRB;
      const int64_t SB = half_units_before(B, H.m64, H.k), SE = half_units_before(B + 1, H.m64, H.k);
      // workgroups holding the units SB and SE - 1 (ranges [T g / G, T (g+1) / G))
      const int glo = (int)(((SB + 1) * H.G + H.T - 1) / H.T) - 1;
      const int ghi = (int)((SE * H.G + H.T - 1) / H.T) - 1;
      const int nseg = ghi - glo + 1;
      const int nterm = nseg + B;
      const int ii = i - kRB * B;
      int q = sl;
      for (; q < nseg && q < nterm; q += S) {  // segment row sums (few)
        int64_t us = SB;
        bool ok = true;
        if (q > 0) {
          const int gq = glo + q;
          us = H.T * gq / H.G;
          ok = H.T * (gq + 1) / H.G != us;  // a workgroup without units has no segment
        }
        if (ok) s[0] += rpart[(size_t)us * kRB + ii];
      }
      // column sums of the blocks above, NB loads issued before any add
      for (; q < nterm; q += NB * S) {
        AT v[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          const int qk = q + k * S;
          v[k] = qk < nterm ? cpart[(size_t)(qk - nseg) * (size_t)H.ld + i] : AT(0);
        }
#pragma unroll
        for (int k = 0; k < NB; ++k) s[k] += v[k];
      }
    }
#pragma unroll
    for (int h = NB / 2; h > 0; h >>= 1)
#pragma unroll
      for (int k = 0; k < h; ++k) s[k] += s[k + h];
    lpart[w * 64 + lane] = s[0];
    __syncthreads();
    if (w < gpp) {
      const int gg = p0 + w, iw = r0 + 64 * gg + lane;
      if (gg < ngr && iw < r1) {
        AT tot = AT(0);
        for (int q = 0; q < S; ++q) tot += lpart[(w * S + q) * 64 + lane];
        band[iw - r0] = tot;
      }
    }
    __syncthreads();
  }
}

template <typename AT>
__device__ __noinline__ void half_gather(const HalfPlan &H, int r0, int r1, gptr<const AT> rpart,
                                         gptr<const AT> cpart, lptr<AT> lpart, lptr<AT> band) {
  half_gather_body<AT>(H, r0, r1, rpart, cpart, lpart, band);
}

// ------------------------------------------------- symmetric strip product
// y = V x for one vector, reading V only on its diagonal blocks and above
// them, in strips of 256 bytes of each row (SW = 64 FP32 or 32 FP64 columns;
// strips_before).  The wavefronts of a system ("holders", 16 per workgroup)
// take equal contiguous ranges of the strips, so each strip belongs to one
// wavefront and its column sums are complete inside it: no workgroup
// barrier and no LDS exchange per strip, and the wavefronts of a workgroup
// run apart.  A 256-byte row piece keeps the HBM pages open as well as the
// 1 KiB rows of the unit sweep did; 128-byte pieces lost a fifth of the rate.
//
// A wavefront reads a strip in four batches of 32 rows; in batch h lane l
// holds VEC = 16 / sizeof(MT) entries (16 bytes) of the rows
// l/16 + 32 h + 4 k (k = 0..7), at columns VEC (l % 16) .. +VEC, so that one
// load instruction covers 4 rows x 256 contiguous bytes.
//  * Row sums: per batch a lane's 8 row partials are reduced over the 16
//    lanes of its row group (row16_scatter8), which leaves lane l the row
//    l/16 + 32 h + 4 ((l >> 1) & 7); the lane adds it to acc[h] across the
//    strips of one block (a segment) and the segment's 128 sums are stored at
//    slot (holder + block) of rpart (strip_slots).
//  * Column sums: a lane's VEC column partials over its 32 rows of the strip
//    are reduced over the four lanes of its column group (col4_scatter) and
//    stored per row block (cpart), for the columns right of the diagonal
//    block (the diagonal block's own columns are covered by its rows).
//  * The x values of the block's rows sit in the wavefront's 128 LDS entries
//    (row r at (r % 4) 32 + r / 4, so a lane reads its batch's 8 as a run).
// With DELTA the product also returns this wavefront's share of x^T V x
// (from the column partials: weight 1 on the diagonal block, 2 right of it).
// Every sum has a fixed order: the result depends on N and the workgroup
// count only.
struct StripPlan {
  int64_t ld, T;  // row stride; strips of the sweep
  int N, nB, GH;  // rows; row blocks; holders (wavefronts of the system)
  int g0;         // holder of this workgroup's first wavefront
  int sw;         // strip width in columns
};

__device__ __forceinline__ StripPlan strip_plan(int64_t N, int64_t ld, int sw, int G, int rank) {
  StripPlan P;
  P.ld = ld;
  P.N = (int)N;
  P.nB = (int)((N + kRB - 1) / kRB);
  P.T = strips_before(P.nB, ld, sw);
  P.GH = 16 * G;
  P.g0 = 16 * rank;
  P.sw = sw;
  return P;
}

// Reduce-scatter of 8 values over 16 lanes (a group of l/16): lane l keeps
// the sum over its group of value 4 b3 + 2 b2 + b1 (b: the bits of l),
// exchanging with the lanes l^8, l^7 and l^3 and finally adding lane l^1's
// copy.  The exchanges are lane permutes through the LDS crossbar
// (ds_bpermute); the same exchanges as DPP row operations gave wrong sums in
// some builds of the solver kernel and were dropped.
template <typename AT>
__device__ __forceinline__ AT row16_scatter8(const AT (&v)[8], int lane) {
  const bool b3 = lane & 8, b2 = lane & 4, b1 = lane & 2;
  AT a[4], b[2];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const AT keep = b3 ? v[j + 4] : v[j], give = b3 ? v[j] : v[j + 4];
    a[j] = keep + __shfl_xor(give, 8, 64);
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const AT keep = b2 ? a[j + 2] : a[j], give = b2 ? a[j] : a[j + 2];
    b[j] = keep + __shfl_xor(give, 7, 64);
  }
  const AT keep = b1 ? b[1] : b[0], give = b1 ? b[0] : b[1];
  const AT c = keep + __shfl_xor(give, 3, 64);
  return c + __shfl_xor(c, 1, 64);
}

// Column sums over the four lanes l, l^16, l^32, l^48 of a column group:
// lane l keeps column 2 b4 + b5 of its group's four (VEC = 4), or column b4
// of two (VEC = 2, where lanes l and l^32 both hold it).
template <typename AT, int VEC>
__device__ __forceinline__ AT col4_scatter(const AT (&cs)[VEC], int lane) {
  const bool b4 = lane & 16, b5 = lane & 32;
  if constexpr (VEC == 4) {
    AT a[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const AT keep = b4 ? cs[j + 2] : cs[j], give = b4 ? cs[j] : cs[j + 2];
      a[j] = keep + __shfl_xor(give, 16, 64);
    }
    const AT keep = b5 ? a[1] : a[0], give = b5 ? a[0] : a[1];
    return keep + __shfl_xor(give, 32, 64);
  } else {
    static_assert(VEC == 2, "four or two columns per lane");
    const AT keep = b4 ? cs[1] : cs[0], give = b4 ? cs[0] : cs[1];
    const AT c = keep + __shfl_xor(give, 16, 64);
    return c + __shfl_xor(c, 32, 64);
  }
}

template <typename MT, typename XT, typename AT, bool DELTA>
__device__ __forceinline__ void strip_product(gptr<const MT> V, gptr<const XT> x, const StripPlan &H,
                                              gptr<AT> rpart, gptr<AT> cpart, lptr<AT> lxall, double &delta) {
  using L = Load16<MT, XT>;
  constexpr int VEC = L::VEC;
  constexpr int SW = 16 * VEC;
  constexpr int NDIAG = kRB / SW;  // strips of the diagonal block
  static_assert(SW * (int)sizeof(MT) == kStripBytes, "a strip is 256 bytes of a row");
  const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int hold = H.g0 + w;
  int64_t u = H.T * hold / H.GH;
  const int64_t u1 = H.T * (hold + 1) / H.GH;
  if (u >= u1) return;
  const int lane = (int)__lane_id();
  const int rq = lane >> 4, cq = lane & 15;
  const int N = H.N;
  const int64_t ld = H.ld;
  lptr<AT> lx = lxall + w * kRB;
  // block of the first strip
  int B;
  {
    int lo = 0, hi = H.nB - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (strips_before(mid, ld, SW) <= u) lo = mid; else hi = mid - 1;
    }
    B = lo;
  }
  int64_t SE = strips_before(B + 1, ld, SW);
  int c = (int)(u - strips_before(B, ld, SW));

  // the block's x values: lane l brings rows l and l + 64, stored at the
  // start of the block's first strip
  AT xn0, xn1;
  auto x_rows = [&](int Bl) {
    const int i0 = kRB * Bl + lane, i1 = i0 + 64;
    xn0 = i0 < N ? (AT)x[i0] : AT(0);
    xn1 = i1 < N ? (AT)x[i1] : AT(0);
  };
  bool fresh = true;
  x_rows(B);
  MT va[8][VEC];
  XT xa[VEC];
  auto load = [&](int Bl, int cl, int h, bool with_x) {
    const int64_t col = (int64_t)kRB * Bl + (int64_t)SW * cl + VEC * cq;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int row = min(kRB * Bl + rq + 32 * h + 4 * k, N - 1);
      L::mat(V + (size_t)row * (size_t)ld + col, va[k]);
    }
    if (with_x) L::vec(x + col, xa);
  };
  // acc[0] always takes the current batch: the four are rotated after each
  // batch, so that the batch loop needs no register indexing
  AT acc[4], cs[VEC];
#pragma unroll
  for (int h = 0; h < 4; ++h) acc[h] = AT(0);
#pragma unroll
  for (int q = 0; q < VEC; ++q) cs[q] = AT(0);
  int h = 0;
  load(B, c, 0, true);
  while (true) {
    if (h == 0 && fresh) {
      lx[(lane & 3) * 32 + (lane >> 2)] = xn0;       // row lane
      lx[(lane & 3) * 32 + 16 + (lane >> 2)] = xn1;  // row lane + 64
      fresh = false;
    }
    AT xq[VEC], xb[8], rp[8];
#pragma unroll
    for (int q = 0; q < VEC; ++q) xq[q] = (AT)xa[q];
#pragma unroll
    for (int k = 0; k < 8; ++k) xb[k] = lx[rq * 32 + 8 * h + k];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      AT r = (AT)va[k][0] * xq[0];
#pragma unroll
      for (int q = 1; q < VEC; ++q) r = fma_t((AT)va[k][q], xq[q], r);
      rp[k] = r;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
      for (int q = 0; q < VEC; ++q) cs[q] = fma_t((AT)va[k][q], xb[k], cs[q]);
    // the next loads go out before the lane exchanges of the row sums
    auto rows_done = [&]() {
      const AT a0 = acc[0] + row16_scatter8<AT>(rp, lane);
      acc[0] = acc[1]; acc[1] = acc[2]; acc[2] = acc[3]; acc[3] = a0;
    };
    if (h < 3) {
      ++h;
      load(B, c, h, false);
      rows_done();
      continue;
    }
    // end of the strip
    const bool more = u + 1 < u1, same = u + 1 < SE;
    const int Bn = same ? B : B + 1, cn = same ? c + 1 : 0;
    if (DELTA) {
      double d = 0.0;
#pragma unroll
      for (int q = 0; q < VEC; ++q) d = __builtin_fma((double)xq[q], (double)cs[q], d);
      delta = __builtin_fma(c < NDIAG ? 1.0 : 2.0, d, delta);
    }
    if (more) {
      load(Bn, cn, 0, true);
      if (!same) {
        x_rows(Bn);
        fresh = true;
      }
    }
    rows_done();
    // the strip's column sums (right of the diagonal block)
    {
      const AT sum = col4_scatter<AT, VEC>(cs, lane);
      const int q = VEC == 4 ? 2 * ((lane >> 4) & 1) + ((lane >> 5) & 1) : (lane >> 4) & 1;
      if (c >= NDIAG && (VEC == 4 || lane < 32))
        cpart[(size_t)B * (size_t)ld + (size_t)(kRB * B + SW * c + VEC * cq + q)] = sum;
#pragma unroll
      for (int j = 0; j < VEC; ++j) cs[j] = AT(0);
    }
    if (!more || !same) {
      // end of a segment: its row sums at slot (holder + block); after the
      // four rotations acc[h] holds batch h
      const int rk = 4 * ((lane >> 1) & 7) + rq;
#pragma unroll
      for (int hh = 0; hh < 4; ++hh) {
        const int row = 32 * hh + rk;
        if (!(lane & 1) && kRB * B + row < N) rpart[(size_t)(hold + B) * kRB + row] = acc[hh];
        acc[hh] = AT(0);
      }
    }
    if (!more) break;
    ++u;
    h = 0;
    B = Bn;
    c = cn;
    if (!same) SE = strips_before(B + 1, ld, SW);
  }
}

// y_i for the rows [r0, r1) of this workgroup into band[i - r0] after a
// strip product: the row sums of the segments of i's block (one per
// wavefront that holds strips of it, in wavefront order) and then the
// column sums of the row blocks 0 .. B(i)-1.  The band is cut into groups of
// 64 rows (a lane per row); the sixteen wavefronts are shared out over up to
// sixteen groups at a time, S per group, and the S wavefronts of a group take
// every S-th term.  A wavefront issues the loads of sixteen of its terms
// before adding any, keeps one partial sum per load slot and adds them in a
// fixed tree, and the S wavefront sums of a row are added in wavefront order.
template <typename AT>
__device__ __forceinline__ void strip_gather_body(const StripPlan &H, int r0, int r1, gptr<const AT> rpart,
                                                  gptr<const AT> cpart, lptr<AT> lpart, lptr<AT> band) {
  constexpr int NB = 16;  // loads in flight per wavefront
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int ngr = (r1 - r0 + 63) >> 6;  // groups of 64 rows
  const int gpp = ngr < 16 ? ngr : 16;  // groups per pass
  const int S = 16 / (gpp > 0 ? gpp : 1);  // wavefronts per group
  const int64_t T = H.T, GH = H.GH;
  for (int p0 = 0; p0 < ngr; p0 += gpp) {
    const int g = p0 + w / S, sl = w % S;
    const int i = r0 + 64 * g + lane;
    AT s[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) s[k] = AT(0);
    if (w < S * gpp && g < ngr && i < r1) {
      const int B = i / kRB;
      const int64_t SB = strips_before(B, H.ld, H.sw), SE = strips_before(B + 1, H.ld, H.sw);
      // holders of the strips SB and SE - 1 (ranges [T g / GH, T (g+1) / GH))
      const int glo = (int)(((SB + 1) * GH + T - 1) / T) - 1;
      const int ghi = (int)((SE * GH + T - 1) / T) - 1;
      const int nseg = ghi - glo + 1;
      const int nterm = nseg + B;
      const int ii = i - kRB * B;
      int q = sl;
      for (; q < nseg && q < nterm; q += S) {  // segment row sums
        const int64_t gq = glo + q;
        if (T * (gq + 1) / GH != T * gq / GH)  // a holder without strips has no segment
          s[0] += rpart[(size_t)(gq + B) * kRB + ii];
      }
      // column sums of the blocks above, NB loads issued before any add
      for (; q < nterm; q += NB * S) {
        AT v[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          const int qk = q + k * S;
          v[k] = qk < nterm ? cpart[(size_t)(qk - nseg) * (size_t)H.ld + i] : AT(0);
        }
#pragma unroll
        for (int k = 0; k < NB; ++k) s[k] += v[k];
      }
    }
#pragma unroll
    for (int h = NB / 2; h > 0; h >>= 1)
#pragma unroll
      for (int k = 0; k < h; ++k) s[k] += s[k + h];
    lpart[w * 64 + lane] = s[0];
    __syncthreads();
    if (w < gpp) {
      const int gg = p0 + w, iw = r0 + 64 * gg + lane;
      if (gg < ngr && iw < r1) {
        AT tot = AT(0);
        for (int q = 0; q < S; ++q) tot += lpart[(w * S + q) * 64 + lane];
        band[iw - r0] = tot;
      }
    }
    __syncthreads();
  }
}

template <typename AT>
__device__ __noinline__ void strip_gather(const StripPlan &H, int r0, int r1, gptr<const AT> rpart,
                                          gptr<const AT> cpart, lptr<AT> lpart, lptr<AT> band) {
  strip_gather_body<AT>(H, r0, r1, rpart, cpart, lpart, band);
}

// The solver's products as a call of their own.  Inlined into k_solve, the
// product loop shares the kernel's 128 registers with the state of the
// whole state machine and spills inside the loop; as a call it has the
// registers to itself and the caller's state is saved once per product.
// Arguments of a call arrive in vector registers, so the plan and the
// pointers, the same in every lane, are first read back as such.
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ gptr<T> uniform_ptr(gptr<T> p) {
  return (gptr<T>)uniform64((int64_t)(uintptr_t)p);
}

__device__ __forceinline__ double uniform_f64(double v) {
  return __builtin_bit_cast(double, uniform64(__builtin_bit_cast(int64_t, v)));
}
__device__ __forceinline__ int uniform32(int v) { return __builtin_amdgcn_readfirstlane(v); }
template <typename T>
__device__ __forceinline__ lptr<T> uniform_lptr(lptr<T> p) {
  return (lptr<T>)(uintptr_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(uintptr_t)p);
}
template <typename SP>
__device__ __forceinline__ StripPlan uniform_strip(const SP &H) {
  StripPlan U;
  U.ld = uniform64(H.ld);
  U.T = uniform64(H.T);
  U.N = uniform32(H.N);
  U.nB = uniform32(H.nB);
  U.GH = uniform32(H.GH);
  U.g0 = uniform32(H.g0);
  U.sw = uniform32(H.sw);
  return U;
}

// Its operands are read from an LDS record written by the caller, as the CG
// phase reads its own (with them passed as call arguments the FP64 solver
// gave wrong products in some builds).
struct ProdArgs {
  gptr<const void> V, x;
  gptr<void> rp, cp;
  StripPlan H;
};
template <typename MT, typename XT, typename AT, bool DELTA>
__device__ __noinline__ double solver_product(lptr<ProdArgs> P, lptr<AT> lx) {
  P = uniform_lptr(P);
  double delta = 0.0;
  strip_product<MT, XT, AT, DELTA>(uniform_ptr((gptr<const MT>)P->V), uniform_ptr((gptr<const XT>)P->x),
                                   uniform_strip(P->H), uniform_ptr((gptr<AT>)P->rp), uniform_ptr((gptr<AT>)P->cp),
                                   uniform_lptr(lx), delta);
  return delta;
}

// ---------------------------------------------------------- CG iterations
// The CG phase of one system as a call of its own that runs iterations until
// the inner tolerance, the iteration cap, the launch's budget, a breakdown
// or an abort ends it.  Its product, gather and barriers are inlined, and
// its state (pointers and scalars, the same in every lane) is read from LDS
// at entry and written back at exit, so that nothing of the state machine
// stays live across the iterations' inner calls; inlined into k_solve the
// iteration spilled registers and saved them around every call, and the
// barriers' fences sent that scratch traffic to HBM.
template <typename MT>
struct CGCtx {
  gptr<const MT> V;
  gptr<MT> vr, vu, vp, vs, vd, idg, rp, cp;
  gptr<BarSlot> slots;
  gptr<BarRel> rel;
  StripPlan H;
  int r0, r1, G, rank;
  uint32_t spin_limit;
  int32_t max_iter;
};
struct CGState {
  double alpha, beta, gamma, eta, itol;
  // capacity stop (QUAD): the last four terms alpha_j gamma_j, the sum of
  // all of them, their scale rnorm^2, J at the inner start, 0.3 cap_rtol, and
  // the error estimate at exit (< 0: none yet)
  double hs[4], hs_sum, hs_scale, jres, hs_tol, est;
  int32_t hs_n;
  int32_t iters, inner, budget;
  uint32_t epoch;
  int32_t exit;  // 0 budget used up, 1 inner solve done, 2 breakdown, 3 aborted
};

// QUAD: the capacity stop.  The inner problem A d = r_hat (||r_hat|| = 1)
// starts from d = 0, and CG's step j lowers the squared energy norm of its
// error by exactly alpha_j gamma_j (gamma_j = r_j^T M^-1 r_j), so the error
// of the iterate four steps back is the sum of the last four terms plus the
// current iterate's error: the sum is a lower bound on the former and above
// the latter once the error halves over four steps (Hestenes and Stiefel;
// the estimate stays reliable in finite precision).  Scaled by rnorm^2 it is the algebraic error of the capacity
// functional J(x) = 2 b^T x - x^T A x at x + rnorm d, whose value is J at the
// inner start plus rnorm^2 times the sum of all terms.  The inner solve stops
// once the estimate is at most 0.3 cap_rtol J.
template <typename MT, bool QUAD>
__device__ __noinline__ void cg_loop(lptr<CGCtx<MT>> Cp, lptr<CGState> Sp, lptr<MT> lbuf, lptr<MT> lpart,
                                     lptr<MT> band, lptr<double> lred, lptr<int> lflag) {
  using VT = MT;
  Cp = uniform_lptr(Cp);
  Sp = uniform_lptr(Sp);
  lbuf = uniform_lptr(lbuf);
  lpart = uniform_lptr(lpart);
  band = uniform_lptr(band);
  lred = uniform_lptr(lred);
  lflag = uniform_lptr(lflag);
  const gptr<const MT> V = uniform_ptr(Cp->V);
  const gptr<VT> vr = uniform_ptr(Cp->vr), vu = uniform_ptr(Cp->vu), vp = uniform_ptr(Cp->vp);
  const gptr<VT> vs = uniform_ptr(Cp->vs), vd = uniform_ptr(Cp->vd), idg = uniform_ptr(Cp->idg);
  const gptr<VT> rp = uniform_ptr(Cp->rp), cp = uniform_ptr(Cp->cp);
  const StripPlan H = uniform_strip(Cp->H);
  const int r0 = uniform32(Cp->r0), r1 = uniform32(Cp->r1), max_iter = uniform32(Cp->max_iter);
  SysBar bar{uniform_ptr(Cp->slots), uniform_ptr(Cp->rel), uniform32(Cp->G), uniform32(Cp->rank),
             (unsigned)uniform32((int)Sp->epoch), (uint32_t)uniform32((int)Cp->spin_limit)};
  double alpha = uniform_f64(Sp->alpha), beta = uniform_f64(Sp->beta), gamma = uniform_f64(Sp->gamma);
  double eta = uniform_f64(Sp->eta);
  const double itol = uniform_f64(Sp->itol);
  double h0 = 0.0, h1 = 0.0, h2 = 0.0, h3 = 0.0, hs_sum = 0.0, hs_scale = 0.0, jres = 0.0, hs_tol = 0.0;
  int hs_n = 0;
  if (QUAD) {
    h0 = uniform_f64(Sp->hs[0]); h1 = uniform_f64(Sp->hs[1]); h2 = uniform_f64(Sp->hs[2]); h3 = uniform_f64(Sp->hs[3]);
    hs_sum = uniform_f64(Sp->hs_sum); hs_scale = uniform_f64(Sp->hs_scale); jres = uniform_f64(Sp->jres);
    hs_tol = uniform_f64(Sp->hs_tol); hs_n = uniform32(Sp->hs_n);
  }
  int iters = uniform32(Sp->iters), inner = uniform32(Sp->inner), budget = uniform32(Sp->budget);
  const int t = threadIdx.x;
  int ex = 0;
  while (true) {
    if (budget <= 0) { ex = 0; break; }
    budget -= 1;
    // w = V u of the last product
    strip_gather_body<VT>(H, r0, r1, rp, cp, lpart, band);
    const VT a = (VT)alpha, bt = (VT)beta;
    double pru = 0.0, prr = 0.0;
    // the lane's first row, formed anew in every iteration: kept across the
    // product instead, the vectors' addresses would be spilled
    int i0 = r0 + t;
    asm volatile("" : "+v"(i0));
    for (int i = i0; i < r1; i += kSolveWG) {
      const VT pi = vu[i] + bt * vp[i];
      const VT si = band[i - r0] + bt * vs[i];
      vp[i] = pi;
      vs[i] = si;
      const VT di = vd[i] + a * pi;
      vd[i] = di;
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
      if (!sys_sync_body<2>(bar, v, tot, lred, lflag)) { ex = 3; break; }
      gnew = tot[0];
      rr = tot[1];
    }
    inner += 1;
    bool cap_met = false;
    if (QUAD) {
      // the step just taken (with alpha, gamma) lowered the error by alpha gamma
      const double term = alpha * gamma;
      h0 = h1; h1 = h2; h2 = h3; h3 = term;
      hs_n += 1;
      hs_sum += term;
      if (hs_n >= 4) cap_met = hs_scale * (((h0 + h1) + h2) + h3) <= hs_tol * (jres + hs_scale * hs_sum);
    }
    if (!(sqrt(rr) > itol) || cap_met || iters >= max_iter) { ex = 1; break; }
    double pwu = 0.0;
    strip_product<MT, VT, VT, true>(V, vu, H, rp, cp, lbuf, pwu);
    double delta;
    {
      const double v[1] = {pwu};
      double tot[1];
      if (!sys_sync_body<1>(bar, v, tot, lred, lflag)) { ex = 3; break; }
      delta = tot[0];
    }
    iters += 1;
    beta = gnew / gamma;
    eta = delta - beta * gnew / alpha;
    if (!(eta > 0.0)) { ex = 2; break; }
    alpha = gnew / eta;
    gamma = gnew;
  }
  __syncthreads();  // every lane has read the state before it is rewritten
  if (t == 0) {
    Sp->alpha = alpha; Sp->beta = beta; Sp->gamma = gamma; Sp->eta = eta;
    Sp->iters = iters; Sp->inner = inner; Sp->budget = budget; Sp->epoch = bar.epoch; Sp->exit = ex;
    if (QUAD) {
      Sp->hs[0] = h0; Sp->hs[1] = h1; Sp->hs[2] = h2; Sp->hs[3] = h3;
      Sp->hs_sum = hs_sum; Sp->hs_n = hs_n;
      Sp->est = hs_n >= 4 ? hs_scale * (((h0 + h1) + h2) + h3) : -1.0;
    }
  }
  __syncthreads();
}

// At most 128 VGPRs, so that one 1024-thread workgroup fits on every CU.
template <typename MT>
__global__ __launch_bounds__(kSolveWG) __attribute__((amdgpu_waves_per_eu(4))) void k_solve(
    const SysDesc *__restrict__ descs, SolveParams P) {
  using VT = MT;
  constexpr bool MIXED = sizeof(MT) == 4;
  __shared__ double s_red[80];
  __shared__ int s_flag;
  __shared__ double s_buf[16 * kRB];   // x of the product's row blocks, per wavefront (16 KB)
  __shared__ double s_part[16 * 64];   // per-wavefront sums of half_gather
  __shared__ double s_band[kMaxBand];  // V x on this workgroup's rows
  __shared__ CGCtx<MT> s_cg;
  __shared__ CGState s_st;
  __shared__ ProdArgs s_prod;
  const lptr<double> l_red = (lptr<double>)s_red;
  const lptr<int> l_flag = (lptr<int>)&s_flag;

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
  const int t = threadIdx.x;
  const int r0 = (int)((int64_t)N * rank / G), r1 = (int)((int64_t)N * (rank + 1) / G);
  const SolveLayout Lay(S.N, MIXED ? BC_MIXED : BC_FP64);
  const int64_t ld = Lay.ld;
  const StripPlan H = strip_plan(N, ld, Lay.sw, G, rank);
  gptr<char> ws = as_global(S.ws);
  gptr<SolveCtl> ctl = reinterpret_cast<gptr<SolveCtl>>(ws + Lay.ctl);
  gptr<double> x64 = reinterpret_cast<gptr<double>>(ws + Lay.x64);
  gptr<double> r64 = reinterpret_cast<gptr<double>>(ws + Lay.r64);
  gptr<VT> vr = reinterpret_cast<gptr<VT>>(ws + Lay.vec);
  gptr<VT> vu = vr + ld, vw = vu + ld, vp = vw + ld, vs = vp + ld, vd = vs + ld, idg = vd + ld;
  gptr<double> rpD = reinterpret_cast<gptr<double>>(ws + Lay.rpart);
  gptr<double> cpD = reinterpret_cast<gptr<double>>(ws + Lay.cpart);
  gptr<VT> rpV = reinterpret_cast<gptr<VT>>(ws + Lay.rpart);
  gptr<VT> cpV = reinterpret_cast<gptr<VT>>(ws + Lay.cpart);
  gptr<const MT> V = as_global(static_cast<const MT *>(S.V));
  gptr<const double> b = as_global(S.area);
  gptr<double> sigma = as_global(S.sigma);
  gptr<bc_result> result = as_global(S.result);
  gptr<const double> pcorr = as_global(S.pcorr);
  gptr<const int32_t> prowptr = as_global(S.prowptr), pcol = as_global(S.pcol);

  SysBar bar{reinterpret_cast<gptr<BarSlot>>(ws + Lay.slots), reinterpret_cast<gptr<BarRel>>(ws + Lay.rel), G, rank, 0u,
             P.spin_limit};

  int32_t phase, iters, outer, inner, hs_n;
  double bnorm, rnorm, scale, gamma, eta, alpha, beta, itol;
  double hs[4], hs_sum, jres, est;  // the capacity stop's state (QUAD in cg_loop)
  if (S.start) {
    phase = PH_INIT; iters = 0; outer = 0; inner = 0; hs_n = 0;
    bnorm = rnorm = scale = gamma = eta = alpha = beta = itol = 0.0;
    hs[0] = hs[1] = hs[2] = hs[3] = hs_sum = jres = 0.0;
    est = -1.0;
  } else {
    phase = ctl->phase; iters = ctl->iters; outer = ctl->outer; inner = ctl->inner; bar.epoch = ctl->epoch;
    bnorm = ctl->bnorm; rnorm = ctl->rnorm; scale = ctl->scale; gamma = ctl->gamma; eta = ctl->eta;
    alpha = ctl->alpha; beta = ctl->beta; itol = ctl->itol;
    hs_n = ctl->hs_n;
    for (int q = 0; q < 4; ++q) hs[q] = ctl->hs[q];
    hs_sum = ctl->hs_sum; jres = ctl->jres; est = ctl->est;
  }
  if (phase == PH_DONE) return;
  int32_t status = BC_OK;
  int budget = S.budget > 0 ? S.budget : (P.iter_budget > 0 ? P.iter_budget : INT_MAX);
  bool aborted = false;
  const double none[1] = {0.0};
  if (t == 0) {
    s_cg.V = V;
    s_cg.vr = vr; s_cg.vu = vu; s_cg.vp = vp; s_cg.vs = vs; s_cg.vd = vd; s_cg.idg = idg;
    s_cg.rp = rpV; s_cg.cp = cpV;
    s_cg.slots = bar.slots; s_cg.rel = bar.rel;
    s_cg.H = H;
    s_cg.r0 = r0; s_cg.r1 = r1; s_cg.G = G; s_cg.rank = rank;
    s_cg.spin_limit = P.spin_limit;
    s_cg.max_iter = P.max_iter;
  }
  __syncthreads();

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
      if (!sys_sync<1>(bar, none, dummy, l_red, l_flag)) { aborted = true; break; }
      phase = PH_RESID;
      continue;
    }
    if (phase == PH_RESID) {
      if (budget <= 0) break;
      budget -= 2;
      // r = b - A x in FP64 (x = 0 at the first step without an initial guess)
      const bool zero_x = outer == 0 && !P.x0_given;
      if (!zero_x) {
        double dummy[1];
        if (t == 0) {
          s_prod.V = (gptr<const void>)V; s_prod.x = (gptr<const void>)x64;
          s_prod.rp = (gptr<void>)rpD; s_prod.cp = (gptr<void>)cpD; s_prod.H = H;
        }
        __syncthreads();
        (void)solver_product<MT, double, double, false>((lptr<ProdArgs>)&s_prod, (lptr<double>)s_buf);
        if (!sys_sync<1>(bar, none, dummy, l_red, l_flag)) { aborted = true; break; }
        strip_gather<double>(H, r0, r1, rpD, cpD, (lptr<double>)s_part, (lptr<double>)s_band);
        if (MIXED && S.pcorr != nullptr) {
          // the FP64 near-field correction of the mixed matrix: one wavefront
          // per row, its lanes over the row's pattern entries (gathers in
          // parallel), summed in a fixed order and added to the product
          const int lane = t & 63;
          for (int i = r0 + (t >> 6); i < r1; i += kSolveWG / 64) {
            const int e0 = prowptr[i], e1 = prowptr[i + 1];
            double c = 0.0;
            for (int e = e0 + lane; e < e1; e += 64) c = __builtin_fma(pcorr[e], x64[pcol[e]], c);
            c = wave_sum(c);
            if (lane == 0) s_band[i - r0] += c;
          }
          __syncthreads();
        }
      }
      // sums: ||r||^2, then ||b||^2 at the first step and x^T r after it,
      // ||x||^2, b^T x
      const bool first = outer == 0;
      double pr = 0.0, pb = 0.0, pxx = 0.0, pbx = 0.0;
      for (int i = r0 + t; i < r1; i += kSolveWG) {
        const double acc = zero_x ? 0.0 : s_band[i - r0];
        const double ri = b[i] - acc, xi = x64[i];
        r64[i] = ri;
        pr = __builtin_fma(ri, ri, pr);
        pb = first ? __builtin_fma(b[i], b[i], pb) : __builtin_fma(xi, ri, pb);
        pxx = __builtin_fma(xi, xi, pxx);
        pbx = __builtin_fma(b[i], xi, pbx);
      }
      // the residual norm to reach: rtol ||b||, or with a capacity tolerance
      // the norm at which ||x|| ||r|| / |b^T x|, the first-order bound on
      // Cap's relative error (4pi (Cap* - Cap) = x*^T r), is cap_rtol
      // and the capacity functional J(x) = 2 b^T x - x^T A x = b^T x + x^T r
      // (at the first step x = 0, or a caller's guess, for which b^T x
      // serves as the scale of the capacity stop)
      double target, jcur;
      {
        const double v[4] = {pr, pb, pxx, pbx};
        double tot[4];
        if (!sys_sync<4>(bar, v, tot, l_red, l_flag)) { aborted = true; break; }
        if (first) bnorm = sqrt(tot[1]);
        rnorm = sqrt(tot[0]);
        jcur = tot[3] + (first ? 0.0 : tot[1]);
        target = P.rtol * bnorm;
        if (P.cap_rtol > 0.0 && tot[2] > 0.0) target = fmax(target, P.cap_rtol * fabs(tot[3]) / sqrt(tot[2]));
      }
      outer += 1;
      // the capacity stop: the last inner solve's estimate of J's algebraic error
      const bool quad_met = P.cap_rtol > 0.0 && est >= 0.0 && est <= P.cap_rtol * fabs(jcur);
      if (!(rnorm > target) || quad_met) { status = BC_OK; phase = PH_DONE; continue; }
      if (outer > P.max_outer || iters >= P.max_iter) { status = BC_ENOCONV; phase = PH_DONE; continue; }
      scale = 1.0 / rnorm;
      // the inner solve need not go further than the outer target asks; with
      // a capacity tolerance its own estimate usually stops it first, and the
      // residual floor is a tenth of inner_rtol, so that a run is not cut
      // short (and another FP64 residual step taken) just before the estimate
      // would have stopped it
      itol = fmax(P.cap_rtol > 0.0 ? 0.1 * P.inner_rtol : P.inner_rtol, 0.3 * target / rnorm);
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
        if (!sys_sync<1>(bar, v, tot, l_red, l_flag)) { aborted = true; break; }
        gamma = tot[0];
      }
      double pwu = 0.0;
      if (t == 0) {
        s_prod.V = (gptr<const void>)V; s_prod.x = (gptr<const void>)vu;
        s_prod.rp = (gptr<void>)rpV; s_prod.cp = (gptr<void>)cpV; s_prod.H = H;
      }
      __syncthreads();
      pwu = solver_product<MT, VT, VT, true>((lptr<ProdArgs>)&s_prod, (lptr<VT>)s_buf);
      {
        const double v[1] = {pwu};
        double tot[1];
        if (!sys_sync<1>(bar, v, tot, l_red, l_flag)) { aborted = true; break; }
        eta = tot[0];
      }
      iters += 1;
      inner = 0;
      if (!(eta > 0.0)) { status = BC_EBREAKDOWN; phase = PH_DONE; continue; }
      alpha = gamma / eta;
      beta = 0.0;
      // a new inner solve: its terms alpha_j gamma_j start afresh
      hs[0] = hs[1] = hs[2] = hs[3] = hs_sum = 0.0;
      hs_n = 0;
      jres = jcur;
      est = -1.0;
      phase = PH_CG;
      continue;
    }
    if (phase == PH_CG) {
      // with a capacity tolerance every inner solve also stops on its estimate
      // of the capacity's algebraic error (everything here is kept in the
      // control block, so a resumed launch decides the same)
      const bool quad = P.cap_rtol > 0.0;
      if (t == 0) {
        s_st.alpha = alpha; s_st.beta = beta; s_st.gamma = gamma; s_st.eta = eta; s_st.itol = itol;
        for (int q = 0; q < 4; ++q) s_st.hs[q] = hs[q];
        s_st.hs_sum = hs_sum; s_st.hs_n = hs_n; s_st.hs_scale = rnorm * rnorm; s_st.jres = jres;
        s_st.hs_tol = 0.3 * P.cap_rtol; s_st.est = est;
        s_st.iters = iters; s_st.inner = inner; s_st.budget = budget; s_st.epoch = bar.epoch;
      }
      __syncthreads();
      if (quad)
        cg_loop<MT, true>((lptr<CGCtx<MT>>)&s_cg, (lptr<CGState>)&s_st, (lptr<VT>)s_buf, (lptr<VT>)s_part,
                          (lptr<VT>)s_band, l_red, l_flag);
      else
        cg_loop<MT, false>((lptr<CGCtx<MT>>)&s_cg, (lptr<CGState>)&s_st, (lptr<VT>)s_buf, (lptr<VT>)s_part,
                           (lptr<VT>)s_band, l_red, l_flag);
      alpha = uniform_f64(s_st.alpha); beta = uniform_f64(s_st.beta); gamma = uniform_f64(s_st.gamma);
      eta = uniform_f64(s_st.eta);
      iters = uniform32(s_st.iters); inner = uniform32(s_st.inner); budget = uniform32(s_st.budget);
      bar.epoch = (unsigned)uniform32((int)s_st.epoch);
      if (quad) {
        for (int q = 0; q < 4; ++q) hs[q] = uniform_f64(s_st.hs[q]);
        hs_sum = uniform_f64(s_st.hs_sum); hs_n = uniform32(s_st.hs_n); est = uniform_f64(s_st.est);
      }
      const int ex = uniform32(s_st.exit);
      __syncthreads();  // the state is read before a later phase writes it again
      if (ex == 0) break;  // this launch's budget is used up; the next one resumes here
      if (ex == 3) { aborted = true; break; }
      if (ex == 2) { status = BC_EBREAKDOWN; est = -1.0; phase = PH_DONE; continue; }
      phase = PH_UPDATE;
      continue;
    }
    if (phase == PH_UPDATE) {
      for (int i = r0 + t; i < r1; i += kSolveWG) x64[i] = __builtin_fma((double)vd[i], rnorm, x64[i]);
      double dummy[1];
      if (!sys_sync<1>(bar, none, dummy, l_red, l_flag)) { aborted = true; break; }
      phase = PH_RESID;
      continue;
    }
    // PH_DONE: sigma = x, Cap = (1/4pi) J(x) with J(x) = b^T x + x^T r
    // (r = b - A x, the residual of the last step, which is x's), which equals
    // (1/4pi) sum x_i |T_i| at the exact solution and differs from it by
    // (1/4pi) ||x* - x||_A^2 >= 0 for every x
    double pc = 0.0, pxx = 0.0, pxr = 0.0;
    for (int i = r0 + t; i < r1; i += kSolveWG) {
      const double xi = x64[i];
      sigma[i] = xi;
      pc = __builtin_fma(xi, b[i], pc);
      pxx = __builtin_fma(xi, xi, pxx);
      pxr = __builtin_fma(xi, r64[i], pxr);
    }
    double cap, cap_bound;
    {
      const double v[3] = {pc, pxx, pxr};
      double tot[3];
      if (!sys_sync<3>(bar, v, tot, l_red, l_flag)) { aborted = true; break; }
      const double J = tot[0] + tot[2];
      cap = J * kInv4Pi;
      if (P.cap_rtol > 0.0 && est >= 0.0)
        cap_bound = J != 0.0 ? est / fabs(J) : 0.0;  // the capacity stop's estimate
      else
        cap_bound = tot[0] != 0.0 ? sqrt(tot[1]) * rnorm / fabs(tot[0]) : 0.0;  // first-order bound
    }
    if (rank == 0 && t == 0) {
      result->cap = cap;
      result->cap_bound = cap_bound;
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
      result->cap_bound = 0.0;
      ctl->phase = PH_DONE;
    } else {
      ctl->phase = phase; ctl->iters = iters; ctl->outer = outer; ctl->inner = inner; ctl->epoch = bar.epoch;
      ctl->bnorm = bnorm; ctl->rnorm = rnorm; ctl->scale = scale; ctl->gamma = gamma; ctl->eta = eta;
      ctl->alpha = alpha; ctl->beta = beta; ctl->itol = itol;
      ctl->hs_n = hs_n;
      for (int q = 0; q < 4; ++q) ctl->hs[q] = hs[q];
      ctl->hs_sum = hs_sum; ctl->jres = jres; ctl->est = est;
      result->iters = iters;
      result->outer = outer;
      result->status = BC_RUNNING;
      result->precision = MIXED ? BC_MIXED : BC_FP64;
      result->cap_bound = 0.0;
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
  const SolveLayout Lay(S.N, BC_FP64);  // the control block, slots and records do not depend on precision
  const int t = threadIdx.x;
  BarSlot *slots = reinterpret_cast<BarSlot *>(S.ws + Lay.slots);
  BarRel *rel = reinterpret_cast<BarRel *>(S.ws + Lay.rel);
  if (t < kGMax) slots[t].tag = 0u;
  if (t < kNRep) {
    rel[t].gen = 0u;
    rel[t].abort = 0;
  }
  if (t == 0) {
    SolveCtl *ctl = reinterpret_cast<SolveCtl *>(S.ws + Lay.ctl);
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

int solve_workgroups(int64_t N) { return solve_wg_count(N); }

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

// ------------------------------------------------- standalone product
// Y = V X for NR vectors (X: NR columns of N entries, column-major) with the
// symmetric product of k_solve, as three launches (the launch boundaries
// take the place of the system barrier): padding, partial sums, gather.
// Same partition and order as inside the solver, so the result depends on N
// only; the NR vectors share each pass over V.  MT is the matrix type, XT
// the vectors' and the accumulation's: (double, double), (float, float) or
// (float, double).
template <typename MT, typename XT>
constexpr int32_t matvec_kind() {
  return sizeof(MT) == 8 ? BC_FP64 : (sizeof(XT) == 8 ? kMatvecF32X64 : BC_MIXED);
}

// skip (may be NULL): when *skip != 0 the launch does nothing (a product
// queued behind a solver's stop decision on the device).
template <typename MT, typename XT, int NR>
__global__ __launch_bounds__(kSolveWG) void k_matvec_pad(const XT *__restrict__ x, int64_t N, char *ws,
                                                         const int32_t *__restrict__ skip) {
  if (skip && *skip) return;
  const MatvecLayout Lay(N, matvec_kind<MT, XT>(), NR);
  XT *xp = reinterpret_cast<XT *>(ws + Lay.xpad);
  for (int64_t i = (int64_t)blockIdx.x * kSolveWG + threadIdx.x; i < NR * Lay.ld; i += (int64_t)gridDim.x * kSolveWG) {
    const int64_t m = i / Lay.ld, j = i - m * Lay.ld;
    xp[i] = j < N ? x[m * N + j] : XT(0);
  }
}

__device__ __forceinline__ HalfPlan matvec_plan(const MatvecLayout &Lay, int64_t N, int G, int rank) {
  HalfPlan H;
  H.ld = Lay.ld; H.m64 = Lay.ld / 64; H.T = Lay.T; H.N = (int)N; H.nB = (int)Lay.nB; H.k = Lay.k; H.G = G;
  H.u0 = Lay.T * rank / G; H.u1 = Lay.T * (rank + 1) / G;
  return H;
}

// One vector: the strip product (LDS: the x values of each wavefront's row
// block).  Several: the unit sweep with 8-byte matrix loads (one FP64 or FP32
// column per lane), so that the NR x 8 row sums stay in registers; LDS: two
// buffers of NR x 16 wavefronts x CW column sums and the 16 x 8 x NR row x
// values.
template <typename MT, typename XT, int NR>
__global__ __launch_bounds__(kSolveWG) __attribute__((amdgpu_waves_per_eu(4))) void k_matvec_part(
    const MT *__restrict__ V, int64_t N, char *ws, const int32_t *__restrict__ skip) {
  if (skip && *skip) return;
  static_assert(NR == 1 || sizeof(XT) == 8, "several vectors: FP64 vectors only");
  const MatvecLayout Lay(N, matvec_kind<MT, XT>(), NR);
  gptr<char> w = as_global(ws);
  double unused = 0.0;
  if constexpr (NR == 1) {
    __shared__ XT s_x[16 * kRB];
    const StripPlan H = strip_plan(N, Lay.ld, Lay.sw, (int)gridDim.x, (int)blockIdx.x);
    strip_product<MT, XT, XT, false>(as_global(V), reinterpret_cast<gptr<const XT>>(w + Lay.xpad), H,
                                     reinterpret_cast<gptr<XT>>(w + Lay.rpart),
                                     reinterpret_cast<gptr<XT>>(w + Lay.cpart), (lptr<XT>)s_x, unused);
  } else {
    using L = typename std::conditional<sizeof(MT) == sizeof(XT), LoadD1, LoadF1D>::type;
    constexpr int CW = 64 * L::VEC;
    __shared__ XT s_buf[2 * NR * 16 * CW + 16 * 8 * NR];
    const HalfPlan H = matvec_plan(Lay, N, (int)gridDim.x, (int)blockIdx.x);
    half_product<MT, XT, XT, false, true, NR, L>(as_global(V), reinterpret_cast<gptr<const XT>>(w + Lay.xpad), H,
                                                 reinterpret_cast<gptr<XT>>(w + Lay.rpart),
                                                 reinterpret_cast<gptr<XT>>(w + Lay.cpart), (lptr<XT>)s_buf, unused);
  }
}

template <typename MT, typename XT, int NR>
__global__ __launch_bounds__(kSolveWG) void k_matvec_gather(int64_t N, const char *ws, XT *__restrict__ y,
                                                            const int32_t *__restrict__ skip) {
  if (skip && *skip) return;
  __shared__ double s_part[16 * 64];
  __shared__ double s_band[kMaxBand];
  const MatvecLayout Lay(N, matvec_kind<MT, XT>(), NR);
  const int G = (int)gridDim.x, rank = (int)blockIdx.x;
  const int r0 = (int)(N * rank / G), r1 = (int)(N * (rank + 1) / G);
  gptr<const char> w = as_global(ws);
  XT *band = reinterpret_cast<XT *>(s_band);
  if constexpr (NR == 1) {
    const StripPlan H = strip_plan(N, Lay.ld, Lay.sw, G, rank);
    strip_gather<XT>(H, r0, r1, reinterpret_cast<gptr<const XT>>(w + Lay.rpart),
                     reinterpret_cast<gptr<const XT>>(w + Lay.cpart), (lptr<XT>)s_part, (lptr<XT>)s_band);
    for (int i = r0 + (int)threadIdx.x; i < r1; i += kSolveWG) y[i] = band[i - r0];
  } else {
    const HalfPlan H = matvec_plan(Lay, N, G, rank);
    for (int m = 0; m < NR; ++m) {
      half_gather<XT>(H, r0, r1, reinterpret_cast<gptr<const XT>>(w + Lay.rpart) + (size_t)m * kRB * Lay.T,
                      reinterpret_cast<gptr<const XT>>(w + Lay.cpart) + (size_t)m * Lay.nB * Lay.ld,
                      (lptr<XT>)s_part, (lptr<XT>)s_band);
      for (int i = r0 + (int)threadIdx.x; i < r1; i += kSolveWG) y[m * N + i] = band[i - r0];
      __syncthreads();  // band is rewritten by the next vector's gather
    }
  }
}

template <typename MT, typename XT, int NR>
static void matvec_launch(const void *V, int64_t N, const void *x, void *y, char *w, const int32_t *skip,
                          hipStream_t s) {
  const int G = solve_workgroups(N);
  hipLaunchKernelGGL((k_matvec_pad<MT, XT, NR>), dim3(16), dim3(kSolveWG), 0, s, static_cast<const XT *>(x), N, w,
                     skip);
  hipLaunchKernelGGL((k_matvec_part<MT, XT, NR>), dim3(G), dim3(kSolveWG), 0, s, static_cast<const MT *>(V), N, w,
                     skip);
  hipLaunchKernelGGL((k_matvec_gather<MT, XT, NR>), dim3(G), dim3(kSolveWG), 0, s, N, (const char *)w,
                     static_cast<XT *>(y), skip);
}

int launch_matvec(int32_t kind, const void *V, int64_t N, int nr, const void *x, void *y, void *ws, hipStream_t s,
                  const int32_t *skip) {
  char *w = static_cast<char *>(ws);
  if (kind == BC_FP64 && nr == 1) matvec_launch<double, double, 1>(V, N, x, y, w, skip, s);
  else if (kind == BC_FP64 && nr == 3) matvec_launch<double, double, 3>(V, N, x, y, w, skip, s);
  else if (kind == BC_MIXED && nr == 1) matvec_launch<float, float, 1>(V, N, x, y, w, skip, s);
  else if (kind == kMatvecF32X64 && nr == 1) matvec_launch<float, double, 1>(V, N, x, y, w, skip, s);
  else if (kind == kMatvecF32X64 && nr == 3) matvec_launch<float, double, 3>(V, N, x, y, w, skip, s);
  else return BC_EINVAL;
  return hipGetLastError() == hipSuccess ? BC_OK : BC_EDEVICE;
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
